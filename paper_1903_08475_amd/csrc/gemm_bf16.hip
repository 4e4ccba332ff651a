// Split-BF16 MFMA contractions of the solve (Sec. 4.3 steps 2 and 5).
//
// Each operand x, taken in FP32, is written as x = h + m + l, with h, m, l
// the round-to-nearest bf16 of the successive residuals (exact: 24
// significant bits).  A product a*b is formed from the six partial products
// whose combined weight is at least 2^-18 of the leading one:
//   ah*bh + ah*bm + am*bh + ah*bl + am*bm + al*bh
// on v_mfma_f32_32x32x16_bf16 (bf16 products are exact in FP32).  GEMM1's
// FP32 accumulators are flushed into FP64 registers every kFlushSlabs K
// slabs, so no FP32 sum runs over more than kFlushSlabs*32 terms (GEMM2's K
// is the moment count, short enough for FP32 sums).
//
// GEMM1 (moments, Eq. B_CS) reads A = rho_Yin +- rho_Yang (U_Yang =
// (-1)^m U_Yin, Sec. 4.2) pre-split into three bf16 planes per parity by
// k_fold_split, and U pre-split by the plan.
// GEMM2 (expansion, Eq. gravpotmult) reads M pre-split by the radial scan
// and Q pre-split by the plan, sums even- and odd-m columns separately and
// writes Phi_Yin = E + O, Phi_Yang = E - O.  Its K loop runs from the
// highest degree down to l = 0, so the dominant low-degree terms are added
// to the smallest partial sums last.
//
// Tiles: 128x128 per block of 512 threads (2x4 waves of 64x32, each 2x1
// MFMA blocks of 32x32: two waves per SIMD, so one wave's barrier, copy
// issue and LDS reads overlap the other's MFMAs), K slabs of 32.  A slab (both operands, three pieces:
// 48 KB) is copied from global memory straight into LDS by
// global_load_lds_dwordx4 (no staging registers) into a ring of three
// slab buffers (144 KB): slab s+2 is in flight while slab s is multiplied,
// with one barrier per slab.  Inside a buffer each piece is a [128][32]
// bf16 array of 16-byte chunks stored at chunk position
//   4*row + (kchunk ^ ((row >> 2) & 3)).
// The LDS serves a 16-byte-per-lane read 16 lanes per clock over 64 banks
// (measured: a group is conflict-free when its 16 chunk positions differ
// modulo 16); the lanes of a fragment read cover 16 consecutive rows at one
// kchunk, whose positions modulo 16 are then all distinct.
#include "mpg_internal.h"

namespace mpg {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
// native vector types (HIP's uint4/float4 classes defeat register promotion)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

constexpr int TB = kSplitTile, TK = 32;
constexpr int kPiece = TB * TK;       // bf16 elements of one piece of one operand in a slab
constexpr int kFlushSlabs = 15;       // GEMM1: FP32 runs of at most 480 terms (a multiple of the ring size)
#ifndef MPG_WAVES
#define MPG_WAVES 8
#endif
// 2 x (kWaves/2) waves per block; a wave owns a 64 x kWN output tile
constexpr int kWaves = MPG_WAVES, kThreads = 64 * kWaves;
constexpr int kWN = TB / (kWaves / 2), kNB = kWN / 32;  // wave tile width, its 32-wide MFMA blocks
constexpr int kParts = 8 / kWaves;                      // 64-chunk parts of each piece a wave copies
constexpr int kLoadsPerSlab = 6 * kParts;               // global_load_lds instructions per wave per slab

// one K slab of both operands, three pieces each, swizzled (see above)
struct Slab {
    bf16 a[3][kPiece];
    bf16 b[3][kPiece];
};

// s_waitcnt immediates (gfx9 encoding): vmcnt <= n with the other counters
// unconstrained, and lgkmcnt == 0 with the others unconstrained
#define MPG_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x0F70 | ((n) & 15) | (((n) >> 4) << 14))
#define MPG_WAIT_LGKM0() __builtin_amdgcn_s_waitcnt(0xC07F)

// C/D layout of v_mfma_f32_32x32x16_bf16 (measured): register r of lane l
// holds D[8(r/4) + 4(l/32) + r%4][l%32]; A rows are lane%32 with K elements
// 8(l/32)..+7, B columns lane%32 with the same K elements.
__device__ inline int d_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

// three bf16 pieces of an FP32 value (exact: 24 significant bits)
__device__ inline void split3f(float v, bf16 &h, bf16 &m, bf16 &l) {
    h = (bf16)v;
    float r = v - (float)h;
    m = (bf16)r;
    l = (bf16)(r - (float)m);
}

__device__ __forceinline__ uint32_t pack2(bf16 a, bf16 b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

__device__ inline void zero(v16f (&acc)[2][kNB]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kNB; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
}

// ---------------------------------------------------------------------------
// Input split: A = rho_Yin + rho_Yang (even-m block) and rho_Yin - rho_Yang
// (odd-m block) under the fold (U_Yang = (-1)^m U_Yin, Sec. 4.2), else A =
// rho, rounded once to FP32 and written as three bf16 pieces in tile-slab
// blocks (one plane per parity; zero past n_ang and past the last row).
// Thread = one 16-byte chunk (8 consecutive K of one row) of one block, so
// consecutive threads write consecutive chunks.
template <typename T, bool FOLD>
__device__ __forceinline__ void fold_split_chunk(const SplitArgs &g, size_t t) {
    const size_t blk = t / 512;
    const int c = (int)(t - blk * 512);
    const int tile = (int)(blk / g.ks1), slab = (int)(blk - (size_t)tile * g.ks1);
    const int r = c >> 2, kc = (c & 3) ^ ((r >> 2) & 3);
    const int row = tile * TB + r;
    int k0 = slab * TK + kc * 8;
    const int n_r = g.n_r, n_ang = g.n_ang;
    const bool row_ok = row < g.rows;
    const int f = row_ok ? row / n_r : 0, i = row_ok ? row - f * n_r : 0;
    const size_t pstride = (size_t)n_r * n_ang, fld = (size_t)g.n_patches * pstride;
    // without the fold K runs over every patch's cells (k = patch*n_angp + cell)
    const int gp = FOLD ? 0 : k0 / g.n_angp;
    k0 -= gp * g.n_angp;
    const T *r0 = (const T *)g.rho + f * fld + gp * pstride + (size_t)i * n_ang;
    const T *r1 = r0 + pstride;
    double d0[8], d1[8];
    if (sizeof(T) == 4 && (n_ang & 7) == 0) {
        // whole chunk inside or outside the row; 32-byte aligned
        f32x4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0, b0 = a0, b1 = a0;
        if (row_ok && k0 < n_ang) {
            a0 = *(const f32x4 *)(r0 + k0);
            a1 = *(const f32x4 *)(r0 + k0 + 4);
            if (FOLD) {
                b0 = *(const f32x4 *)(r1 + k0);
                b1 = *(const f32x4 *)(r1 + k0 + 4);
            }
        }
        d0[0] = a0.x; d0[1] = a0.y; d0[2] = a0.z; d0[3] = a0.w;
        d0[4] = a1.x; d0[5] = a1.y; d0[6] = a1.z; d0[7] = a1.w;
        d1[0] = b0.x; d1[1] = b0.y; d1[2] = b0.z; d1[3] = b0.w;
        d1[4] = b1.x; d1[5] = b1.y; d1[6] = b1.z; d1[7] = b1.w;
    } else {
        // FP64 input (or rows not a multiple of 8): element by element
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool in = row_ok && k0 + q < n_ang;
            d0[q] = in ? (double)r0[k0 + q] : 0.0;
            d1[q] = in && FOLD ? (double)r1[k0 + q] : 0.0;
        }
    }
    const size_t plane = (size_t)g.row_tiles * g.ks1 * 3 * kBlk;
#pragma unroll
    for (int par = 0; par < (FOLD ? 2 : 1); ++par) {
        uint32_t h[4], m[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float x0 = (float)(par ? d0[2 * q] - d1[2 * q] : d0[2 * q] + d1[2 * q]);
            float x1 = (float)(par ? d0[2 * q + 1] - d1[2 * q + 1] : d0[2 * q + 1] + d1[2 * q + 1]);
            bf16 h0, m0, l0, h1, m1, l1;
            split3f(x0, h0, m0, l0);
            split3f(x1, h1, m1, l1);
            h[q] = pack2(h0, h1);
            m[q] = pack2(m0, m1);
            l[q] = pack2(l0, l1);
        }
        bf16 *o = g.A + par * plane + blk * 3 * kBlk + (size_t)c * 8;
        *(u32x4 *)(o) = (u32x4){h[0], h[1], h[2], h[3]};
        *(u32x4 *)(o + kBlk) = (u32x4){m[0], m[1], m[2], m[3]};
        *(u32x4 *)(o + 2 * kBlk) = (u32x4){l[0], l[1], l[2], l[3]};
    }
}

template <typename T, bool FOLD>
__global__ __launch_bounds__(256) void k_fold_split(SplitArgs g, size_t n_threads) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_threads) fold_split_chunk<T, FOLD>(g, t);
}

// batch version: the field's arguments come from device memory
template <typename T>
__global__ __launch_bounds__(256) void k_batch_fold_split(const SplitArgs *args, int f, size_t n_threads) {
    const SplitArgs g = args[f];
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_threads) return;
    if (g.fold) fold_split_chunk<T, true>(g, t);
    else fold_split_chunk<T, false>(g, t);
}

// ---------------------------------------------------------------------------
// Slab loader.  A slab of an operand tile is one tile-slab block, already
// in LDS order: wave w copies chunks 64P .. 64P+63 (P = kParts*w + h) of
// every piece of both operands, lane l copying chunk 64P + l, so that each
// copy instruction moves 1 KB of consecutive global memory into
// consecutive LDS.
struct Loader {
    const bf16 *a, *b;  // first block (slab 0) of the A and B tiles
    int lo[kParts];     // element offsets of this lane's chunks in a piece
    int part[kParts];   // element offsets of the wave's parts in a piece (wave-uniform)
};

__device__ __forceinline__ void init_loader(Loader &L, int wave, int lane, const bf16 *a, const bf16 *b) {
    L.a = a;
    L.b = b;
#pragma unroll
    for (int h = 0; h < kParts; ++h) {
        L.part[h] = (kParts * wave + h) * 512;
        L.lo[h] = L.part[h] + lane * 8;
    }
}

__device__ __forceinline__ void load_slab(Slab &S, const Loader &L, int slab) {
    const bf16 *a = L.a + (size_t)slab * 3 * kBlk, *b = L.b + (size_t)slab * 3 * kBlk;
#pragma unroll
    for (int h = 0; h < kParts; ++h)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            __builtin_amdgcn_global_load_lds((glb_void *)(a + q * kBlk + L.lo[h]), (lds_void *)(S.a[q] + L.part[h]),
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds((glb_void *)(b + q * kBlk + L.lo[h]), (lds_void *)(S.b[q] + L.part[h]),
                                             16, 0, 0);
        }
}

// 8 bf16 (16 bytes) of row `row`, kchunk kc of one swizzled piece
__device__ __forceinline__ v8bf frag(const bf16 *piece, int row, int kc) {
    return *(const v8bf *)(piece + (row * 4 + (kc ^ ((row >> 2) & 3))) * 8);
}

// one 32-deep slab for a wave's 64 x kWN tile: for each 16-deep step the
// six partial products are issued product by product over the wave's
// accumulators, smallest weight first.
__device__ __forceinline__ void mma_slab(const Slab &S, int wm, int wn, int lane, v16f (&acc)[2][kNB]) {
    const int r = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int kc = 2 * ks + kh;
        v8bf ah[2], am[2], al[2], bh[kNB], bm[kNB], bl[kNB];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = frag(S.a[0], wm + 32 * i + r, kc);
            am[i] = frag(S.a[1], wm + 32 * i + r, kc);
            al[i] = frag(S.a[2], wm + 32 * i + r, kc);
        }
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            bh[j] = frag(S.b[0], wn + 32 * j + r, kc);
            bm[j] = frag(S.b[1], wn + 32 * j + r, kc);
            bl[j] = frag(S.b[2], wn + 32 * j + r, kc);
        }
#define MMP(X, Y)                                                                           \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) _Pragma("unroll") for (int j = 0; j < kNB; ++j) \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X[i], Y[j], acc[i][j], 0, 0, 0);
        MMP(al, bh)
        MMP(am, bm)
        MMP(ah, bl)
        MMP(am, bh)
        MMP(ah, bm)
        MMP(ah, bh)
#undef MMP
    }
}

// Workgroup barrier for the slab ring.  It waits for this wave's copies up
// to the slab about to be read (at most `pending` copy instructions of the
// next slab stay in flight), then joins the other waves.  The empty asm
// statements keep the compiler from moving LDS accesses across it;
// __syncthreads() is not used because its fence would also wait for the
// copies still in flight.
template <int pending>
__device__ __forceinline__ void ring_barrier() {
    asm volatile("" ::: "memory");
    MPG_WAIT_VM(pending);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Multiplies nsl consecutive K slabs of the tile into acc through the ring
// S0 -> S1 -> S2.  Slab t is block k0 + t*dk of the tiles (dk = +-1).  With
// FLUSH, acc is added into acc64 and cleared after every kFlushSlabs slabs.
// Every step copies a slab two ahead; past the end it copies the last slab
// again (same addresses, cache hits), so each step waits for the same count
// of copies.
// Every wave must call it with the same arguments; on return all copies
// have landed, and the ring may be refilled after a barrier.
template <bool FLUSH>
__device__ __forceinline__ void run_ring(Slab &S0, Slab &S1, Slab &S2, const Loader &L, int k0, int dk, int nsl,
                                         int wm, int wn, int lane, v16f (&acc)[2][kNB], double (&acc64)[2][kNB][16]) {
    if (nsl <= 0) return;
    const int last = nsl - 1;
    load_slab(S0, L, k0);
    load_slab(S1, L, k0 + min(1, last) * dk);
#define RING_STEP(CUR, NXT, O)                                  \
    ring_barrier<kLoadsPerSlab>();                              \
    load_slab(NXT, L, k0 + min(t + O + 2, last) * dk);          \
    if (t + O < nsl) mma_slab(CUR, wm, wn, lane, acc);
    // A group of kFlushSlabs slabs is unrolled in full, and the barriers and
    // copies of a turn of the ring run even where its last slabs lie past
    // the end: the compiler then follows which buffer every LDS read and
    // copy touches and adds no wait for copies still in flight.
    for (int s = 0; s < nsl; s += kFlushSlabs) {
#pragma unroll
        for (int j = 0; j < kFlushSlabs / 3; ++j) {
            const int t = s + 3 * j;
            if (t < nsl) {
                RING_STEP(S0, S2, 0)
                RING_STEP(S1, S0, 1)
                RING_STEP(S2, S1, 2)
            }
        }
        if (FLUSH) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < kNB; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)acc[a][b][r];
            zero(acc);
        }
    }
#undef RING_STEP
    // the two trailing copies land before anyone may reuse or free the LDS
    asm volatile("" ::: "memory");
    MPG_WAIT_VM(0);
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// One output tile of GEMM1 (column tile tn: even-m tiles first, then odd-m
// tiles; row tile tm; K split tz).  Writes Bpart[tz][row][col] in FP64.
template <bool FOLD>
__device__ __forceinline__ void gemm1_tile(const SplitArgs &g, int tn, int tm, int tz, Slab &S0, Slab &S1,
                                           Slab &S2) {
    const int rows = g.rows, np = g.np, ne_p = g.ne_p;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * kWN;
    const bool odd = FOLD && tn >= g.tiles_e;
    const int c0 = odd ? ne_p + (tn - g.tiles_e) * TB : tn * TB;
    const int cend = odd ? np : (FOLD ? ne_p : np);
    const int m0 = tm * TB;
    const int kbeg = tz * g.kchunk;
    const int kend = min(g.kang, kbeg + g.kchunk);
    const int nsl = kend > kbeg ? (kend - kbeg) / TK : 0;

    // A: the pre-split rho (+-) of this tile's column parity; B: split U
    Loader L;
    const size_t tstride = (size_t)g.ks1 * 3 * kBlk;
    const bf16 *A0 = g.A + (odd ? (size_t)g.row_tiles * tstride : 0) + (size_t)tm * tstride;
    init_loader(L, wave, lane, A0, g.U + (size_t)tn * tstride);

    v16f acc[2][kNB];
    double acc64[2][kNB][16];
    zero(acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < kNB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;
    run_ring<true>(S0, S1, S2, L, kbeg / TK, 1, nsl, wm, wn, lane, acc, acc64);

    double *out = g.Bpart + (size_t)tz * rows * np;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < kNB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int rr = m0 + wm + 32 * a + d_row(lane, r);
                int cc = c0 + wn + 32 * b + (lane & 31);
                if (rr < rows && cc < cend) out[(size_t)rr * np + cc] = acc64[a][b][r];
            }
}

// One output tile of GEMM2 (row tile tm, angular tile tn): the even-m K
// block into acc_e, then the odd-m block into acc_o, each walked from its
// top slab down.
template <typename T, bool FOLD>
__device__ __forceinline__ void gemm2_tile(const SplitArgs &g, int tm, int tn, Slab &S0, Slab &S1, Slab &S2) {
    T *phi = (T *)g.phi;
    const int rows = g.rows, np = g.np, ne_p = g.ne_p, n_ang = g.n_ang, n_r = g.n_r;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * kWN;
    const int m0 = tm * TB, n0 = tn * TB;

    Loader L;
    const size_t tstride = (size_t)g.ks2 * 3 * kBlk;
    init_loader(L, wave, lane, g.M + (size_t)tm * tstride, g.Q + (size_t)tn * tstride);

    v16f acc_e[2][kNB], acc_o[2][kNB];
    double acc64[2][kNB][16];
    zero(acc_e);
    zero(acc_o);
    const bool pp = !FOLD && g.nq > 1;
    if (FOLD) {
        const int ne = ne_p / TK, no = (np - ne_p) / TK;
        run_ring<false>(S0, S1, S2, L, ne - 1, -1, ne, wm, wn, lane, acc_e, acc64);
        // the odd block refills buffers the even block's last slabs were read from
        __syncthreads();
        run_ring<false>(S0, S1, S2, L, ne + no - 1, -1, no, wm, wn, lane, acc_o, acc64);
    } else if (!pp) {
        const int ns = g.ks2;
        run_ring<false>(S0, S1, S2, L, ns - 1, -1, ns, wm, wn, lane, acc_e, acc64);
    } else {
        // per-patch method: the moment sets of the patches one after the
        // other, each from its highest degree down, each flushed into FP64
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < kNB; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;
        const int nsb = np / TK;
        for (int gq = 0; gq < g.nq; ++gq) {
            if (gq) __syncthreads();
            run_ring<true>(S0, S1, S2, L, (gq + 1) * nsb - 1, -1, nsb, wm, wn, lane, acc_e, acc64);
        }
    }

    const size_t pstride = (size_t)n_r * n_ang, fld = (size_t)g.n_patches * pstride;
    const int n_angp = g.n_angp;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < kNB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int rr = m0 + wm + 32 * a + d_row(lane, r);
                int kk = n0 + wn + 32 * b + (lane & 31);
                const int gp = kk / n_angp, jk = kk - gp * n_angp;
                if (rr >= rows || jk >= n_ang) continue;
                int f = rr / n_r, i = rr - f * n_r;
                T *o = phi + f * fld + gp * pstride + (size_t)i * n_ang + jk;
                double e = (double)acc_e[a][b][r];
                if (!FOLD && pp) e = acc64[a][b][r];
                if (FOLD) {
                    double od = (double)acc_o[a][b][r];
                    o[0] = (T)(e + od);
                    o[pstride] = (T)(e - od);
                } else {
                    o[0] = (T)e;
                }
            }
}

// ---------------------------------------------------------------------------
// Grid launches for one plan: GEMM1 grid x = column tile, y = row tile,
// z = K split; GEMM2 grid x = row tile, y = angular tile.
template <bool FOLD>
__global__ __launch_bounds__(kThreads) void k_gemm1(SplitArgs g) {
    __shared__ Slab s0, s1, s2;
    gemm1_tile<FOLD>(g, blockIdx.x, blockIdx.y, blockIdx.z, s0, s1, s2);
}

template <typename T, bool FOLD>
__global__ __launch_bounds__(kThreads) void k_gemm2(SplitArgs g) {
    __shared__ Slab s0, s1, s2;
    gemm2_tile<T, FOLD>(g, blockIdx.x, blockIdx.y, s0, s1, s2);
}

// Persistent batch kernels: every block takes work items from a queue
// (items[], ordered longest first) through an atomic head until the queue
// is empty.  Item = (field, tile coordinates); args[] holds each field's
// arguments.  No item waits on another, so every block exits.  The barrier
// in next_item also keeps the next tile's first copies from overwriting
// slabs other waves are still reading.
__device__ __forceinline__ int next_item(int *head, int *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(head, 1);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

__global__ __launch_bounds__(kThreads) void k_batch_gemm1(const SplitArgs *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head) {
    __shared__ Slab s0, s1, s2;
    __shared__ int slot;
    for (;;) {
        const int it = next_item(head, &slot);
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const SplitArgs g = args[w.f];
        if (g.fold) gemm1_tile<true>(g, w.a, w.b, w.c, s0, s1, s2);
        else gemm1_tile<false>(g, w.a, w.b, w.c, s0, s1, s2);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_gemm2(const SplitArgs *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head) {
    __shared__ Slab s0, s1, s2;
    __shared__ int slot;
    for (;;) {
        const int it = next_item(head, &slot);
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const SplitArgs g = args[w.f];
        if (g.fold) gemm2_tile<T, true>(g, w.a, w.b, s0, s1, s2);
        else gemm2_tile<T, false>(g, w.a, w.b, s0, s1, s2);
    }
}

}  // namespace

SplitArgs split_args(const Plan &p, int n_fields, const void *rho, void *phi, int io_dtype, bool expansion) {
    SplitArgs g;
    g.rho = rho;
    g.phi = phi;
    g.io_f64 = io_dtype == MPG_F64;
    g.rows = n_fields * p.n_r;
    g.n_r = p.n_r;
    g.n_ang = p.n_ang;
    g.n_angp = p.n_angp;
    g.np = p.np;
    g.ne_p = p.ne_p;
    g.fold = p.fold;
    // per-patch method: GEMM1 sees single-patch fields; GEMM2 writes every
    // patch and reads every patch's moment set
    const bool pp2 = p.per_patch && expansion;
    g.n_patches = p.per_patch && !expansion ? 1 : p.n_patches;
    g.kang = pp2 ? p.n2() : p.kang();
    g.nq = pp2 ? p.nq() : 1;
    g.kq = pp2 ? p.kq() : p.np;
    g.tiles_e = p.tiles_e();
    g.tiles_o = p.tiles_o();
    g.kchunk = ((p.kang() / p.splitk + TK - 1) / TK) * TK;
    g.splitk = p.splitk;
    g.U = p.Us;
    g.Q = p.Qs;
    g.M = p.Ms;
    g.Bpart = p.Bpart;
    g.A = p.A_split;
    g.row_tiles = p.row_tiles();
    g.ks1 = p.kang() / TK;
    g.ks2 = p.kq() / TK;
    return g;
}

// one thread per 16-byte chunk of the row tiles holding the fields' rows
size_t split_input_threads(const Plan &p, int n_fields) {
    return (size_t)((n_fields * p.n_r + TB - 1) / TB) * (p.kang() / TK) * 512;
}

hipError_t split_input_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    SplitArgs g = split_args(p, n_fields, rho, nullptr, rho_dtype);
    const size_t threads = split_input_threads(p, n_fields);
    dim3 grid((unsigned)((threads + 255) / 256));
    if (rho_dtype == MPG_F64) {
        if (p.fold) hipLaunchKernelGGL((k_fold_split<double, true>), grid, dim3(256), 0, p.stream, g, threads);
        else hipLaunchKernelGGL((k_fold_split<double, false>), grid, dim3(256), 0, p.stream, g, threads);
    } else {
        if (p.fold) hipLaunchKernelGGL((k_fold_split<float, true>), grid, dim3(256), 0, p.stream, g, threads);
        else hipLaunchKernelGGL((k_fold_split<float, false>), grid, dim3(256), 0, p.stream, g, threads);
    }
    return hipGetLastError();
}

hipError_t gemm1_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    SplitArgs g = split_args(p, n_fields, rho, nullptr, rho_dtype);
    dim3 grid(g.tiles_e + g.tiles_o, (g.rows + TB - 1) / TB, p.splitk);
    if (p.fold) hipLaunchKernelGGL((k_gemm1<true>), grid, dim3(kThreads), 0, p.stream, g);
    else hipLaunchKernelGGL((k_gemm1<false>), grid, dim3(kThreads), 0, p.stream, g);
    return hipGetLastError();
}

hipError_t gemm2_bf16(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    SplitArgs g = split_args(p, n_fields, nullptr, phi, phi_dtype, true);
    dim3 grid((g.rows + TB - 1) / TB, g.kang / TB);
    if (phi_dtype == MPG_F64) {
        if (p.fold) hipLaunchKernelGGL((k_gemm2<double, true>), grid, dim3(kThreads), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm2<double, false>), grid, dim3(kThreads), 0, p.stream, g);
    } else {
        if (p.fold) hipLaunchKernelGGL((k_gemm2<float, true>), grid, dim3(kThreads), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm2<float, false>), grid, dim3(kThreads), 0, p.stream, g);
    }
    return hipGetLastError();
}

hipError_t batch_split_input_bf16(const SplitArgs *args, int f, size_t n_threads, int io_dtype, hipStream_t s) {
    dim3 grid((unsigned)((n_threads + 255) / 256));
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_fold_split<double>), grid, dim3(256), 0, s, args, f, n_threads);
    else
        hipLaunchKernelGGL((k_batch_fold_split<float>), grid, dim3(256), 0, s, args, f, n_threads);
    return hipGetLastError();
}

hipError_t batch_gemm1_bf16(const SplitArgs *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                            int blocks, hipStream_t s) {
    (void)io_dtype;
    hipLaunchKernelGGL(k_batch_gemm1, dim3(blocks), dim3(kThreads), 0, s, args, items, n_items, head);
    return hipGetLastError();
}

hipError_t batch_gemm2_bf16(const SplitArgs *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                            int blocks, hipStream_t s) {
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_gemm2<double>), dim3(blocks), dim3(kThreads), 0, s, args, items, n_items, head);
    else
        hipLaunchKernelGGL((k_batch_gemm2<float>), dim3(blocks), dim3(kThreads), 0, s, args, items, n_items, head);
    return hipGetLastError();
}

}  // namespace mpg
