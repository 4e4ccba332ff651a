// Split-BF16 MFMA contractions of the solve (Sec. 4.3 steps 2 and 5).
//
// Each operand x, taken in FP32, is written as x = h + m + l, with h, m, l
// the round-to-nearest bf16 of the successive residuals (exact: 24
// significant bits).  A product a*b is formed from the six partial products
// whose combined weight is at least 2^-18 of the leading one:
//   ah*bh + ah*bm + am*bh + ah*bl + am*bm + al*bh
// on v_mfma_f32_32x32x16_bf16 (bf16 products are exact in FP32).  The
// tiered form keeps the six for the leading (low-degree) columns of each
// m-parity block (six_e, six_o) and forms the others from the three
// products of weight >= 2^-9, ah*bh + ah*bm + am*bh, i.e. with 16-bit
// operands h + m: whole GEMM1 wave tiles of 64 moment columns, and whole
// K slabs of GEMM2, take one form or the other.  GEMM1's
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
// Tiles: GEMM1 128x256 (rows x moment columns: two column tiles, so every
// rho+- slab serves 256 columns), GEMM2 128x256 by default (one row tile x
// two angular tiles: consecutive blocks share the Q tiles, and each M row
// tile is read once per 256 angular cells) or 256x128 (the autotuner's
// other choice); 512 threads = 8 waves of 64x64 (2x2 MFMA blocks of 32x32,
// two waves per SIMD); K slabs of 32.  A slab of a block (both operands,
// three pieces, 72 KB) is copied from global memory straight into LDS by
// global_load_lds_dwordx4 (no staging registers) into two slab buffers
// (144 KB of the 160 KB LDS): slab s+1 is in flight while slab s is
// multiplied, one barrier per slab.  Inside a buffer each piece is a
// [128][32] bf16 array of 16-byte chunks at chunk position
//   4*row + (kchunk ^ ((row >> 2) & 3)).
// The LDS serves a 16-byte-per-lane read 16 lanes per clock over 64 banks
// (measured: a group is conflict-free when its 16 chunk positions differ
// modulo 16); the lanes of a fragment read cover 16 consecutive rows at one
// kchunk, whose positions modulo 16 are then all distinct.
#include "mpg_internal.h"
#include "scan_core.h"

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
constexpr int kPiece = TB * TK;  // bf16 elements of one piece of one 128-row block in a slab
constexpr int kFlushSlabs = 16;  // GEMM1: FP32 runs of at most 512 terms (a multiple of the ring size)
constexpr int kThreads = 512;    // 8 waves of 64x64

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

__device__ inline void zero(v16f (&acc)[2][2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
}

// ---------------------------------------------------------------------------
// Input split: A = rho_Yin + rho_Yang (even-m block) and rho_Yin - rho_Yang
// (odd-m block) under the fold (U_Yang = (-1)^m U_Yin, Sec. 4.2), else A =
// rho, rounded once to FP32 and written as three bf16 pieces in tile-slab
// blocks (one plane per parity; zero past n_ang and past the last row).
// Thread = one 16-byte chunk (8 consecutive K of one row) of one block:
// the loads of a chunk (widened to FP64) and its destination, then the
// pieces and their stores, so a thread can hold several chunks' loads in
// flight before it stores any.
struct ChunkIn {
    double d0[8], d1[8];
    size_t dst;  // piece-0 element offset of the chunk in its parity plane
    bool live;   // the chunk lies in the plane (slabs past the last do not)
};

template <typename T, bool FOLD>
__device__ __forceinline__ void fold_split_load(const SplitArgs &g, size_t t, ChunkIn &in) {
    // a wave covers 4 rows x 4 slabs: 512 consecutive bytes of each row
    // read (FP32), 256 consecutive bytes of each piece of each slab written
    const size_t unit = t / 2048;  // (row tile, group of 4 slabs)
    const int rem = (int)(t - unit * 2048);
    const int ng = (g.ks1 + 3) / 4;
    const int tile = (int)(unit / ng), sg = (int)(unit - (size_t)tile * ng);
    const int lane = rem & 63, r = 4 * (rem >> 6) + (lane >> 4), qq = lane & 15;
    const int slab = 4 * sg + (qq >> 2), kc = qq & 3;
    in.live = slab < g.ks1;
    const size_t blk = (size_t)tile * g.ks1 + slab;
    const int c = 4 * r + (kc ^ ((r >> 2) & 3));  // stored chunk position
    in.dst = blk * 3 * kBlk + (size_t)c * 8;
    const int row = tile * TB + r;
    int k0 = slab * TK + kc * 8;
    const int n_r = g.n_r, n_ang = g.n_ang;
    const bool row_ok = in.live && row < g.rows;
    const int f = row_ok ? row / n_r : 0, i = row_ok ? row - f * n_r : 0;
    const size_t pstride = (size_t)n_r * n_ang, fld = (size_t)g.n_patches * pstride;
    // without the fold K runs over every patch's cells (k = patch*n_angp + cell)
    const int gp = FOLD ? 0 : k0 / g.n_angp;
    k0 -= gp * g.n_angp;
    const T *r0 = (const T *)g.rho + f * fld + gp * pstride + (size_t)i * n_ang;
    const T *r1 = r0 + pstride;
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
        in.d0[0] = a0.x; in.d0[1] = a0.y; in.d0[2] = a0.z; in.d0[3] = a0.w;
        in.d0[4] = a1.x; in.d0[5] = a1.y; in.d0[6] = a1.z; in.d0[7] = a1.w;
        in.d1[0] = b0.x; in.d1[1] = b0.y; in.d1[2] = b0.z; in.d1[3] = b0.w;
        in.d1[4] = b1.x; in.d1[5] = b1.y; in.d1[6] = b1.z; in.d1[7] = b1.w;
    } else {
        // FP64 input (or rows not a multiple of 8): element by element
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool on = row_ok && k0 + q < n_ang;
            in.d0[q] = on ? (double)r0[k0 + q] : 0.0;
            in.d1[q] = on && FOLD ? (double)r1[k0 + q] : 0.0;
        }
    }
}

template <bool FOLD, bool NT = false>
__device__ __forceinline__ void fold_split_store(const SplitArgs &g, const ChunkIn &in) {
    if (!in.live) return;
    const size_t plane = (size_t)g.row_tiles * g.ks1 * 3 * kBlk;
#pragma unroll
    for (int par = 0; par < (FOLD ? 2 : 1); ++par) {
        uint32_t h[4], m[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float x0 = (float)(par ? in.d0[2 * q] - in.d1[2 * q] : in.d0[2 * q] + in.d1[2 * q]);
            float x1 = (float)(par ? in.d0[2 * q + 1] - in.d1[2 * q + 1] : in.d0[2 * q + 1] + in.d1[2 * q + 1]);
            bf16 h0, m0, l0, h1, m1, l1;
            split3f(x0, h0, m0, l0);
            split3f(x1, h1, m1, l1);
            h[q] = pack2(h0, h1);
            m[q] = pack2(m0, m1);
            l[q] = pack2(l0, l1);
        }
        bf16 *o = g.A + par * plane + in.dst;
        store<NT>((u32x4 *)(o), (u32x4){h[0], h[1], h[2], h[3]});
        store<NT>((u32x4 *)(o + kBlk), (u32x4){m[0], m[1], m[2], m[3]});
        store<NT>((u32x4 *)(o + 2 * kBlk), (u32x4){l[0], l[1], l[2], l[3]});
    }
}

template <typename T, bool FOLD>
__device__ __forceinline__ void fold_split_chunk(const SplitArgs &g, size_t t) {
    ChunkIn in;
    fold_split_load<T, FOLD>(g, t, in);
    fold_split_store<FOLD>(g, in);
}

// the 2048 chunks of one split unit by a block of kThreads threads: every
// thread's loads first, then its stores
template <typename T, bool FOLD, bool NT = false>
__device__ __forceinline__ void fold_split_unit(const SplitArgs &g, size_t u, int tid) {
    constexpr int kPer = 2048 / kThreads;
    ChunkIn in[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) fold_split_load<T, FOLD>(g, u * 2048 + k * kThreads + tid, in[k]);
#pragma unroll
    for (int k = 0; k < kPer; ++k) fold_split_store<FOLD, NT>(g, in[k]);
}

template <typename T, bool FOLD>
__global__ __launch_bounds__(256) void k_fold_split(SplitArgs g, size_t n_threads) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_threads) fold_split_chunk<T, FOLD>(g, t);
}

// ---------------------------------------------------------------------------
// One K slab of a block: NA 128-row blocks of A and NB of B, three pieces
// each, in the layout of the tile-slab blocks (see above).
template <int NA, int NB>
struct SlabT {
    bf16 a[3][NA * kPiece];
    bf16 b[3][NB * kPiece];
};

// Slab loader.  Every 128-row block of a slab is one tile-slab block,
// already in LDS order: wave w copies chunks 64w .. 64w+63 of every piece,
// lane l copying chunk 64w + l, so each copy instruction moves 1 KB of
// consecutive global memory into consecutive LDS (9 per wave per slab).
template <int NA, int NB>
struct LoaderT {
    const bf16 *a[NA], *b[NB];  // slab-0 blocks of the A and B row tiles
    int lo, part;               // this lane's / this wave's element offsets in a piece
};

template <int NA, int NB>
__device__ __forceinline__ void load_slab(SlabT<NA, NB> &S, const LoaderT<NA, NB> &L, int slab, bool six) {
    const size_t o = (size_t)slab * 3 * kBlk;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        // the three-product form reads no l piece
        if (q == 2 && !six) break;
#pragma unroll
        for (int i = 0; i < NA; ++i)
            __builtin_amdgcn_global_load_lds((glb_void *)(L.a[i] + o + q * kBlk + L.lo),
                                             (lds_void *)(S.a[q] + i * kPiece + L.part), 16, 0, 0);
#pragma unroll
        for (int j = 0; j < NB; ++j)
            __builtin_amdgcn_global_load_lds((glb_void *)(L.b[j] + o + q * kBlk + L.lo),
                                             (lds_void *)(S.b[q] + j * kPiece + L.part), 16, 0, 0);
    }
}

// 8 bf16 (16 bytes) of row `row`, kchunk kc of one swizzled piece
__device__ __forceinline__ v8bf frag(const bf16 *piece, int row, int kc) {
    return *(const v8bf *)(piece + (row * 4 + (kc ^ ((row >> 2) & 3))) * 8);
}

// one 32-deep slab for a wave's 64x64 tile at (wm, wn) of the block: for
// each 16-deep step the partial products (six, or with SIX false the three
// h*h + h*m + m*h) are issued product by product over the four
// accumulators, smallest weight first, so consecutive MFMAs never depend on
// each other.
template <int NA, int NB, bool SIX>
__device__ __forceinline__ void mma_slab(const SlabT<NA, NB> &S, int wm, int wn, int lane, v16f (&acc)[2][2]) {
    const int r = lane & 31, kh = lane >> 5;
    const int ao = (wm >> 7) * kPiece, ar = wm & 127, bo = (wn >> 7) * kPiece, br = wn & 127;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int kc = 2 * ks + kh;
        v8bf ah[2], am[2], al[2], bh[2], bm[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = frag(S.a[0] + ao, ar + 32 * i + r, kc);
            am[i] = frag(S.a[1] + ao, ar + 32 * i + r, kc);
            bh[i] = frag(S.b[0] + bo, br + 32 * i + r, kc);
            bm[i] = frag(S.b[1] + bo, br + 32 * i + r, kc);
            if (SIX) {
                al[i] = frag(S.a[2] + ao, ar + 32 * i + r, kc);
                bl[i] = frag(S.b[2] + bo, br + 32 * i + r, kc);
            }
        }
#define MMP(X, Y)                                                                              \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) _Pragma("unroll") for (int j = 0; j < 2; ++j) \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X[i], Y[j], acc[i][j], 0, 0, 0);
        if (SIX) {
            MMP(al, bh)
            MMP(am, bm)
            MMP(ah, bl)
        }
        MMP(am, bh)
        MMP(ah, bm)
        MMP(ah, bh)
#undef MMP
    }
}

// Workgroup barrier for the slab ring: waits for this wave's copies of the
// slab about to be read, then joins the other waves.  The empty asm
// statements keep the compiler from moving LDS accesses across it;
// __syncthreads() is not used because its fence would also wait for copies
// still in flight.
template <int pending>
__device__ __forceinline__ void ring_barrier() {
    asm volatile("" ::: "memory");
    MPG_WAIT_VM(pending);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// Software-pipelined ring.  The fragments of one 16-deep step of a wave's
// 64x64 tile (h and m pieces of its two A row blocks and two B column
// blocks, plus the l pieces with six products) are read from LDS while the
// MFMAs of the previous step run, so LDS latency hides behind MFMA work.
// The workgroup barrier of a slab sits between its two steps: the second
// step's fragments are already in registers, and the first step of the
// next slab is read right after it, while the second step's MFMAs run.
template <bool SIX>
struct Frags {
    v8bf a[SIX ? 3 : 2][2], b[SIX ? 3 : 2][2];  // [piece][block]
};

template <int NA, int NB, bool SIX>
__device__ __forceinline__ void read_frags(Frags<SIX> &F, const SlabT<NA, NB> &S, int ks, int wm, int wn,
                                           int lane) {
    const int r = lane & 31, kc = 2 * ks + (lane >> 5);
    const int ao = (wm >> 7) * kPiece, ar = wm & 127, bo = (wn >> 7) * kPiece, br = wn & 127;
#pragma unroll
    for (int q = 0; q < (SIX ? 3 : 2); ++q)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            F.a[q][i] = frag(S.a[q] + ao, ar + 32 * i + r, kc);
            F.b[q][i] = frag(S.b[q] + bo, br + 32 * i + r, kc);
        }
}

// the partial products of one step, in the order of mma_slab (smallest
// weight first, product by product over the four accumulators)
template <bool SIX>
__device__ __forceinline__ void mma_frags(const Frags<SIX> &F, v16f (&acc)[2][2]) {
#define MMQ(X, Y)                                                                              \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) _Pragma("unroll") for (int j = 0; j < 2; ++j) \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.a[X][i], F.b[Y][j], acc[i][j], 0, 0, 0);
    if constexpr (SIX) {
        MMQ(2, 0)
        MMQ(1, 1)
        MMQ(0, 2)
    }
    MMQ(1, 0)
    MMQ(0, 1)
    MMQ(0, 0)
#undef MMQ
}

// Barrier of the pipelined ring: this wave's fragment reads and slab copies
// are complete, then every wave joins.  The scheduling barriers keep the
// compiler from moving MFMAs or LDS reads across it.
__device__ __forceinline__ void pipe_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// The first slab of the run that follows (block k0 of the tiles, six: with
// its l pieces), when a run issues its copy into S0 from its last steps so
// that the next run starts with it in flight (on: there is such a run).
struct NextRun {
    int k0;
    bool six, on;
};

// Multiplies nsl consecutive K slabs (slab t is block k0 + t*dk of the
// tiles), all with six products (SIX) or all with three, into acc through
// the two buffers S0, S1.  Step t: read the second step's fragments of slab
// t, multiply the first step's, barrier (slab t+1 has landed, and no wave
// reads slab t's buffer any more), copy slab t+2 into that buffer, read the
// first step's fragments of slab t+1, multiply the second step's.  With
// FLUSH, acc is added into acc64 and cleared after every kFlushSlabs slabs
// and at the end.  Every wave calls it with the same k0, dk, nsl; both
// buffers must be free on entry (no wave reading them, no copy in flight),
// and are free again on return.  Without MMA only the copies, reads and
// barriers (waves whose tile lies past the end of the block).
// With pre, slab 0's copy into S0 was issued by the run before.  With
// nx.on (nsl even, so that step nsl - 2 reads S0), step nsl - 2 copies the
// next run's first slab into S0 once every wave is past its barrier.
template <int NA, int NB, bool SIX, bool FLUSH, bool MMA = true>
__device__ __forceinline__ void run_pipe(SlabT<NA, NB> &S0, SlabT<NA, NB> &S1, const LoaderT<NA, NB> &L, int k0,
                                         int dk, int nsl, int wm, int wn, int lane, v16f (&acc)[2][2],
                                         double (&acc64)[2][2][16], bool pre = false,
                                         NextRun nx = NextRun{0, false, false}) {
    if (nsl <= 0) return;
    Frags<SIX> F0, F1;
    if (!pre) load_slab(S0, L, k0, SIX);
    pipe_barrier();
    if (nsl > 1) load_slab(S1, L, k0 + dk, SIX);
    read_frags<NA, NB, SIX>(F0, S0, 0, wm, wn, lane);
#define PIPE_STEP(CUR, NXT, O)                                               \
    {                                                                        \
        const int t = s + O;                                                 \
        read_frags<NA, NB, SIX>(F1, CUR, 1, wm, wn, lane);                   \
        if (MMA) mma_frags<SIX>(F0, acc);                                    \
        pipe_barrier();                                                      \
        if (t + 2 < nsl) load_slab(CUR, L, k0 + (t + 2) * dk, SIX);          \
        else if (nx.on && t + 2 == nsl) load_slab(CUR, L, nx.k0, nx.six);    \
        if (t + 1 < nsl) read_frags<NA, NB, SIX>(F0, NXT, 0, wm, wn, lane);  \
        if (MMA) mma_frags<SIX>(F1, acc);                                    \
    }
    for (int s0 = 0; s0 < nsl; s0 += kFlushSlabs) {
#pragma unroll
        for (int j = 0; j < kFlushSlabs / 2; ++j) {
            const int s = s0 + 2 * j;
            if (s < nsl) PIPE_STEP(S0, S1, 0)
            if (s + 1 < nsl) PIPE_STEP(S1, S0, 1)
        }
        if (FLUSH && MMA) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)acc[a][b][r];
            zero(acc);
        }
    }
#undef PIPE_STEP
}


// Steps t0 <= t < t1 of run_ring (below), all with six products (SIX) or
// all with three; without MMA only the copies and barriers.
template <int NA, int NB, bool FLUSH, bool SIX, bool MMA>
__device__ __forceinline__ void ring_phase(SlabT<NA, NB> &S0, SlabT<NA, NB> &S1, const LoaderT<NA, NB> &L, int k0,
                                           int dk, int t0, int t1, int last, int n3_load, int wm, int wn, int lane,
                                           v16f (&acc)[2][2], double (&acc64)[2][2][16], NextRun nx, int fin) {
#define RING_STEP(CUR, NXT, O)                                       \
    ring_barrier<0>();                                               \
    if (nx.on && t + O + 1 == fin) load_slab(NXT, L, nx.k0, nx.six); \
    else load_slab(NXT, L, k0 + min(t + O + 1, last) * dk, t + O + 1 >= n3_load); \
    if (MMA && t + O < t1) mma_slab<NA, NB, SIX>(CUR, wm, wn, lane, acc);
    for (int s = t0; s < t1; s += kFlushSlabs) {
#pragma unroll
        for (int j = 0; j < kFlushSlabs / 2; ++j) {
            const int t = s + 2 * j;
            if (t < t1) {
                RING_STEP(S0, S1, 0)
                RING_STEP(S1, S0, 1)
            }
        }
        if (FLUSH && MMA) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)acc[a][b][r];
            zero(acc);
        }
    }
#undef RING_STEP
}

// Multiplies nsl consecutive K slabs of the block into acc through the two
// buffers S0, S1.  Slab t is block k0 + t*dk of the tiles (dk = +-1); slabs
// t < n3 take three products, the others six; the copies of slabs
// t < n3_load skip the l pieces (n3_load <= n3).  n3 is even or nsl, so
// slab n3 always lands in S0.  Each step waits
// for the one copy in flight (its slab), then, once every wave is past the
// barrier, copies the next slab into the buffer the previous step read;
// past the end it copies the last slab again (same addresses, cache hits),
// so the steps are alike.  With FLUSH, acc is added into acc64 and cleared
// after every kFlushSlabs slabs of a phase and at the end.  A group of
// kFlushSlabs slabs is unrolled in full so the compiler can tell which
// buffer every LDS read and copy touches (and adds no wait of its own).
// Every wave must call it with the same k0, dk, nsl and n3_load; n3 may
// differ between waves when it is 0 or nsl (each wave then runs nsl steps,
// rounded up to even, and as many barriers).  On return all copies have
// landed, and the buffers may be refilled after a barrier.  With pre, slab
// 0's copy into S0 was issued by the run before; with nx.on, the last step
// (whose copy goes to S0, the step count being even) copies the next run's
// first slab instead of this run's last again, and it is left in flight.
template <int NA, int NB, bool FLUSH, bool MMA = true>
__device__ __forceinline__ void run_ring(SlabT<NA, NB> &S0, SlabT<NA, NB> &S1, const LoaderT<NA, NB> &L, int k0,
                                         int dk, int nsl, int n3, int n3_load, int wm, int wn, int lane,
                                         v16f (&acc)[2][2], double (&acc64)[2][2][16], bool pre = false,
                                         NextRun nx = NextRun{0, false, false}) {
    if (nsl <= 0) return;
    const int last = nsl - 1, fin = (nsl + 1) & ~1;  // steps run: nsl rounded up to even
    if (!pre) load_slab(S0, L, k0, n3_load == 0);
    ring_phase<NA, NB, FLUSH, false, MMA>(S0, S1, L, k0, dk, 0, n3, last, n3_load, wm, wn, lane, acc, acc64, nx, fin);
    ring_phase<NA, NB, FLUSH, true, MMA>(S0, S1, L, k0, dk, n3, nsl, last, n3_load, wm, wn, lane, acc, acc64, nx, fin);
    if (!nx.on) {
        // the trailing copy lands before anyone may reuse or free the LDS
        asm volatile("" ::: "memory");
        MPG_WAIT_VM(0);
        asm volatile("" ::: "memory");
    }
}

// nsl slabs whose first n3 take three products (pipelined ring) and the
// rest six (the plain ring, which keeps one step's fragments in registers:
// the expansion's two accumulator sets leave no room for two six-product
// fragment sets).  The runs are chained: each issues the next one's first
// copy from its last steps (pre: this call's first copy was issued so;
// nx: the run after this call, whose first copy the call issues if it can,
// and then returns true).  PIPE false: the plain ring for both, unchained,
// for kernels with no registers to spare for a second fragment set.
template <int NA, int NB, bool PIPE = true>
__device__ __forceinline__ bool run_tiered(SlabT<NA, NB> &S0, SlabT<NA, NB> &S1, const LoaderT<NA, NB> &L, int k0,
                                           int dk, int nsl, int n3, int wm, int wn, int lane, v16f (&acc)[2][2],
                                           double (&acc64)[2][2][16], bool pre = false,
                                           NextRun nx = NextRun{0, false, false}) {
    if constexpr (!PIPE) {
        run_ring<NA, NB, false>(S0, S1, L, k0, dk, nsl, n3, n3, wm, wn, lane, acc, acc64);
        __syncthreads();
        return false;
    }
    if (nsl <= 0) return false;
    if (n3 > 0 && nsl > n3) {
        // n3 is even here: the three-product run's step n3 - 2 reads S0
        run_pipe<NA, NB, false, false>(S0, S1, L, k0, dk, n3, wm, wn, lane, acc, acc64, pre,
                                       NextRun{k0 + n3 * dk, true, true});
        run_ring<NA, NB, false>(S0, S1, L, k0 + n3 * dk, dk, nsl - n3, 0, 0, wm, wn, lane, acc, acc64, true, nx);
    } else if (n3 > 0) {
        const bool chain = nx.on && (n3 & 1) == 0;
        run_pipe<NA, NB, false, false>(S0, S1, L, k0, dk, n3, wm, wn, lane, acc, acc64, pre,
                                       NextRun{nx.k0, nx.six, chain});
        return chain;
    } else {
        run_ring<NA, NB, false>(S0, S1, L, k0, dk, nsl, 0, 0, wm, wn, lane, acc, acc64, pre, nx);
    }
    if (!nx.on) __syncthreads();  // no wave still reads the buffers the next run refills
    return nx.on;
}


// ---------------------------------------------------------------------------
// One output block of GEMM1, NA row tiles x (3 - NA) column tiles of 128:
// NA = 1 is 128 x 256 (column pair tn: two 128-column tiles, pairs of the
// even-m block first, then of the odd-m block; row tile tm), NA = 2 is
// 256 x 128 (column tile tn, tiles of the even-m block first; row tile pair
// tm); K split tz.  Writes Bpart[tz][row][col] in FP64 (non-temporally
// with NT).  Each output takes the same products in the same order in both
// shapes.
template <bool FOLD, int NA, bool NT = false>
__device__ __forceinline__ void gemm1_tile(const SplitArgs &g, int tn, int tm, int tz, SlabT<NA, 3 - NA> &S0,
                                           SlabT<NA, 3 - NA> &S1) {
    constexpr int NB = 3 - NA;
    const int rows = g.rows, np = g.np, ne_p = g.ne_p;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = (wave % (2 * NA)) * 64, wn = (wave / (2 * NA)) * 64;
    // column units (pairs or tiles) of the even block
    const int ue = NA == 1 ? (g.tiles_e + 1) / 2 : g.tiles_e;
    const bool odd = FOLD && tn >= ue;
    const int u = odd ? tn - ue : tn;  // column unit within the parity block
    const int ct0 = (odd ? g.tiles_e : 0) + NB * u;
    // a second tile past the block's end: in bounds, and its columns are never stored
    const int ct1 = min(ct0 + 1, g.tiles_e + g.tiles_o - 1);
    const int cl = NB * u * TB;  // first column within the parity block
    const int c0 = (odd ? ne_p : 0) + cl;
    const int cend = odd ? np : (FOLD ? ne_p : np);
    const int m0 = tm * NA * TB;
    const int rt_used = (rows + TB - 1) / TB;  // row tiles holding this call's rows
    const int kbeg = tz * g.kchunk;
    const int kend = min(g.kang, kbeg + g.kchunk);
    const int nsl = kend > kbeg ? (kend - kbeg) / TK : 0;

    // A: the pre-split rho (+-) of this block's column parity; B: split U
    // (a second row tile past the rows in use is read in bounds and never stored)
    LoaderT<NA, NB> L;
    const size_t tstride = (size_t)g.ks1 * 3 * kBlk;
    const bf16 *A = g.A + (odd ? (size_t)g.row_tiles * tstride : 0);
    L.a[0] = A + (size_t)(NA * tm) * tstride;
    if constexpr (NA == 2) L.a[1] = A + (size_t)min(2 * tm + 1, rt_used - 1) * tstride;
    L.b[0] = g.U + (size_t)ct0 * tstride;
    if constexpr (NB == 2) L.b[1] = g.U + (size_t)ct1 * tstride;
    L.part = wave * 512;
    L.lo = L.part + lane * 8;

    v16f acc[2][2];
    double acc64[2][2][16];
    zero(acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;
    // six products for a wave whose first column lies in its parity block's
    // tier; the block copies the l pieces when any of its waves needs them
    const int six_par = odd ? g.six_o : g.six_e;
    const bool six_b = cl < six_par, six_w = cl + wn < six_par;
    // the waves on a second tile past the parity block's last, or on a
    // second row tile past the rows in use, only copy and wait (the same
    // steps and barriers); the SIMD they share goes to the other wave
    const bool idle = NA == 1 ? wn >= TB && 2 * u + 1 >= (odd ? g.tiles_o : g.tiles_e)
                              : wm >= TB && 2 * tm + 1 >= rt_used;
    const int n3 = six_w ? 0 : nsl, n3_load = six_b ? 0 : nsl;
    if (idle) run_ring<NA, NB, true, false>(S0, S1, L, kbeg / TK, 1, nsl, n3, n3_load, wm, wn, lane, acc, acc64);
    else run_ring<NA, NB, true, true>(S0, S1, L, kbeg / TK, 1, nsl, n3, n3_load, wm, wn, lane, acc, acc64);

    double *out = g.Bpart + (size_t)tz * rows * np;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int rr = m0 + wm + 32 * a + d_row(lane, r);
                int cc = c0 + wn + 32 * b + (lane & 31);
                if (rr < rows && cc < cend) store<NT>(out + (size_t)rr * np + cc, acc64[a][b][r]);
            }
}

// 128 rows x 256 columns (GEMM1) or angular cells (GEMM2), and 256 x 128
typedef SlabT<1, 2> Slab1;
typedef SlabT<2, 1> Slab2;
static_assert(sizeof(Slab1) == sizeof(Slab2), "both block shapes use the same LDS");

// One output block of GEMM2, NA row tiles x (3 - NA) angular tiles of 128:
// NA = 1 is 128 x 256 (row tile tm, angular tile pair tn), NA = 2 is
// 256 x 128 (row tile pair tm, angular tile tn).  The even-m K block goes
// into acc_e, then the odd-m block into acc_o, each walked from its top slab
// down; per-patch method: the moment sets of the patches one after the
// other, each flushed into FP64.
// NT: Phi is stored non-temporally (the fused batch kernel, whose L2
// write-backs should not carry it).
template <typename T, bool FOLD, bool PP, int NA, bool NT = false>
__device__ __forceinline__ void gemm2_tile(const SplitArgs &g, int tm, int tn, SlabT<NA, 3 - NA> &S0,
                                           SlabT<NA, 3 - NA> &S1) {
    constexpr int NB = 3 - NA;
    T *phi = (T *)g.phi;
    const int rows = g.rows, np = g.np, ne_p = g.ne_p, n_ang = g.n_ang, n_r = g.n_r;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = (wave % (2 * NA)) * 64, wn = (wave / (2 * NA)) * 64;
    const int m0 = tm * NA * TB, n0 = tn * NB * TB;
    const int n_cols = g.kang;                  // angular cells of all output patches (tiles of TB)
    const int rt_used = (rows + TB - 1) / TB;   // row tiles holding this call's rows

    // a second tile past the end is read in bounds and never stored
    LoaderT<NA, NB> L;
    const size_t tstride = (size_t)g.ks2 * 3 * kBlk;
    L.a[0] = g.M + (size_t)(NA * tm) * tstride;
    if constexpr (NA == 2) L.a[1] = g.M + (size_t)min(2 * tm + 1, rt_used - 1) * tstride;
    L.b[0] = g.Q + (size_t)(NB * tn) * tstride;
    if constexpr (NB == 2) L.b[1] = g.Q + (size_t)min(2 * tn + 1, n_cols / TB - 1) * tstride;
    L.part = wave * 512;
    L.lo = L.part + lane * 8;

    v16f acc_e[2][2], acc_o[2][2];
    double acc64[2][2][16];
    zero(acc_e);
    zero(acc_o);
    constexpr bool pp = !FOLD && PP;  // per-patch method: g.nq moment sets
    if (FOLD) {
        const int ne = ne_p / TK, no = (np - ne_p) / TK;
        const int e3 = three_slabs(ne, g.six_e / TK), o3 = three_slabs(no, g.six_o / TK);
        // the even block's last run issues the odd block's first copy (its
        // top slab, with l pieces when the odd block starts with six products)
        const bool pre = run_tiered<NA, NB>(S0, S1, L, ne - 1, -1, ne, e3, wm, wn, lane, acc_e, acc64, false,
                                            NextRun{ne + no - 1, o3 == 0, no > 0});
        run_tiered<NA, NB>(S0, S1, L, ne + no - 1, -1, no, o3, wm, wn, lane, acc_o, acc64, pre);
    } else if (!pp) {
        const int ns = g.ks2, n3 = three_slabs(ns, g.six_e / TK);
        run_tiered<NA, NB>(S0, S1, L, ns - 1, -1, ns, n3, wm, wn, lane, acc_e, acc64);
    } else {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;
        const int nsb = np / TK, n3 = three_slabs(nsb, g.six_e / TK);
        for (int gq = 0; gq < g.nq; ++gq) {
            run_tiered<NA, NB, false>(S0, S1, L, (gq + 1) * nsb - 1, -1, nsb, n3, wm, wn, lane, acc_e, acc64);
            // each patch's moment set is summed in FP32 (as the single set
            // of the other forms) and added in FP64
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)acc_e[a][b][r];
            zero(acc_e);
        }
    }

    // Output: row rr = f*n_r + i of (field, shell), column kk = gp*n_angp +
    // jk of (patch, cell), at phi + f*fld + gp*pstride + i*n_ang + jk.  The
    // row offsets of the block go to LDS once (one division per row; -1:
    // past the last row), the column offsets of this thread's two columns
    // are computed once, and a block inside the output on both axes stores
    // without checks.
    const size_t pstride = (size_t)n_r * n_ang, fld = (size_t)g.n_patches * pstride;
    const int n_angp = g.n_angp;
    __syncthreads();  // every wave is past its last read of the slab buffers
    long long *row_off = reinterpret_cast<long long *>(&S0);
    for (int j = threadIdx.x; j < NA * TB; j += kThreads) {
        const int rr = m0 + j;
        long long v = -1;
        if (rr < rows) {
            const int f = rr / n_r, i = rr - f * n_r;
            v = (long long)f * (long long)fld + (long long)i * n_ang;
        }
        row_off[j] = v;
    }
    long long col_off[2];
    bool col_ok[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int kk = n0 + wn + 32 * b + (lane & 31);
        const int gp = kk / n_angp, jk = kk - gp * n_angp;
        col_ok[b] = kk < n_cols && jk < n_ang;
        col_off[b] = (long long)gp * (long long)pstride + jk;
    }
    // the block's columns lie in one patch's cells and its rows in the output
    const int c_last = n0 + NB * TB - 1;
    const bool full = m0 + NA * TB <= rows && c_last < n_cols && n0 / n_angp == c_last / n_angp &&
                      c_last - (c_last / n_angp) * n_angp < n_ang;
    __syncthreads();
    auto put = [&](int a, int b, int r) {
        const long long ro = row_off[wm + 32 * a + d_row(lane, r)];
        T *o = phi + ro + col_off[b];
        double e = (double)acc_e[a][b][r];
        if (!FOLD && pp) e = acc64[a][b][r];
        if (FOLD) {
            const double od = (double)acc_o[a][b][r];
            store<NT>(o, (T)(e + od));
            store<NT>(o + pstride, (T)(e - od));
        } else {
            store<NT>(o, (T)e);
        }
    };
    if (full) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) put(a, b, r);
    } else {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (col_ok[b] && row_off[wm + 32 * a + d_row(lane, r)] >= 0) put(a, b, r);
    }
}

// ---------------------------------------------------------------------------
// Grid launches for one plan: GEMM1 grid x = (column unit, row unit), z =
// K split; GEMM2 grid x = row tile (pair), y = angular tile pair (tile).
// A GEMM1 column unit is a pair of 128-column tiles (NA = 1) or one tile
// (NA = 2), a row unit one row tile or a pair.  GEMM1's blocks in x run
// over (column unit, row unit), the units that take six products first
// (they take about twice as long as the others), so the long blocks are
// dispatched before the short ones.
template <int NA>
__host__ __device__ inline void gemm1_units(int tiles_e, int tiles_o, int &ue, int &uo) {
    ue = NA == 1 ? (tiles_e + 1) / 2 : tiles_e;
    uo = NA == 1 ? (tiles_o + 1) / 2 : tiles_o;
}

template <bool FOLD, int NA>
__global__ __launch_bounds__(kThreads) void k_gemm1(SplitArgs g) {
    __shared__ SlabT<NA, 3 - NA> s0, s1;
    int ue, uo;
    gemm1_units<NA>(g.tiles_e, g.tiles_o, ue, uo);
    const int he = six_units(g.six_e, ue, 3 - NA), ho = FOLD ? six_units(g.six_o, uo, 3 - NA) : 0;
    const int nh = he + ho, nl = ue + uo - nh;
    const int rt = gridDim.x / (ue + uo);
    int b = blockIdx.x, tn, tm;
    if (b < nh * rt) {
        const int i = b % nh;
        tm = b / nh;
        tn = i < he ? i : ue + (i - he);
    } else {
        b -= nh * rt;
        const int i = b % nl;
        tm = b / nl;
        tn = i < ue - he ? he + i : ue + ho + (i - (ue - he));
    }
    gemm1_tile<FOLD, NA>(g, tn, tm, blockIdx.z, s0, s1);
}

template <typename T, bool FOLD, bool PP, int NA>
__global__ __launch_bounds__(kThreads) void k_gemm2(SplitArgs g) {
    __shared__ SlabT<NA, 3 - NA> s0, s1;
    gemm2_tile<T, FOLD, PP, NA>(g, blockIdx.x, blockIdx.y, s0, s1);
}

// The fused batch kernel: one persistent block per CU takes items of every
// stage of every field from one queue (ordered by batch_order.h, so an
// item's producers were taken before it).  Before an item of stage s of
// field f, the first thread waits until every item of stage s-1 of f has
// finished (a bounded poll; on giving up it sets the status word and every
// block drains).  After an item, once every thread's stores are complete,
// the first thread makes them visible device-wide (release fence: this
// XCD's L2 written back) and counts the item; the item that completes a
// field's expansion stamps the field's completion time (the expansion's
// output is read by no item, needs no write-back and is stored
// non-temporally).  Each field's items take its plan's choices: the block
// shapes of both contractions and the scans' chunk count (eight thread
// rows of 64 lanes, on the slab buffers' LDS).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_fused(const SplitArgs *__restrict__ args,
                                                          const ScanArgs *__restrict__ sargs,
                                                          const FusedItem *__restrict__ items, int n_items,
                                                          FusedCtl c) {
    __shared__ Slab1 sl[2];
    __shared__ int slot, go;
    Slab1 &s0 = sl[0], &s1 = sl[1];
    // the same two buffers in the 256 x 128 block shape
    Slab2 &t0 = *reinterpret_cast<Slab2 *>(&sl[0]), &t1 = *reinterpret_cast<Slab2 *>(&sl[1]);
    const int tid = threadIdx.x;
    for (;;) {
        __syncthreads();  // every thread is done with the previous item and the shared slots
        if (tid == 0) slot = atomicAdd(c.head, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(slot);
        if (it >= n_items) break;
        const FusedItem w = items[it];
        if (tid == 0) {
            int ok = 1;
            if (w.st > 0) {
                const int *cnt = c.done + w.f * kFusedStages + w.st - 1;
                const int need = c.need[w.f * kFusedStages + w.st - 1];
                for (int spins = 0; __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need;
                     ++spins) {
                    if (spins >= c.spin_limit ||
                        __hip_atomic_load(c.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        ok = 0;
                        __hip_atomic_store(c.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
            }
            go = ok;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(go)) break;
        const SplitArgs &g = args[w.f];
        if (w.st == 0) {
            // input split: units of 2048 chunks
            for (int u = w.a; u < w.a + w.b; ++u) {
                if (g.fold) fold_split_unit<T, true, true>(g, u, tid);
                else fold_split_unit<T, false, true>(g, u, tid);
            }
        } else if (w.st == 1) {
            if (g.g1_rows == 2) {
                if (g.fold) gemm1_tile<true, 2, true>(g, w.a, w.b, w.c, t0, t1);
                else gemm1_tile<false, 2, true>(g, w.a, w.b, w.c, t0, t1);
            } else {
                if (g.fold) gemm1_tile<true, 1, true>(g, w.a, w.b, w.c, s0, s1);
                else gemm1_tile<false, 1, true>(g, w.a, w.b, w.c, s0, s1);
            }
        } else if (w.st == 2) {
            // the field's own chunk count, eight thread rows
            constexpr int kMC = scan_detail::kMaxChunks * scan_detail::kLanes;
            static_assert(4 * kMC * sizeof(double) <= sizeof(Slab1), "scan carries fit in one slab buffer");
            double *lds = reinterpret_cast<double *>(&s0);
            scan_detail::scan_block_core<true>(sargs[w.f], w.a, tid & 63, tid >> 6, kThreads / 64, lds, lds + kMC,
                                               lds + 2 * kMC, lds + 3 * kMC);
        } else {
            // w.c angular units of row unit w.a, from unit w.b
            for (int k = 0; k < w.c; ++k) {
                if (k) __syncthreads();  // every wave is done with the slab buffers
                if (g.g2_rows == 2) {
                    if (g.fold) gemm2_tile<T, true, false, 2, true>(g, w.a, w.b + k, t0, t1);
                    else gemm2_tile<T, false, false, 2, true>(g, w.a, w.b + k, t0, t1);
                } else {
                    if (g.fold) gemm2_tile<T, true, false, 1, true>(g, w.a, w.b + k, s0, s1);
                    else gemm2_tile<T, false, false, 1, true>(g, w.a, w.b + k, s0, s1);
                }
            }
        }
        // this block's stores are complete; then (but after the expansion,
        // whose output no item reads) one wave writes this XCD's L2 back
        __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0) lgkmcnt(0)
        __syncthreads();
        if (tid == 0 && w.st < kFusedStages - 1) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tid == 0) {
            const int old = atomicAdd(c.done + w.f * kFusedStages + w.st, 1);
            if (w.st == kFusedStages - 1 && old + 1 == c.need[w.f * kFusedStages + w.st])
                c.stamps[w.f] = wall_clock64();
        }
    }
}

}  // namespace

hipError_t batch_fused_bf16(const SplitArgs *args, const ScanArgs *sargs, const FusedItem *items, int n_items,
                            FusedCtl ctl, int io_dtype, int blocks, hipStream_t s) {
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_fused<double>), dim3(blocks), dim3(kThreads), 0, s, args, sargs, items, n_items,
                           ctl);
    else
        hipLaunchKernelGGL((k_batch_fused<float>), dim3(blocks), dim3(kThreads), 0, s, args, sargs, items, n_items,
                           ctl);
    return hipGetLastError();
}

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
    g.kchunk = ksplit_chunk(p.kang(), p.splitk, TK);
    g.splitk = p.splitk;
    g.U = p.Us;
    g.Q = p.Qs;
    g.M = p.Ms;
    g.Bpart = p.Bpart;
    g.A = p.A_split;
    g.row_tiles = p.row_tiles();
    g.ks1 = p.kang() / TK;
    g.ks2 = p.kq() / TK;
    g.six_e = p.six_e;
    g.six_o = p.six_o;
    g.g1_rows = p.gemm1_rows;
    g.g2_rows = p.gemm2_rows;
    return g;
}

// one thread per 16-byte chunk of the row tiles holding the fields' rows
// (slabs in groups of four)
size_t split_input_threads(const Plan &p, int n_fields) {
    return (size_t)((n_fields * p.n_r + TB - 1) / TB) * ((p.kang() / TK + 3) / 4) * 2048;
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
    const int rt = (g.rows + TB - 1) / TB;
    int ue, uo;
    if (g.g1_rows == 2) {
        gemm1_units<2>(g.tiles_e, g.tiles_o, ue, uo);
        dim3 grid((ue + uo) * ((rt + 1) / 2), 1, p.splitk);
        if (p.fold) hipLaunchKernelGGL((k_gemm1<true, 2>), grid, dim3(kThreads), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm1<false, 2>), grid, dim3(kThreads), 0, p.stream, g);
    } else {
        gemm1_units<1>(g.tiles_e, g.tiles_o, ue, uo);
        dim3 grid((ue + uo) * rt, 1, p.splitk);
        if (p.fold) hipLaunchKernelGGL((k_gemm1<true, 1>), grid, dim3(kThreads), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm1<false, 1>), grid, dim3(kThreads), 0, p.stream, g);
    }
    return hipGetLastError();
}

template <typename T, int NA>
void launch_gemm2(const Plan &p, const SplitArgs &g, dim3 grid) {
    if (p.fold) hipLaunchKernelGGL((k_gemm2<T, true, false, NA>), grid, dim3(kThreads), 0, p.stream, g);
    else if (g.nq > 1) hipLaunchKernelGGL((k_gemm2<T, false, true, NA>), grid, dim3(kThreads), 0, p.stream, g);
    else hipLaunchKernelGGL((k_gemm2<T, false, false, NA>), grid, dim3(kThreads), 0, p.stream, g);
}

hipError_t gemm2_bf16(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    SplitArgs g = split_args(p, n_fields, nullptr, phi, phi_dtype, true);
    const int rt = (g.rows + TB - 1) / TB, at = g.kang / TB;
    if (p.gemm2_rows == 2) {
        dim3 grid((rt + 1) / 2, at);
        if (phi_dtype == MPG_F64) launch_gemm2<double, 2>(p, g, grid);
        else launch_gemm2<float, 2>(p, g, grid);
    } else {
        dim3 grid(rt, (at + 1) / 2);
        if (phi_dtype == MPG_F64) launch_gemm2<double, 1>(p, g, grid);
        else launch_gemm2<float, 1>(p, g, grid);
    }
    return hipGetLastError();
}

}  // namespace mpg
