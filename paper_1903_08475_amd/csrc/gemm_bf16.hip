// Split-BF16 MFMA contractions of the solve (Sec. 4.3 steps 2 and 5).
//
// Each operand x, taken in FP32, is written as x = h + m + l, with h, m, l
// the round-to-nearest bf16 of the successive residuals (exact: 24
// significant bits).  A product a*b is formed from the six partial products whose
// combined weight is at least 2^-18 of the leading one:
//   ah*bh + ah*bm + am*bh + ah*bl + am*bm + al*bh
// on v_mfma_f32_32x32x16_bf16 (bf16 products are exact in FP32).  The FP32
// accumulators are flushed into FP64 registers every `flush` K steps, so
// no FP32 sum runs over more than flush*32 terms (GEMM1; GEMM2's K is the
// moment count, short enough for FP32 sums).
//
// GEMM1 (moments, Eq. B_CS) folds and splits rho in its tile loader:
// A = rho_Yin +- rho_Yang (U_Yang = (-1)^m U_Yin, Sec. 4.2), rounded once
// to FP32 and converted to three bf16 pieces in LDS; U comes pre-split from
// the plan.
// GEMM2 (expansion, Eq. gravpotmult) reads M pre-split by the radial scan
// and Q pre-split by the plan, sums even- and odd-m columns separately and
// writes Phi_Yin = E + O, Phi_Yang = E - O.  Its K loop runs from the
// highest degree down to l = 0, so the dominant low-degree terms are added
// to the smallest partial sums last.
//
// Tiles: 128x128 per block of 256 threads (2x2 waves of 64x64 = 2x2 MFMA
// blocks of 32x32), K slabs of 32, double-buffered in LDS (120 KB): while the
// waves multiply slab s from one buffer, slab s+1 is written to the other
// from registers and slab s+2 is fetched from memory; one barrier per slab.
#include "mpg_internal.h"

namespace mpg {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
// native vector types (HIP's uint4/float4 classes defeat register promotion)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int TB = kSplitTile, TK = 32, LDK = TK + 8;
constexpr int kFlush1 = 16;  // GEMM1: FP32 runs of at most 512 terms

struct Pieces {
    bf16 h[TB][LDK];
    bf16 m[TB][LDK];
    bf16 l[TB][LDK];
};

struct Stage {
    Pieces A, B;
};

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

// rho_Yin +- rho_Yang rounded once to FP32 (the split path's input precision)
__device__ inline float fold(float a, float b, bool odd) { return odd ? a - b : a + b; }
__device__ inline float fold(double a, double b, bool odd) { return (float)(odd ? a - b : a + b); }

// one 32-deep slab from LDS for a wave's 64x64 tile: for each 16-deep step
// the six partial products are issued product by product over the four
// accumulators, smallest weight first, so consecutive MFMAs never depend on
// each other.
__device__ inline void mma_slab(const Pieces &A, const Pieces &B, int wm, int wn, int lane, v16f (&acc)[2][2]) {
    const int lr = lane & 31, lk = 8 * (lane >> 5);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
        v8bf ah0, ah1, am0, am1, al0, al1, bh0, bh1, bm0, bm1, bl0, bl1;
        ah0 = *(const v8bf *)&A.h[wm + lr][ks + lk];
        ah1 = *(const v8bf *)&A.h[wm + 32 + lr][ks + lk];
        am0 = *(const v8bf *)&A.m[wm + lr][ks + lk];
        am1 = *(const v8bf *)&A.m[wm + 32 + lr][ks + lk];
        al0 = *(const v8bf *)&A.l[wm + lr][ks + lk];
        al1 = *(const v8bf *)&A.l[wm + 32 + lr][ks + lk];
        bh0 = *(const v8bf *)&B.h[wn + lr][ks + lk];
        bh1 = *(const v8bf *)&B.h[wn + 32 + lr][ks + lk];
        bm0 = *(const v8bf *)&B.m[wn + lr][ks + lk];
        bm1 = *(const v8bf *)&B.m[wn + 32 + lr][ks + lk];
        bl0 = *(const v8bf *)&B.l[wn + lr][ks + lk];
        bl1 = *(const v8bf *)&B.l[wn + 32 + lr][ks + lk];
#define MM4(X0, X1, Y0, Y1)                                                              \
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X0, Y0, acc[0][0], 0, 0, 0); \
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X0, Y1, acc[0][1], 0, 0, 0); \
    acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X1, Y0, acc[1][0], 0, 0, 0); \
    acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X1, Y1, acc[1][1], 0, 0, 0)
        MM4(al0, al1, bh0, bh1);
        MM4(am0, am1, bm0, bm1);
        MM4(ah0, ah1, bl0, bl1);
        MM4(am0, am1, bh0, bh1);
        MM4(ah0, ah1, bm0, bm1);
        MM4(ah0, ah1, bh0, bh1);
#undef MM4
    }
#ifdef MPG_SCHED
    // issue the second step's fragment reads between the first step's MFMAs
    __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 24, 0);
#endif
}

// 16 consecutive K values of the three pieces of one row, held in registers
struct Raw16 {
    u32x4 h0, h1, m0, m1, l0, l1;
};

__device__ __forceinline__ void load_pieces(Raw16 &r, const bf16 *h, const bf16 *m, const bf16 *l, size_t off) {
    r.h0 = *(const u32x4 *)(h + off);
    r.h1 = *(const u32x4 *)(h + off + 8);
    r.m0 = *(const u32x4 *)(m + off);
    r.m1 = *(const u32x4 *)(m + off + 8);
    r.l0 = *(const u32x4 *)(l + off);
    r.l1 = *(const u32x4 *)(l + off + 8);
}

__device__ __forceinline__ void store_pieces(Pieces &S, const Raw16 &r, int row, int k) {
    *(u32x4 *)&S.h[row][k] = r.h0;
    *(u32x4 *)&S.h[row][k + 8] = r.h1;
    *(u32x4 *)&S.m[row][k] = r.m0;
    *(u32x4 *)&S.m[row][k + 8] = r.m1;
    *(u32x4 *)&S.l[row][k] = r.l0;
    *(u32x4 *)&S.l[row][k + 8] = r.l1;
}

__device__ __forceinline__ uint32_t pack2(bf16 a, bf16 b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

__device__ __forceinline__ void store_split(Pieces &S, const float (&av)[16], int row, int k) {
    uint32_t h[8], m[8], l[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        bf16 h0, m0, l0, h1, m1, l1;
        split3f(av[2 * q], h0, m0, l0);
        split3f(av[2 * q + 1], h1, m1, l1);
        h[q] = pack2(h0, h1);
        m[q] = pack2(m0, m1);
        l[q] = pack2(l0, l1);
    }
    *(u32x4 *)&S.h[row][k] = (u32x4){h[0], h[1], h[2], h[3]};
    *(u32x4 *)&S.h[row][k + 8] = (u32x4){h[4], h[5], h[6], h[7]};
    *(u32x4 *)&S.m[row][k] = (u32x4){m[0], m[1], m[2], m[3]};
    *(u32x4 *)&S.m[row][k + 8] = (u32x4){m[4], m[5], m[6], m[7]};
    *(u32x4 *)&S.l[row][k] = (u32x4){l[0], l[1], l[2], l[3]};
    *(u32x4 *)&S.l[row][k + 8] = (u32x4){l[4], l[5], l[6], l[7]};
}

// 16 consecutive values of rho_Yin +- rho_Yang (or rho) of one row, in FP32.
// vec: n_ang % 16 == 0, so the 16 values are all inside the row or all
// outside it, and 16-byte aligned.
template <typename T, bool FOLD>
__device__ __forceinline__ void load_rho(float (&av)[16], const T *r0, const T *r1, int k, int n_ang, bool row_ok,
                                         bool odd, bool vec) {
    if (vec) {
        if (row_ok && k < n_ang) {
            if (sizeof(T) == 4) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    f32x4 x = *(const f32x4 *)(r0 + k + 4 * q);
                    f32x4 y = FOLD ? *(const f32x4 *)(r1 + k + 4 * q) : (f32x4){0.f, 0.f, 0.f, 0.f};
                    av[4 * q + 0] = FOLD ? fold(x.x, y.x, odd) : x.x;
                    av[4 * q + 1] = FOLD ? fold(x.y, y.y, odd) : x.y;
                    av[4 * q + 2] = FOLD ? fold(x.z, y.z, odd) : x.z;
                    av[4 * q + 3] = FOLD ? fold(x.w, y.w, odd) : x.w;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    f64x2 x = *(const f64x2 *)(r0 + k + 2 * q);
                    f64x2 y = FOLD ? *(const f64x2 *)(r1 + k + 2 * q) : (f64x2){0.0, 0.0};
                    av[2 * q + 0] = FOLD ? fold(x.x, y.x, odd) : (float)x.x;
                    av[2 * q + 1] = FOLD ? fold(x.y, y.y, odd) : (float)x.y;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) av[q] = 0.0f;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float v = 0.0f;
            if (row_ok && k + q < n_ang) v = FOLD ? fold(r0[k + q], r1[k + q], odd) : (float)r0[k + q];
            av[q] = v;
        }
    }
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
// rho, rounded once to FP32 and written as three bf16 pieces
// A[parity][piece][row][k] (k < n_angp; zero past n_ang).  Thread = 8
// consecutive k of one row.
template <typename T, bool FOLD>
__device__ __forceinline__ void fold_split_row8(const SplitArgs &g, size_t t) {
    const int per_row = g.n_angp / 8;
    const int row = (int)(t / per_row), k0 = (int)(t - (size_t)row * per_row) * 8;
    if (row >= g.rows) return;
    const int n_r = g.n_r, n_ang = g.n_ang;
    const int f = row / n_r, i = row - f * n_r;
    const size_t fld = (size_t)(FOLD ? 2 : 1) * n_r * n_ang;
    const T *r0 = (const T *)g.rho + f * fld + (size_t)i * n_ang;
    const T *r1 = r0 + (size_t)n_r * n_ang;
    float v0[8], v1[8];
    if ((n_ang & 7) == 0) {
        if (k0 < n_ang) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                v0[q] = (float)0;
                v1[q] = (float)0;
            }
            if (sizeof(T) == 4) {
                f32x4 a0 = *(const f32x4 *)(r0 + k0), a1 = *(const f32x4 *)(r0 + k0 + 4);
                v0[0] = a0.x; v0[1] = a0.y; v0[2] = a0.z; v0[3] = a0.w;
                v0[4] = a1.x; v0[5] = a1.y; v0[6] = a1.z; v0[7] = a1.w;
                if (FOLD) {
                    f32x4 b0 = *(const f32x4 *)(r1 + k0), b1 = *(const f32x4 *)(r1 + k0 + 4);
                    v1[0] = b0.x; v1[1] = b0.y; v1[2] = b0.z; v1[3] = b0.w;
                    v1[4] = b1.x; v1[5] = b1.y; v1[6] = b1.z; v1[7] = b1.w;
                }
            }
        }
    }
    // FP64 input (or unaligned rows): element by element in double
    double d0[8], d1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = k0 + q;
        const bool in = k < n_ang;
        if (sizeof(T) == 4 && (n_ang & 7) == 0) {
            d0[q] = in ? (double)v0[q] : 0.0;
            d1[q] = in && FOLD ? (double)v1[q] : 0.0;
        } else {
            d0[q] = in ? (double)r0[k] : 0.0;
            d1[q] = in && FOLD ? (double)r1[k] : 0.0;
        }
    }
    const size_t plane = (size_t)g.rows_alloc * g.n_angp, off = (size_t)row * g.n_angp + k0;
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
        bf16 *base = g.A + (size_t)(3 * par) * plane + off;
        *(u32x4 *)(base) = (u32x4){h[0], h[1], h[2], h[3]};
        *(u32x4 *)(base + plane) = (u32x4){m[0], m[1], m[2], m[3]};
        *(u32x4 *)(base + 2 * plane) = (u32x4){l[0], l[1], l[2], l[3]};
    }
}

template <typename T, bool FOLD>
__global__ __launch_bounds__(256) void k_fold_split(SplitArgs g) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    fold_split_row8<T, FOLD>(g, t);
}

// batch version: the field's arguments come from device memory
template <typename T>
__global__ __launch_bounds__(256) void k_batch_fold_split(const SplitArgs *args, int f) {
    const SplitArgs g = args[f];
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g.fold) fold_split_row8<T, true>(g, t);
    else fold_split_row8<T, false>(g, t);
}

// ---------------------------------------------------------------------------
// One output tile of GEMM1 (column tile tn: even-m tiles first, then odd-m
// tiles; row tile tm; K split tz).  Writes Bpart[tz][row][col] in FP64.
template <bool FOLD>
__device__ __forceinline__ void gemm1_tile(const SplitArgs &g, int tn, int tm, int tz, Stage (&st)[2]) {
    const int rows = g.rows, n_r = g.n_r, n_ang = g.n_ang, n_angp = g.n_angp, np = g.np, ne_p = g.ne_p;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const bool odd = FOLD && tn >= g.tiles_e;
    const int c0 = odd ? ne_p + (tn - g.tiles_e) * TB : tn * TB;
    const int cend = odd ? np : (FOLD ? ne_p : np);
    const int m0 = tm * TB;
    const int kbeg = tz * g.kchunk;
    const int kend = min(n_angp, kbeg + g.kchunk);
    const int nsl = kend > kbeg ? (kend - kbeg) / TK : 0;

    // loader: thread t covers row t/2 and 16 K values from 16*(t%2); A is
    // the pre-split rho (+-) of this tile's column parity
    const int lr = t >> 1, lk = (t & 1) * 16;
    const int row = m0 + lr;
    const bool row_ok = row < rows;
    const size_t plane = (size_t)g.rows_alloc * n_angp;
    const bf16 *Ah = g.A + (size_t)(odd ? 3 : 0) * plane;
    const bf16 *Am = Ah + plane, *Al = Am + plane;
    const size_t aoff = (size_t)(row_ok ? row : 0) * n_angp;
    const size_t uoff = (size_t)(c0 + lr) * n_angp;
    const bf16 *Uh = g.Uh, *Um = g.Um, *Ul = g.Ul;
    (void)n_r;
    (void)n_ang;
    const u32x4 z = {0u, 0u, 0u, 0u};

    v16f acc[2][2];
    double acc64[2][2][16];
    zero(acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;

    Raw16 ra, bu;
    ra.h0 = ra.h1 = ra.m0 = ra.m1 = ra.l0 = ra.l1 = z;
    if (nsl > 0) {
        if (row_ok) load_pieces(ra, Ah, Am, Al, aoff + kbeg + lk);
        load_pieces(bu, Uh, Um, Ul, uoff + kbeg + lk);
        store_pieces(st[0].A, ra, lr, lk);
        store_pieces(st[0].B, bu, lr, lk);
        if (nsl > 1) {
            if (row_ok) load_pieces(ra, Ah, Am, Al, aoff + kbeg + TK + lk);
            load_pieces(bu, Uh, Um, Ul, uoff + kbeg + TK + lk);
        }
    }
    __syncthreads();
    int step = 0;
    for (int s = 0; s < nsl; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsl) {
            store_pieces(st[cur ^ 1].A, ra, lr, lk);
            store_pieces(st[cur ^ 1].B, bu, lr, lk);
            if (s + 2 < nsl) {
                const int k = kbeg + (s + 2) * TK + lk;
                if (row_ok) load_pieces(ra, Ah, Am, Al, aoff + k);
                load_pieces(bu, Uh, Um, Ul, uoff + k);
            }
        }
        mma_slab(st[cur].A, st[cur].B, wm, wn, lane, acc);
        if (++step == kFlush1) {
            step = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)acc[a][b][r];
            zero(acc);
        }
        __syncthreads();
    }
    double *out = g.Bpart + (size_t)tz * rows * np;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int rr = m0 + wm + 32 * a + d_row(lane, r);
                int cc = c0 + wn + 32 * b + (lane & 31);
                if (rr < rows && cc < cend) out[(size_t)rr * np + cc] = acc64[a][b][r] + (double)acc[a][b][r];
            }
}

// One column block of GEMM2 (nsl slabs starting at column cbase), walked
// from its top slab down to cbase, double-buffered through st.
__device__ __forceinline__ void gemm2_block(Stage (&st)[2], const bf16 *Mh, const bf16 *Mm, const bf16 *Ml,
                                            const bf16 *Qh, const bf16 *Qm, const bf16 *Ql, size_t aoff,
                                            size_t boff, bool row_ok, int cbase, int nsl, int lr, int lk, int wm,
                                            int wn, int lane, v16f (&acc)[2][2]) {
    Raw16 ra, rb;
    const u32x4 z = {0u, 0u, 0u, 0u};
    ra.h0 = ra.h1 = ra.m0 = ra.m1 = ra.l0 = ra.l1 = z;
    if (nsl > 0) {
        int k = cbase + (nsl - 1) * TK + lk;
        if (row_ok) load_pieces(ra, Mh, Mm, Ml, aoff + k);
        load_pieces(rb, Qh, Qm, Ql, boff + k);
        store_pieces(st[0].A, ra, lr, lk);
        store_pieces(st[0].B, rb, lr, lk);
        if (nsl > 1) {
            k -= TK;
            if (row_ok) load_pieces(ra, Mh, Mm, Ml, aoff + k);
            load_pieces(rb, Qh, Qm, Ql, boff + k);
        }
    }
    __syncthreads();
    for (int s = 0; s < nsl; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsl) {
            store_pieces(st[cur ^ 1].A, ra, lr, lk);
            store_pieces(st[cur ^ 1].B, rb, lr, lk);
            if (s + 2 < nsl) {
                const int k = cbase + (nsl - 3 - s) * TK + lk;
                if (row_ok) load_pieces(ra, Mh, Mm, Ml, aoff + k);
                load_pieces(rb, Qh, Qm, Ql, boff + k);
            }
        }
        mma_slab(st[cur].A, st[cur].B, wm, wn, lane, acc);
        __syncthreads();
    }
}

#ifdef MPG_G2_OCC2
// single-buffered variant (two blocks per CU hide each other's latency)
__device__ __forceinline__ void gemm2_block_sb(Stage &st, const bf16 *Mh, const bf16 *Mm, const bf16 *Ml,
                                               const bf16 *Qh, const bf16 *Qm, const bf16 *Ql, size_t aoff,
                                               size_t boff, bool row_ok, int cbase, int nsl, int lr, int lk, int wm,
                                               int wn, int lane, v16f (&acc)[2][2]) {
    Raw16 ra, rb;
    const u32x4 z = {0u, 0u, 0u, 0u};
    ra.h0 = ra.h1 = ra.m0 = ra.m1 = ra.l0 = ra.l1 = z;
    if (nsl > 0) {
        int k = cbase + (nsl - 1) * TK + lk;
        if (row_ok) load_pieces(ra, Mh, Mm, Ml, aoff + k);
        load_pieces(rb, Qh, Qm, Ql, boff + k);
    }
    for (int s = 0; s < nsl; ++s) {
        __syncthreads();
        store_pieces(st.A, ra, lr, lk);
        store_pieces(st.B, rb, lr, lk);
        __syncthreads();
        if (s + 1 < nsl) {
            const int k = cbase + (nsl - 2 - s) * TK + lk;
            if (row_ok) load_pieces(ra, Mh, Mm, Ml, aoff + k);
            load_pieces(rb, Qh, Qm, Ql, boff + k);
        }
        mma_slab(st.A, st.B, wm, wn, lane, acc);
    }
    __syncthreads();
}
#endif

// One output tile of GEMM2 (row tile tm, angular tile tn).  The K slabs of
// the even block come first, then those of the odd block.
template <typename T, bool FOLD, int NS>
__device__ __forceinline__ void gemm2_tile(const SplitArgs &g, int tm, int tn, Stage (&st)[NS]) {
    T *phi = (T *)g.phi;
    const int rows = g.rows, np = g.np, ne_p = g.ne_p, n_ang = g.n_ang, n_r = g.n_r;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int m0 = tm * TB, n0 = tn * TB;
    const int lr = t >> 1, lk = (t & 1) * 16;
    const bool row_ok = m0 + lr < rows;
    const size_t aoff = (size_t)(row_ok ? m0 + lr : 0) * np;
    const size_t boff = (size_t)(n0 + lr) * np;

    v16f acc_e[2][2], acc_o[2][2];
    zero(acc_e);
    zero(acc_o);
#ifdef MPG_G2_OCC2
#define gemm2_block(ST, ...) gemm2_block_sb(ST[0], __VA_ARGS__)
#endif
    if (FOLD) {
        gemm2_block(st, g.Mh, g.Mm, g.Ml, g.Qh, g.Qm, g.Ql, aoff, boff, row_ok, 0, ne_p / TK, lr, lk, wm, wn, lane,
                    acc_e);
        gemm2_block(st, g.Mh, g.Mm, g.Ml, g.Qh, g.Qm, g.Ql, aoff, boff, row_ok, ne_p, (np - ne_p) / TK, lr, lk, wm,
                    wn, lane, acc_o);
    } else {
        gemm2_block(st, g.Mh, g.Mm, g.Ml, g.Qh, g.Qm, g.Ql, aoff, boff, row_ok, 0, np / TK, lr, lk, wm, wn, lane,
                    acc_e);
    }
#ifdef MPG_G2_OCC2
#undef gemm2_block
#endif
    const size_t fld = (size_t)(FOLD ? 2 : 1) * n_r * n_ang;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int rr = m0 + wm + 32 * a + d_row(lane, r);
                int jk = n0 + wn + 32 * b + (lane & 31);
                if (rr >= rows || jk >= n_ang) continue;
                int f = rr / n_r, i = rr - f * n_r;
                T *o = phi + f * fld + (size_t)i * n_ang + jk;
                double e = (double)acc_e[a][b][r];
                if (FOLD) {
                    double od = (double)acc_o[a][b][r];
                    o[0] = (T)(e + od);
                    o[(size_t)n_r * n_ang] = (T)(e - od);
                } else {
                    o[0] = (T)e;
                }
            }
}

// ---------------------------------------------------------------------------
// Grid launches for one plan: GEMM1 grid x = column tile, y = row tile,
// z = K split; GEMM2 grid x = row tile, y = angular tile.
template <bool FOLD>
__global__ __launch_bounds__(256) void k_gemm1(SplitArgs g) {
    __shared__ Stage st[2];
    gemm1_tile<FOLD>(g, blockIdx.x, blockIdx.y, blockIdx.z, st);
}

#ifdef MPG_G2_OCC2
#define G2_BOUNDS __launch_bounds__(256, 2)
#define G2_STAGES 1
#else
#define G2_BOUNDS __launch_bounds__(256)
#define G2_STAGES 2
#endif
template <typename T, bool FOLD>
__global__ G2_BOUNDS void k_gemm2(SplitArgs g) {
    __shared__ Stage st[G2_STAGES];
    gemm2_tile<T, FOLD, G2_STAGES>(g, blockIdx.x, blockIdx.y, st);
}

// Persistent batch kernels: every block takes work items from a queue
// (items[], ordered longest first) through an atomic head until the queue
// is empty.  Item = (field, tile coordinates); args[] holds each field's
// arguments.  No item waits on another, so every block exits.
__device__ __forceinline__ int next_item(int *head, int *slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(head, 1);
    __syncthreads();
    int it = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();
    return it;
}

__global__ __launch_bounds__(256) void k_batch_gemm1(const SplitArgs *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head) {
    __shared__ Stage st[2];
    __shared__ int slot;
    for (;;) {
        const int it = next_item(head, &slot);
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const SplitArgs g = args[w.f];
        if (g.fold) gemm1_tile<true>(g, w.a, w.b, w.c, st);
        else gemm1_tile<false>(g, w.a, w.b, w.c, st);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_batch_gemm2(const SplitArgs *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head) {
    __shared__ Stage st[2];
    __shared__ int slot;
    for (;;) {
        const int it = next_item(head, &slot);
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const SplitArgs g = args[w.f];
        if (g.fold) gemm2_tile<T, true, 2>(g, w.a, w.b, st);
        else gemm2_tile<T, false, 2>(g, w.a, w.b, st);
    }
}

}  // namespace

SplitArgs split_args(const Plan &p, int n_fields, const void *rho, void *phi, int io_dtype) {
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
    g.tiles_e = p.fold ? (p.ne_p + TB - 1) / TB : (p.np + TB - 1) / TB;
    g.tiles_o = p.fold ? (p.no_p + TB - 1) / TB : 0;
    g.kchunk = ((p.n_angp / p.splitk + TK - 1) / TK) * TK;
    g.splitk = p.splitk;
    g.Uh = p.Ut_hi; g.Um = p.Ut_mid; g.Ul = p.Ut_lo;
    g.Qh = p.Qt_hi; g.Qm = p.Qt_mid; g.Ql = p.Qt_lo;
    g.Mh = p.M_hi; g.Mm = p.M_mid; g.Ml = p.M_lo;
    g.Bpart = p.Bpart;
    g.A = p.A_split;
    g.rows_alloc = p.rows_alloc();
    return g;
}

int split_tile_rows(int rows) { return (rows + TB - 1) / TB; }

hipError_t split_input_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    SplitArgs g = split_args(p, n_fields, rho, nullptr, rho_dtype);
    const size_t threads = (size_t)g.rows * (g.n_angp / 8);
    dim3 grid((unsigned)((threads + 255) / 256));
    if (rho_dtype == MPG_F64) {
        if (p.fold) hipLaunchKernelGGL((k_fold_split<double, true>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_fold_split<double, false>), grid, dim3(256), 0, p.stream, g);
    } else {
        if (p.fold) hipLaunchKernelGGL((k_fold_split<float, true>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_fold_split<float, false>), grid, dim3(256), 0, p.stream, g);
    }
    return hipGetLastError();
}

hipError_t gemm1_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    SplitArgs g = split_args(p, n_fields, rho, nullptr, rho_dtype);
    dim3 grid(g.tiles_e + g.tiles_o, (g.rows + TB - 1) / TB, p.splitk);
    if (p.fold) hipLaunchKernelGGL((k_gemm1<true>), grid, dim3(256), 0, p.stream, g);
    else hipLaunchKernelGGL((k_gemm1<false>), grid, dim3(256), 0, p.stream, g);
    return hipGetLastError();
}

hipError_t gemm2_bf16(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    SplitArgs g = split_args(p, n_fields, nullptr, phi, phi_dtype);
    dim3 grid((g.rows + TB - 1) / TB, p.n_angp / TB);
    if (phi_dtype == MPG_F64) {
        if (p.fold) hipLaunchKernelGGL((k_gemm2<double, true>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm2<double, false>), grid, dim3(256), 0, p.stream, g);
    } else {
        if (p.fold) hipLaunchKernelGGL((k_gemm2<float, true>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm2<float, false>), grid, dim3(256), 0, p.stream, g);
    }
    return hipGetLastError();
}

hipError_t batch_split_input_bf16(const SplitArgs *args, int f, size_t rows_x_cols8, int io_dtype, hipStream_t s) {
    dim3 grid((unsigned)((rows_x_cols8 + 255) / 256));
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_fold_split<double>), grid, dim3(256), 0, s, args, f);
    else
        hipLaunchKernelGGL((k_batch_fold_split<float>), grid, dim3(256), 0, s, args, f);
    return hipGetLastError();
}

hipError_t batch_gemm1_bf16(const SplitArgs *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                            int blocks, hipStream_t s) {
    (void)io_dtype;
    hipLaunchKernelGGL(k_batch_gemm1, dim3(blocks), dim3(256), 0, s, args, items, n_items, head);
    return hipGetLastError();
}

hipError_t batch_gemm2_bf16(const SplitArgs *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                            int blocks, hipStream_t s) {
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_gemm2<double>), dim3(blocks), dim3(256), 0, s, args, items, n_items, head);
    else
        hipLaunchKernelGGL((k_batch_gemm2<float>), dim3(blocks), dim3(256), 0, s, args, items, n_items, head);
    return hipGetLastError();
}

}  // namespace mpg
