// Split-BF16 MFMA contractions of the solve (Sec. 4.3 steps 2 and 5).
//
// Each FP64 (or FP32) operand x is written as x = h + m + l, with h, m, l
// the round-to-nearest bf16 of the successive residuals (24 significant
// bits).  A product a*b is formed from the six partial products whose
// combined weight is at least 2^-18 of the leading one:
//   ah*bh + ah*bm + am*bh + ah*bl + am*bm + al*bh
// on v_mfma_f32_32x32x16_bf16 (bf16 products are exact in FP32).  The FP32
// accumulators are flushed into FP64 registers every `flush` K steps, so
// no FP32 sum runs over more than flush*32 terms (GEMM1; GEMM2's K is the
// moment count, short enough for FP32 sums).
//
// GEMM1 (moments, Eq. B_CS) folds and splits rho in its tile loader:
// A = rho_Yin +- rho_Yang (U_Yang = (-1)^m U_Yin, Sec. 4.2), converted once
// per element to three bf16 pieces in LDS; U comes pre-split from the plan.
// GEMM2 (expansion, Eq. gravpotmult) reads M pre-split by the radial scan
// and Q pre-split by the plan, sums even- and odd-m columns separately and
// writes Phi_Yin = E + O, Phi_Yang = E - O.  Its K loop runs from the
// highest degree down to l = 0, so the dominant low-degree terms are added
// to the smallest partial sums last.
//
// Tiles: 128x128 per block of 256 threads (2x2 waves of 64x64 = 2x2 MFMA
// blocks of 32x32), K slabs of 32, next slab prefetched into registers
// while the current one is multiplied from LDS.
#include "mpg_internal.h"

namespace mpg {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int TB = 128, TK = 32, LDK = TK + 8;

struct Pieces {
    bf16 h[TB][LDK];
    bf16 m[TB][LDK];
    bf16 l[TB][LDK];
};

// C/D layout of v_mfma_f32_32x32x16_bf16 (measured): register r of lane l
// holds D[8(r/4) + 4(l/32) + r%4][l%32]; A rows are lane%32 with K elements
// 8(l/32)..+7, B columns lane%32 with the same K elements.
__device__ inline int d_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

__device__ inline void split3(double v, bf16 &h, bf16 &m, bf16 &l) {
    h = (bf16)(float)v;
    double r = v - (double)(float)h;
    m = (bf16)(float)r;
    double r2 = r - (double)(float)m;
    l = (bf16)(float)r2;
}

template <typename T>
__device__ inline double ldd(const T *p) { return (double)*p; }

// the six partial products of one 32x32x16 step into acc
__device__ inline void mma6(v16f &acc, const v8bf &ah, const v8bf &am, const v8bf &al, const v8bf &bh,
                            const v8bf &bm, const v8bf &bl) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
}

// one 32-deep slab from LDS for a wave's 64x64 tile
__device__ inline void mma_slab(const Pieces &A, const Pieces &B, int wm, int wn, int lane, v16f (&acc)[2][2]) {
    const int lr = lane & 31, lk = 8 * (lane >> 5);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
        v8bf ah[2], am[2], al[2], bh[2], bm[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = *(const v8bf *)&A.h[wm + 32 * i + lr][ks + lk];
            am[i] = *(const v8bf *)&A.m[wm + 32 * i + lr][ks + lk];
            al[i] = *(const v8bf *)&A.l[wm + 32 * i + lr][ks + lk];
            bh[i] = *(const v8bf *)&B.h[wn + 32 * i + lr][ks + lk];
            bm[i] = *(const v8bf *)&B.m[wn + 32 * i + lr][ks + lk];
            bl[i] = *(const v8bf *)&B.l[wn + 32 * i + lr][ks + lk];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) mma6(acc[i][j], ah[i], am[i], al[i], bh[j], bm[j], bl[j]);
    }
}

struct Raw16 {
    uint4 v[2];  // 16 bf16
};

__device__ inline void load_pieces(Raw16 (&r)[3], const bf16 *h, const bf16 *m, const bf16 *l, size_t off) {
    r[0].v[0] = *(const uint4 *)(h + off);
    r[0].v[1] = *(const uint4 *)(h + off + 8);
    r[1].v[0] = *(const uint4 *)(m + off);
    r[1].v[1] = *(const uint4 *)(m + off + 8);
    r[2].v[0] = *(const uint4 *)(l + off);
    r[2].v[1] = *(const uint4 *)(l + off + 8);
}

__device__ inline void store_pieces(Pieces &S, const Raw16 (&r)[3], int row, int k) {
    *(uint4 *)&S.h[row][k] = r[0].v[0];
    *(uint4 *)&S.h[row][k + 8] = r[0].v[1];
    *(uint4 *)&S.m[row][k] = r[1].v[0];
    *(uint4 *)&S.m[row][k + 8] = r[1].v[1];
    *(uint4 *)&S.l[row][k] = r[2].v[0];
    *(uint4 *)&S.l[row][k + 8] = r[2].v[1];
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
// GEMM1: grid x = column tile (even-m tiles, then odd-m tiles), y = row tile,
// z = K split.  Bpart[z][row][col] in FP64.
template <typename T, bool FOLD>
__global__ __launch_bounds__(256) void k_gemm1(const T *__restrict__ rho, int rows, int n_r, int n_ang,
                                               const bf16 *__restrict__ Uh, const bf16 *__restrict__ Um,
                                               const bf16 *__restrict__ Ul, int n_angp, int np, int ne_p,
                                               int tiles_e, int kchunk, int flush, double *__restrict__ Bpart) {
    __shared__ Pieces As, Bs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int tn = blockIdx.x;
    const bool odd = FOLD && tn >= tiles_e;
    const int c0 = odd ? ne_p + (tn - tiles_e) * TB : tn * TB;
    const int cend = odd ? np : (FOLD ? ne_p : np);
    const int m0 = blockIdx.y * TB;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(n_angp, kbeg + kchunk);

    // loader: thread t covers row t/2 and 16 K values from 16*(t%2)
    const int lr = t >> 1, lk = (t & 1) * 16;
    const int row = m0 + lr;
    const bool row_ok = row < rows;
    const int f = row_ok ? row / n_r : 0, i = row_ok ? row - f * n_r : 0;
    const size_t fld = (size_t)(FOLD ? 2 : 1) * n_r * n_ang;
    const T *r0 = rho + f * fld + (size_t)i * n_ang;
    const T *r1 = r0 + (size_t)n_r * n_ang;
    const size_t uoff = (size_t)(c0 + lr) * n_angp;

    v16f acc[2][2];
    double acc64[2][2][16];
    zero(acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc64[a][b][r] = 0.0;

    double av[16];
    Raw16 bu[3];
    auto load = [&](int k) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            double v = 0.0;
            if (row_ok && k + q < n_ang) {
                v = ldd(r0 + k + q);
                if (FOLD) {
                    double w = ldd(r1 + k + q);
                    v = odd ? v - w : v + w;
                }
            }
            av[q] = v;
        }
        load_pieces(bu, Uh, Um, Ul, uoff + k);
    };
    if (kbeg < kend) load(kbeg + lk);
    int step = 0;
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) split3(av[q], As.h[lr][lk + q], As.m[lr][lk + q], As.l[lr][lk + q]);
        store_pieces(Bs, bu, lr, lk);
        __syncthreads();
        if (k0 + TK < kend) load(k0 + TK + lk);
        mma_slab(As, Bs, wm, wn, lane, acc);
        if (++step == flush) {
            step = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc64[a][b][r] += (double)acc[a][b][r];
            zero(acc);
        }
    }
    double *out = Bpart + (size_t)blockIdx.z * rows * np;
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

// ---------------------------------------------------------------------------
// GEMM2: grid x = row tile, y = angular tile.
template <typename T, bool FOLD>
__global__ __launch_bounds__(256) void k_gemm2(const bf16 *__restrict__ Mh, const bf16 *__restrict__ Mm,
                                               const bf16 *__restrict__ Ml, int rows, int np, int ne_p,
                                               const bf16 *__restrict__ Qh, const bf16 *__restrict__ Qm,
                                               const bf16 *__restrict__ Ql, int n_ang, int n_r,
                                               T *__restrict__ phi) {
    __shared__ Pieces As, Bs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int m0 = blockIdx.x * TB, n0 = blockIdx.y * TB;
    const int lr = t >> 1, lk = (t & 1) * 16;
    const bool row_ok = m0 + lr < rows;
    const size_t aoff = (size_t)(row_ok ? m0 + lr : 0) * np;
    const size_t boff = (size_t)(n0 + lr) * np;

    v16f acc[2][2][2];
    zero(acc[0]);
    zero(acc[1]);
    const int nblk = FOLD ? 2 : 1;
#pragma unroll
    for (int blk = 0; blk < nblk; ++blk) {
        const int kb = blk ? ne_p : 0, ke = (FOLD && !blk) ? ne_p : np;
        Raw16 ra[3], rb[3];
        // K slabs from the top of the block down to kb (columns are ordered
        // by degree, so the largest terms are added last)
        const int nsl = (ke - kb + TK - 1) / TK;
        auto load = [&](int s) {
            int k = kb + (nsl - 1 - s) * TK + lk;
            if (row_ok) {
                load_pieces(ra, Mh, Mm, Ml, aoff + k);
            } else {
#pragma unroll
                for (int p = 0; p < 3; ++p) ra[p].v[0] = ra[p].v[1] = make_uint4(0, 0, 0, 0);
            }
            load_pieces(rb, Qh, Qm, Ql, boff + k);
        };
        if (nsl > 0) load(0);
        for (int s = 0; s < nsl; ++s) {
            __syncthreads();
            store_pieces(As, ra, lr, lk);
            store_pieces(Bs, rb, lr, lk);
            __syncthreads();
            if (s + 1 < nsl) load(s + 1);
            mma_slab(As, Bs, wm, wn, lane, acc[blk]);
        }
    }
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
                double e = (double)acc[0][a][b][r];
                if (FOLD) {
                    double od = (double)acc[1][a][b][r];
                    o[0] = (T)(e + od);
                    o[(size_t)n_r * n_ang] = (T)(e - od);
                } else {
                    o[0] = (T)e;
                }
            }
}

constexpr int kFlush1 = 16;  // GEMM1: FP32 runs of at most 512 terms

}  // namespace

hipError_t gemm1_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    const int rows = n_fields * p.n_r;
    const int te = p.fold ? (p.ne_p + TB - 1) / TB : (p.np + TB - 1) / TB;
    const int to = p.fold ? (p.no_p + TB - 1) / TB : 0;
    const int kchunk = ((p.n_angp / p.splitk + TK - 1) / TK) * TK;
    dim3 grid(te + to, (rows + TB - 1) / TB, p.splitk);
#define L1(T, F)                                                                                              \
    hipLaunchKernelGGL((k_gemm1<T, F>), grid, dim3(256), 0, p.stream, (const T *)rho, rows, p.n_r, p.n_ang,  \
                       p.Ut_hi, p.Ut_mid, p.Ut_lo, p.n_angp, p.np, p.ne_p, te, kchunk, kFlush1, p.Bpart)
    if (rho_dtype == MPG_F64) {
        if (p.fold) L1(double, true);
        else L1(double, false);
    } else {
        if (p.fold) L1(float, true);
        else L1(float, false);
    }
#undef L1
    return hipGetLastError();
}

hipError_t gemm2_bf16(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    const int rows = n_fields * p.n_r;
    dim3 grid((rows + TB - 1) / TB, p.n_angp / TB);
#define L2(T, F)                                                                                              \
    hipLaunchKernelGGL((k_gemm2<T, F>), grid, dim3(256), 0, p.stream, p.M_hi, p.M_mid, p.M_lo, rows, p.np,    \
                       p.ne_p, p.Qt_hi, p.Qt_mid, p.Qt_lo, p.n_ang, p.n_r, (T *)phi)
    if (phi_dtype == MPG_F64) {
        if (p.fold) L2(double, true);
        else L2(double, false);
    } else {
        if (p.fold) L2(float, true);
        else L2(float, false);
    }
#undef L2
    return hipGetLastError();
}

}  // namespace mpg
