// FP64 MFMA contractions of the solve (Sec. 4.3 steps 2 and 5).
//
// GEMM1 (moments, Eq. B_CS):  B[row][q] = sum_k A[row][k] U[q][k]
//   with A = rho_Yin + rho_Yang for even-m columns and rho_Yin - rho_Yang
//   for odd-m columns under the Yin/Yang fold (U_Yang = (-1)^m U_Yin,
//   Sec. 4.2).  Otherwise k runs over the cells of every patch, patch after
//   patch (k = g*n_angp + jk), and A = rho (the sum over patches of Eq. B_CS
//   is part of the contraction).  Split over K; the partial sums go to a
//   work array that the radial scan reduces in a fixed order.
// GEMM2 (expansion, Eq. gravpotmult):  Phi[row][k] = sum_q M[row][q] Q[k][q]
//   accumulated separately over even- and odd-m columns, written as
//   Phi_Yin = E + O and Phi_Yang = E - O under the fold; otherwise k runs
//   over the cells of every patch as in GEMM1.
//
// Rows are (field, shell) pairs; 256 threads (four waves) per tile on
// v_mfma_f64_16x16x4f64, with the next K slab (16 deep) loaded into
// registers while the current one is multiplied from LDS.  GEMM1 tiles are
// 128x128 (waves of 64x64: 16 MFMAs per 4-deep step); GEMM2, which keeps
// the even- and odd-m sums of its tile apart, uses 64x64 tiles (waves of
// 32x32) so that both sets of accumulators fit two waves per SIMD.
#include "mpg_internal.h"

namespace mpg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;
constexpr int T1 = kF64Tile1, T2 = kF64Tile2;  // GEMM1 / GEMM2 tile sides

// Lane layout of v_mfma_f64_16x16x4f64 on gfx950 (measured): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; result register r of lane l is
// D[l/16 + 4r][l%16].
__device__ inline int out_row(int l, int r) { return (l >> 4) + 4 * r; }
__device__ inline int out_col(int l, int r) { return l & 15; }

template <typename T>
__device__ inline double ld(const T *p) { return (double)*p; }

// one TxBK slab of a K-contiguous operand: thread t covers row
// t / (256/T), kPer consecutive K from (t % (256/T)) * kPer
template <int T>
struct Slab {
    static constexpr int kPer = T * BK / 256;  // elements per thread
    double v[kPer];
};

template <int T>
__device__ inline int slab_row(int t) { return t / (256 / T); }
template <int T>
__device__ inline int slab_k(int t) { return (t % (256 / T)) * Slab<T>::kPer; }

// LDS row pitch of a slab (doubles), chosen by measurement: 144 for the
// 128-wide tiles (rows k and k+1, read by the two halves of a wave's 64-bit
// fragment reads, fall in disjoint bank halves), 66 for the 64-wide ones
// (whose stores of four rows at once conflict less)
template <int T>
constexpr int ldp() { return T == 64 ? T + 2 : T + 16; }

template <int T>
struct Smem {
    double As[BK][ldp<T>()];
    double Bs[BK][ldp<T>()];
};

// kPer consecutive K of one row of A; k = patch*n_angp + cell (they never
// straddle a patch: n_angp is a multiple of 128), r0/r1 the row in patch 0
// and 1, pstride the distance between patches of a field
template <typename T, bool FOLD, int TS>
__device__ inline void load_rho(Slab<TS> &s, const T *r0, const T *r1, int k, int n_ang, int n_angp, size_t pstride,
                                bool row_ok, bool odd) {
    if (!FOLD) {
        const int gp = k / n_angp;
        r0 += gp * pstride;
        k -= gp * n_angp;
    }
    if (sizeof(T) == 4 && (n_ang & 3) == 0) {
        // FP32 rows whose length is a multiple of 4: groups of four K (16-byte
        // aligned; k is a multiple of 4) lie wholly inside or outside the row
#pragma unroll
        for (int q = 0; q < Slab<TS>::kPer; q += 4) {
            f32x4 a = {0.f, 0.f, 0.f, 0.f}, b = a;
            if (row_ok && k + q < n_ang) {
                a = *(const f32x4 *)(r0 + k + q);
                if (FOLD) b = *(const f32x4 *)(r1 + k + q);
            }
            const double av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) s.v[q + u] = FOLD ? (odd ? av[u] - bv[u] : av[u] + bv[u]) : av[u];
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < Slab<TS>::kPer; ++q) {
        double a = 0.0;
        if (row_ok && k + q < n_ang) {
            a = ld(r0 + k + q);
            if (FOLD) {
                double b = ld(r1 + k + q);
                a = odd ? a - b : a + b;
            }
        }
        s.v[q] = a;
    }
}

template <int TS>
__device__ inline void load_rowk(Slab<TS> &s, const double *row, int k, bool ok) {
#pragma unroll
    for (int q = 0; q < Slab<TS>::kPer; ++q) s.v[q] = ok ? row[k + q] : 0.0;
}

template <int TS>
__device__ inline void store_slab(double (*S)[ldp<TS>()], const Slab<TS> &s, int lr, int lk) {
#pragma unroll
    for (int q = 0; q < Slab<TS>::kPer; ++q) S[lk + q][lr] = s.v[q];
}

// a wave's WT x WT tiles of 16x16 (TS/2 x TS/2 per wave, four waves)
template <int TS, int WT = TS / 32>
__device__ inline void mma_slab(const double (*As)[ldp<TS>()], const double (*Bs)[ldp<TS>()], int wm, int wn,
                                int lane, v4d (&acc)[WT][WT]) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
        double a[WT], b[WT];
#pragma unroll
        for (int i = 0; i < WT; ++i) a[i] = As[kk * 4 + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < WT; ++j) b[j] = Bs[kk * 4 + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}


// One output tile of GEMM1, TS x TS (128, or 64 for small problems; each
// output takes the same products in the same order in both): column tile
// tn (even-m tiles first, then odd-m tiles), row tile tm, K split tz.
template <typename T, bool FOLD, int TS>
__device__ __forceinline__ void gemm1_tile(const F64Args &g, int tn, int tm, int tz, Smem<TS> &sm) {
    constexpr int BM = TS, BN = TS, WT = TS / 32;
    const T *rho = (const T *)g.rho;
    const int rows = g.rows, n_r = g.n_r, n_ang = g.n_ang, n_angp = g.n_angp, np = g.np, ne_p = g.ne_p;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
    const bool odd = FOLD && tn >= g.tiles_e;
    const int c0 = odd ? ne_p + (tn - g.tiles_e) * BN : tn * BN;
    const int cend = odd ? np : (FOLD ? ne_p : np);
    const int m0 = tm * BM;
    const int kbeg = tz * g.kchunk;
    const int kend = min(g.kang, kbeg + g.kchunk);

    const int lr = slab_row<TS>(t), lk = slab_k<TS>(t);
    const int row = m0 + lr;
    const bool row_ok = row < rows;
    const int f = row_ok ? row / n_r : 0, i = row_ok ? row - f * n_r : 0;
    const size_t pstride = (size_t)n_r * n_ang, fld = (size_t)g.n_patches * pstride;
    const T *r0 = rho + f * fld + (size_t)i * n_ang;
    const T *r1 = r0 + pstride;
    const double *urow = g.Ut + (size_t)(c0 + lr) * g.kang;

    v4d acc[WT][WT];
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
        for (int b = 0; b < WT; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

    Slab<TS> sa, sb;
    if (kbeg < kend) {
        load_rho<T, FOLD, TS>(sa, r0, r1, kbeg + lk, n_ang, n_angp, pstride, row_ok, odd);
        load_rowk(sb, urow, kbeg + lk, true);
    }
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        store_slab(sm.As, sa, lr, lk);
        store_slab(sm.Bs, sb, lr, lk);
        __syncthreads();
        if (k0 + BK < kend) {
            load_rho<T, FOLD, TS>(sa, r0, r1, k0 + BK + lk, n_ang, n_angp, pstride, row_ok, odd);
            load_rowk(sb, urow, k0 + BK + lk, true);
        }
        mma_slab<TS>(sm.As, sm.Bs, wm, wn, lane, acc);
    }
    __syncthreads();
    double *out = g.Bpart + (size_t)tz * rows * np;
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
        for (int b = 0; b < WT; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int rr = m0 + wm + a * 16 + out_row(lane, r);
                int cc = c0 + wn + b * 16 + out_col(lane, r);
                if (rr < rows && cc < cend) out[(size_t)rr * np + cc] = acc[a][b][r];
            }
}

// One output tile of GEMM2 (row tile tm, angular tile tn).
template <typename T, bool FOLD>
__device__ __forceinline__ void gemm2_tile(const F64Args &g, int tm, int tn, Smem<T2> &sm) {
    constexpr int BM = T2, BN = T2, WT = T2 / 32;
    T *phi = (T *)g.phi;
    const int rows = g.rows, np = g.np, ne_p = g.ne_p, n_ang = g.n_ang, n_r = g.n_r;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
    const int m0 = tm * BM, n0 = tn * BN;
    const int lr = slab_row<T2>(t), lk = slab_k<T2>(t);
    const bool row_ok = m0 + lr < rows;
    const int arw = row_ok ? m0 + lr : 0;
    const double *brow = g.Qt + (size_t)(n0 + lr) * g.kq;

    v4d acc[2][WT][WT];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int a = 0; a < WT; ++a)
#pragma unroll
            for (int b = 0; b < WT; ++b) acc[p][a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

    // one K block [kb, ke) of A row `arow` against Q row `brow`, into acc[blk]
    auto kblock = [&](const double *arow, const double *bq, int kb, int ke, v4d(&ac)[WT][WT]) {
        Slab<T2> sa, sb;
        if (kb < ke) {
            load_rowk(sa, arow, kb + lk, row_ok);
            load_rowk(sb, bq, kb + lk, true);
        }
        for (int k0 = kb; k0 < ke; k0 += BK) {
            __syncthreads();
            store_slab(sm.As, sa, lr, lk);
            store_slab(sm.Bs, sb, lr, lk);
            __syncthreads();
            if (k0 + BK < ke) {
                load_rowk(sa, arow, k0 + BK + lk, row_ok);
                load_rowk(sb, bq, k0 + BK + lk, true);
            }
            mma_slab<T2>(sm.As, sm.Bs, wm, wn, lane, ac);
        }
    };
    if (FOLD) {
        const double *arow = g.M + (size_t)arw * np;
        kblock(arow, brow, 0, ne_p, acc[0]);
        kblock(arow, brow, ne_p, np, acc[1]);
    } else if (g.nq == 1) {
        kblock(g.M + (size_t)arw * np, brow, 0, np, acc[0]);
    } else {
        // per-patch method: K runs over the moment sets of every patch, set gq
        // at row (field, gq, shell) of M
        const int f = arw / n_r, i = arw - f * n_r;
        for (int gq = 0; gq < g.nq; ++gq)
            kblock(g.M + ((size_t)(f * g.nq + gq) * n_r + i) * np, brow + (size_t)gq * np, 0, np, acc[0]);
    }
    __syncthreads();
    const size_t pstride = (size_t)n_r * n_ang, fld = (size_t)g.n_patches * pstride;
    const int n_angp = g.n_angp;
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
        for (int b = 0; b < WT; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int rr = m0 + wm + a * 16 + out_row(lane, r);
                int kk = n0 + wn + b * 16 + out_col(lane, r);
                const int gp = kk / n_angp, jk = kk - gp * n_angp;
                if (rr >= rows || jk >= n_ang) continue;
                int f = rr / n_r, i = rr - f * n_r;
                T *o = phi + f * fld + gp * pstride + (size_t)i * n_ang + jk;
                double e = acc[0][a][b][r];
                if (FOLD) {
                    double od = acc[1][a][b][r];
                    o[0] = (T)(e + od);
                    o[pstride] = (T)(e - od);
                } else {
                    o[0] = (T)e;
                }
            }
}

// grid: x = column tile (E tiles then O tiles), y = row tile, z = K split
template <typename T, bool FOLD, int TS>
__global__ __launch_bounds__(256) void k_gemm1(F64Args g) {
    __shared__ Smem<TS> sm;
    gemm1_tile<T, FOLD, TS>(g, blockIdx.x, blockIdx.y, blockIdx.z, sm);
}

// grid: x = row tile, y = angular tile
template <typename T, bool FOLD>
__global__ __launch_bounds__(256) void k_gemm2(F64Args g) {
    __shared__ Smem<T2> sm;
    gemm2_tile<T, FOLD>(g, blockIdx.x, blockIdx.y, sm);
}

// Persistent batch kernels (see the split-BF16 ones): items from a queue
// through an atomic head until it is empty; no item waits on another.
__device__ __forceinline__ int next_item(int *head, int *slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(head, 1);
    __syncthreads();
    int it = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();
    return it;
}

template <typename T>
__global__ __launch_bounds__(256) void k_batch_gemm1(const F64Args *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head) {
    __shared__ Smem<T1> sm;
    __shared__ int slot;
    static_assert(sizeof(Smem<64>) <= sizeof(Smem<T1>), "both tile sides fit the shared buffers");
    Smem<64> &sm64 = *reinterpret_cast<Smem<64> *>(&sm);
    for (;;) {
        const int it = next_item(head, &slot);
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const F64Args g = args[w.f];
        if (g.t1 == 64) {
            if (g.fold) gemm1_tile<T, true, 64>(g, w.a, w.b, w.c, sm64);
            else gemm1_tile<T, false, 64>(g, w.a, w.b, w.c, sm64);
        } else {
            if (g.fold) gemm1_tile<T, true, T1>(g, w.a, w.b, w.c, sm);
            else gemm1_tile<T, false, T1>(g, w.a, w.b, w.c, sm);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_batch_gemm2(const F64Args *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head,
                                                     BatchTrack track) {
    __shared__ Smem<T2> sm;
    __shared__ int slot;
    for (int prev = -1;;) {
        const int it = next_item_tracked(head, &slot, track, prev);
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const F64Args g = args[w.f];
        if (g.fold) gemm2_tile<T, true>(g, w.a, w.b, sm);
        else gemm2_tile<T, false>(g, w.a, w.b, sm);
        prev = w.f;
    }
}

}  // namespace

F64Args f64_args(const Plan &p, int n_fields, const void *rho, void *phi, int io_dtype, bool expansion) {
    F64Args g;
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
    // GEMM1 tiles: 128 x 128, or 64 x 64 (the plan's second moment shape)
    const int t1 = p.gemm1_rows == 2 ? 64 : T1;
    g.t1 = t1;
    g.tiles_e = p.fold ? (p.ne_p + t1 - 1) / t1 : (p.np + t1 - 1) / t1;
    g.tiles_o = p.fold ? (p.no_p + t1 - 1) / t1 : 0;
    g.kchunk = ksplit_chunk(p.kang(), p.splitk, BK);
    g.splitk = p.splitk;
    g.Ut = p.Ut;
    g.Qt = p.Qt;
    g.M = p.M;
    g.Bpart = p.Bpart;
    return g;
}

template <int TS>
static void launch_gemm1(const Plan &p, const F64Args &g, dim3 grid, int rho_dtype) {
    if (rho_dtype == MPG_F64) {
        if (p.fold) hipLaunchKernelGGL((k_gemm1<double, true, TS>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm1<double, false, TS>), grid, dim3(256), 0, p.stream, g);
    } else {
        if (p.fold) hipLaunchKernelGGL((k_gemm1<float, true, TS>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm1<float, false, TS>), grid, dim3(256), 0, p.stream, g);
    }
}

hipError_t gemm1_f64(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    F64Args g = f64_args(p, n_fields, rho, nullptr, rho_dtype);
    dim3 grid(g.tiles_e + g.tiles_o, (g.rows + g.t1 - 1) / g.t1, p.splitk);
    if (g.t1 == 64) launch_gemm1<64>(p, g, grid, rho_dtype);
    else launch_gemm1<T1>(p, g, grid, rho_dtype);
    return hipGetLastError();
}

hipError_t gemm2_f64(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    F64Args g = f64_args(p, n_fields, nullptr, phi, phi_dtype, true);
    dim3 grid((g.rows + T2 - 1) / T2, g.kang / T2);
    if (phi_dtype == MPG_F64) {
        if (p.fold) hipLaunchKernelGGL((k_gemm2<double, true>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm2<double, false>), grid, dim3(256), 0, p.stream, g);
    } else {
        if (p.fold) hipLaunchKernelGGL((k_gemm2<float, true>), grid, dim3(256), 0, p.stream, g);
        else hipLaunchKernelGGL((k_gemm2<float, false>), grid, dim3(256), 0, p.stream, g);
    }
    return hipGetLastError();
}

hipError_t batch_gemm1_f64(const F64Args *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                           int blocks, hipStream_t s) {
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_gemm1<double>), dim3(blocks), dim3(256), 0, s, args, items, n_items, head);
    else
        hipLaunchKernelGGL((k_batch_gemm1<float>), dim3(blocks), dim3(256), 0, s, args, items, n_items, head);
    return hipGetLastError();
}

hipError_t batch_gemm2_f64(const F64Args *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                           int blocks, BatchTrack track, hipStream_t s) {
    if (io_dtype == MPG_F64)
        hipLaunchKernelGGL((k_batch_gemm2<double>), dim3(blocks), dim3(256), 0, s, args, items, n_items, head, track);
    else
        hipLaunchKernelGGL((k_batch_gemm2<float>), dim3(blocks), dim3(256), 0, s, args, items, n_items, head, track);
    return hipGetLastError();
}

}  // namespace mpg
