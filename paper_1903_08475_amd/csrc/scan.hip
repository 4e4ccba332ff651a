// Radial sums of Eq. M_C (Sec. 4.3 step 4) as two first-order linear
// recurrences per moment column, evaluated in FP64:
//   y_n = a_n y_{n-1} + b_n B_n          (inner mass, = (r_n^+)^{-(l+1)} sum_{i<=n} R_in,i B_i)
//   z_n = c_n z_{n+1} + e_n B_{n+1}      (outer mass, = (r_n^+)^l sum_{i>n} R_out,i B_i)
//   M_n = y_n + z_n
// All coefficients are ratios <= 1 (no r^l, r^-(l+1) overflow at any radius).
//
// A block owns 64 consecutive columns (one lane each) and splits the shells
// into T chunks (one wave-row of threads each).  Every chunk first composes
// its affine maps (product of a or c, local sums), the chunk carries are
// chained through LDS, and a second sweep writes M.  The first sweep also
// reduces the split-K partial sums of the moments in a fixed order, so the
// result does not depend on scheduling.
#include "mpg_internal.h"

namespace mpg {
namespace {

constexpr int kLanes = 64, kMaxChunks = 16;
constexpr int kGroup = 4;  // shells per group of loads in each sweep

// element (row, col) of piece 0 of the tile-slab split copy of M
__device__ inline size_t split_offset(int row, int col, int ks2) {
    const size_t blk = (size_t)(row / kSplitTile) * ks2 + col / kSlabK;
    return blk * 3 * kBlk + blk_pos(row % kSplitTile, col % kSlabK);
}

// where moment q of shell n of (single-patch) field f goes in the split
// copy: row (f, n), column q; for the per-patch method field f is patch
// f % pp of field f / pp, and its moments go to row (f / pp, n), column
// (f % pp, q), the expansion's K
__device__ inline size_t split_offset_of(int f, int n, int q, int n_r, int np, int pp, int ks2) {
    if (pp) return split_offset((f / pp) * n_r + n, (f % pp) * np + q, ks2);
    return split_offset(f * n_r + n, q, ks2);
}

__device__ inline double reduce_parts(const double *Bpart, size_t stride, int splitk, size_t idx) {
    double s = 0.0;
    for (int k = 0; k < splitk; ++k) s += Bpart[k * stride + idx];
    return s;
}

// One block of 64 columns.  Threads with lane >= the column count, and
// chunks past the last shell, hold identity maps and write nothing.  Each
// sweep takes kGroup shells at a time: the loads of a group are issued
// together before the recurrence consumes them, so a wave waits for one
// memory latency per group rather than per shell (the loads of a short
// last group repeat an in-range shell; their values are not used).
__device__ __forceinline__ void scan_block(const ScanArgs &g, int bx) {
    const double *__restrict__ Bpart = g.Bpart;
    const int splitk = g.splitk, n_fields = g.n_fields, n_r = g.n_r, np = g.np, L = g.L;
    const int *__restrict__ col_l = g.col_l;
    const double *__restrict__ coef = g.coef;
    double *__restrict__ Bred = g.Bred;
    double *__restrict__ M = g.M;
    bf16 *__restrict__ Ms = g.Ms;
    __shared__ double sA[kMaxChunks][kLanes], sY[kMaxChunks][kLanes];
    __shared__ double sC[kMaxChunks][kLanes], sZ[kMaxChunks][kLanes];
    const int lane = threadIdx.x, ch = threadIdx.y, T = blockDim.y;
    const int cidx = bx * kLanes + lane;
    const bool active = cidx < n_fields * np;
    const int f = active ? cidx / np : 0, q = active ? cidx - f * np : 0;
    const int l = active ? col_l[q] : -1;
    const int len = (n_r + T - 1) / T;
    // a chunk is one wave (64 lanes): its shell range is wave-uniform
    const int lo = __builtin_amdgcn_readfirstlane(min(n_r, ch * len));
    const int hi = __builtin_amdgcn_readfirstlane(min(n_r, lo + len));
    const size_t stride = (size_t)n_fields * n_r * np;
    const size_t base = (size_t)f * n_r * np + q;
    const int cl = l < 0 ? 0 : l;
    const double *cf = coef + 4 * (size_t)cl;
    const size_t cstep = 4 * (size_t)(L + 1);

    // first sweep: reduce the partial sums, compose the chunk's maps; the
    // outer sum over shells n > lo uses the coefficients (c, e) of shell n - 1
    double A = 1.0, y = 0.0, P = 1.0, zl = 0.0;
    if (l >= 0) {
        double pc = 0.0, pe = 0.0;
        for (int n0 = lo; n0 < hi; n0 += kGroup) {
            const int cnt = min(kGroup, hi - n0);
            double Bv[kGroup], c[kGroup][4];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                Bv[u] = 0.0;
                const double *cn = cf + min(n0 + u, hi - 1) * cstep;
#pragma unroll
                for (int k = 0; k < 4; ++k) c[u][k] = cn[k];
            }
            for (int k = 0; k < splitk; ++k)
#pragma unroll
                for (int u = 0; u < kGroup; ++u)
                    Bv[u] += Bpart[k * stride + base + (size_t)min(n0 + u, hi - 1) * np];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                if (u >= cnt) break;
                const int n = n0 + u;
                Bred[base + (size_t)n * np] = Bv[u];
                y = c[u][0] * y + c[u][1] * Bv[u];
                A *= c[u][0];
                if (n > lo) {
                    zl += P * pe * Bv[u];
                    P *= pc;
                }
                pc = c[u][2];
                pe = c[u][3];
            }
        }
        if (hi > lo && hi < n_r) {
            double Bh = reduce_parts(Bpart, stride, splitk, base + (size_t)hi * np);
            zl += P * pe * Bh;
            P *= pc;
        }
    }
    sA[ch][lane] = A;
    sY[ch][lane] = y;
    sC[ch][lane] = P;
    sZ[ch][lane] = zl;
    __syncthreads();
    if (!active) return;  // after the barrier: every thread must reach it
    double Yin = 0.0, Zin = 0.0;
    for (int c = 0; c < ch; ++c) Yin = sA[c][lane] * Yin + sY[c][lane];
    for (int c = T - 1; c > ch; --c) Zin = sZ[c][lane] + sC[c][lane] * Zin;
    if (l < 0) {
        for (int n = lo; n < hi; ++n) {
            M[base + (size_t)n * np] = 0.0;
            Bred[base + (size_t)n * np] = 0.0;
            if (Ms) {
                bf16 *o = Ms + split_offset_of(f, n, q, n_r, np, g.pp, g.ks2);
                o[0] = o[kBlk] = o[2 * kBlk] = (bf16)0.0f;
            }
        }
        return;
    }
    // inner sums, upwards
    y = Yin;
    for (int n0 = lo; n0 < hi; n0 += kGroup) {
        const int cnt = min(kGroup, hi - n0);
        double Bv[kGroup], a[kGroup], b[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int n = min(n0 + u, hi - 1);
            const double *cn = cf + n * cstep;
            a[u] = cn[0];
            b[u] = cn[1];
            Bv[u] = Bred[base + (size_t)n * np];
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            if (u >= cnt) break;
            y = a[u] * y + b[u] * Bv[u];
            M[base + (size_t)(n0 + u) * np] = y;
        }
    }
    // outer sums, downwards; M = inner + outer
    double z = Zin;
    for (int n1 = hi; n1 > lo; n1 -= kGroup) {
        const int cnt = min(kGroup, n1 - lo);
        double Bv[kGroup], Mv[kGroup], cc[kGroup], e[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int n = max(n1 - 1 - u, lo);
            const double *cn = cf + n * cstep;
            cc[u] = cn[2];
            e[u] = cn[3];
            const double b1 = Bred[base + (size_t)min(n + 1, n_r - 1) * np];
            Bv[u] = n + 1 < n_r ? b1 : 0.0;
            Mv[u] = M[base + (size_t)n * np];
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            if (u >= cnt) break;
            const int n = n1 - 1 - u;
            z = cc[u] * z + e[u] * Bv[u];
            double m = Mv[u] + z;
            M[base + (size_t)n * np] = m;
            if (Ms) {
                // three-piece bf16 copy for the split contraction
                bf16 h = (bf16)(float)m;
                double r = m - (double)(float)h;
                bf16 md = (bf16)(float)r;
                double r2 = r - (double)(float)md;
                bf16 *o = Ms + split_offset_of(f, n, q, n_r, np, g.pp, g.ks2);
                o[0] = h;
                o[kBlk] = md;
                o[2 * kBlk] = (bf16)(float)r2;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_scan(ScanArgs g) {
    scan_block(g, blockIdx.x);
}

// persistent batch version: items (field, column block) from a queue
__global__ __launch_bounds__(1024) void k_batch_scan(const ScanArgs *__restrict__ args,
                                                     const BatchItem *__restrict__ items, int n_items, int *head) {
    __shared__ int slot;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (;;) {
        if (tid == 0) slot = atomicAdd(head, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(slot);
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem w = items[it];
        const ScanArgs g = args[w.f];
        scan_block(g, w.a);
        __syncthreads();
    }
}

// one thread per (row, permuted column), flat over rows * np
__global__ void k_unpermute(const double *src, int rows, int np, int n_lm, const int *col_src, double *dst) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)rows * np) return;
    const size_t row = t / np;
    const int q = (int)(t - row * np);
    const int s = col_src[q];
    if (s >= 0) dst[row * n_lm + s] = src[t];
}

}  // namespace

ScanArgs scan_args(const Plan &p, int n_fields, bool split_out) {
    ScanArgs g;
    g.Bpart = p.Bpart;
    g.splitk = p.splitk;
    g.n_fields = n_fields;
    g.n_r = p.n_r;
    g.np = p.np;
    g.L = p.lmax;
    g.col_l = p.col_l;
    g.coef = p.coef;
    g.Bred = p.Bred;
    g.M = p.M;
    g.Ms = split_out ? p.Ms : nullptr;
    g.ks2 = p.kq() / kSlabK;
    g.pp = p.per_patch ? p.n_patches : 0;
    g.col_blocks = (n_fields * p.np + kLanes - 1) / kLanes;
    return g;
}

hipError_t radial_scan(const Plan &p, int n_fields, bool split_out) {
    ScanArgs g = scan_args(p, n_fields, split_out);
    int T = p.scan_chunks;
    if (T > p.n_r) T = p.n_r;
    if (T < 1) T = 1;
    if (T > kMaxChunks) T = kMaxChunks;
    hipLaunchKernelGGL(k_scan, dim3(g.col_blocks), dim3(kLanes, T), 0, p.stream, g);
    return hipGetLastError();
}

hipError_t batch_scan(const ScanArgs *args, const BatchItem *items, int n_items, int *head, int blocks,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_batch_scan, dim3(blocks), dim3(kLanes, kMaxChunks), 0, s, args, items, n_items, head);
    return hipGetLastError();
}

hipError_t unpermute(const Plan &p, int n_fields, const double *src, double *dst) {
    const size_t n = (size_t)n_fields * p.n_r * p.np;
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_unpermute, grid, dim3(256), 0, p.stream, src, n_fields * p.n_r, p.np, p.n_lm, p.col_src, dst);
    return hipGetLastError();
}

}  // namespace mpg
