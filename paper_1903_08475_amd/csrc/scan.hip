// Radial sums of Eq. M_C (Sec. 4.3 step 4) as two first-order linear
// recurrences per moment column, evaluated in FP64:
//   y_n = a_n y_{n-1} + b_n B_n          (inner mass, = (r_n^+)^{-(l+1)} sum_{i<=n} R_in,i B_i)
//   z_n = c_n z_{n+1} + e_n B_{n+1}      (outer mass, = (r_n^+)^l sum_{i>n} R_out,i B_i)
//   M_n = y_n + z_n
// All coefficients are ratios <= 1 (no r^l, r^-(l+1) overflow at any radius).
//
// A block owns 64 consecutive columns (one lane each) and splits the shells
// into T chunks (the plan's choice; one wave-row of threads each here).
// Every chunk first composes its affine maps (product of a or c, local
// sums), the chunk carries are chained through LDS, and a second sweep
// writes M.  The first sweep also reduces the split-K partial sums of the
// moments in a fixed order, so the result does not depend on scheduling.
#include "scan_core.h"

namespace mpg {
namespace {

using scan_detail::kLanes;
using scan_detail::kMaxChunks;

// one block of the scan kernel: lanes in x, shell chunks in y
__device__ __forceinline__ void scan_block(const ScanArgs &g, int bx) {
    __shared__ double sA[kMaxChunks * kLanes], sY[kMaxChunks * kLanes];
    __shared__ double sC[kMaxChunks * kLanes], sZ[kMaxChunks * kLanes];
    scan_detail::scan_block_core(g, bx, threadIdx.x, threadIdx.y, blockDim.y, sA, sY, sC, sZ);
}

__global__ __launch_bounds__(1024) void k_scan(ScanArgs g) {
    scan_block(g, blockIdx.x);
}

// persistent batch version: items (field, column block) from a queue; each
// field's scan takes its own chunk count (16 thread rows, one chunk each)
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
    int T = p.scan_chunks;
    if (T > p.n_r) T = p.n_r;
    if (T < 1) T = 1;
    if (T > kMaxChunks) T = kMaxChunks;
    g.chunks = T;
    return g;
}

hipError_t radial_scan(const Plan &p, int n_fields, bool split_out) {
    ScanArgs g = scan_args(p, n_fields, split_out);
    hipLaunchKernelGGL(k_scan, dim3(g.col_blocks), dim3(kLanes, g.chunks), 0, p.stream, g);
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
