// Radial sums of Eq. M_C (Sec. 4.3 step 4): the work of one block, shared
// by the scan kernels and the fused batch kernel.  See scan.hip.
#pragma once

#include "mpg_internal.h"

namespace mpg {
namespace scan_detail {

constexpr int kLanes = 64;
constexpr int kGroup = 4;  // shells per group of loads in each sweep
constexpr int kMaxChunks = 16;  // shell chunks per column, at most

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

// First sweep over chunk [lo, hi) of one column: reduces the partial sums
// into Bred and composes the chunk's maps (inner: y -> A y + y0; outer:
// z -> P z + zl).  The outer sum over shells n > lo uses the coefficients
// (c, e) of shell n - 1.  Each sweep takes kGroup shells at a time: the
// loads of a group are issued together before the recurrence consumes
// them, so a wave waits for one memory latency per group rather than per
// shell (the loads of a short last group repeat an in-range shell; their
// values are not used).
struct ChunkMap {
    double A, y, P, zl;
};

template <bool NT>
__device__ __forceinline__ ChunkMap compose_chunk(const ScanArgs &g, size_t base, const double *cf, size_t cstep,
                                                  int lo, int hi) {
    const double *__restrict__ Bpart = g.Bpart;
    const int splitk = g.splitk, n_r = g.n_r, np = g.np;
    const size_t stride = (size_t)g.n_fields * n_r * np;
    double *__restrict__ Bred = g.Bred;
    ChunkMap m{1.0, 0.0, 1.0, 0.0};
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
            for (int u = 0; u < kGroup; ++u) Bv[u] += Bpart[k * stride + base + (size_t)min(n0 + u, hi - 1) * np];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            if (u >= cnt) break;
            const int n = n0 + u;
            store<NT>(Bred + base + (size_t)n * np, Bv[u]);
            m.y = c[u][0] * m.y + c[u][1] * Bv[u];
            m.A *= c[u][0];
            if (n > lo) {
                m.zl += m.P * pe * Bv[u];
                m.P *= pc;
            }
            pc = c[u][2];
            pe = c[u][3];
        }
    }
    if (hi > lo && hi < n_r) {
        const double Bh = reduce_parts(Bpart, stride, splitk, base + (size_t)hi * np);
        m.zl += m.P * pe * Bh;
        m.P *= pc;
    }
    return m;
}

// Second sweep over chunk [lo, hi) of one column, entered with the inner
// sum of the shells below the chunk (Yin) and the outer sum of the shells
// above it (Zin): writes M (and its split copy).
template <bool NT>
__device__ __forceinline__ void finish_chunk(const ScanArgs &g, size_t base, const double *cf, size_t cstep, int f,
                                             int q, int lo, int hi, double Yin, double Zin) {
    const int n_r = g.n_r, np = g.np;
    const double *__restrict__ Bred = g.Bred;
    double *__restrict__ M = g.M;
    bf16 *__restrict__ Ms = g.Ms;
    // inner sums, upwards
    double y = Yin;
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
            store<NT>(M + base + (size_t)n * np, m);
            if (Ms) {
                // three-piece bf16 copy for the split contraction
                bf16 h = (bf16)(float)m;
                double r = m - (double)(float)h;
                bf16 md = (bf16)(float)r;
                double r2 = r - (double)(float)md;
                bf16 *o = Ms + split_offset_of(f, n, q, n_r, np, g.pp, g.ks2);
                store<NT>(o, h);
                store<NT>(o + kBlk, md);
                store<NT>(o + 2 * kBlk, (bf16)(float)r2);
            }
        }
    }
}

// One block of 64 columns, its shells in g.chunks chunks of equal length:
// lane (0..63) is the thread's column, and thread row `row` (0..W-1, a wave
// of lanes each) takes chunks row, row + W, ...; the block's threads must
// all call it (it holds one workgroup barrier).  Every chunk first composes
// its affine maps, the chunk carries are chained through LDS, and a second
// sweep writes M; the result depends on g.chunks only, not on W.  sA, sY,
// sC, sZ: g.chunks x 64 doubles of LDS each.  Threads with lane >= the
// column count, and chunks past the last shell, hold identity maps and
// write nothing.
template <bool NT = false>
__device__ __forceinline__ void scan_block_core(const ScanArgs &g, int bx, int lane, int row, int W, double *sA,
                                                double *sY, double *sC, double *sZ) {
    const int n_r = g.n_r, np = g.np, L = g.L, T = g.chunks;
    const int cidx = bx * kLanes + lane;
    const bool active = cidx < g.n_fields * np;
    const int f = active ? cidx / np : 0, q = active ? cidx - f * np : 0;
    const int l = active ? g.col_l[q] : -1;
    const int len = (n_r + T - 1) / T;
    const size_t base = (size_t)f * n_r * np + q;
    const int cl = l < 0 ? 0 : l;
    const double *cf = g.coef + 4 * (size_t)cl;
    const size_t cstep = 4 * (size_t)(L + 1);

    for (int ch = row; ch < T; ch += W) {
        // a chunk is taken by one wave: its shell range is wave-uniform
        const int lo = __builtin_amdgcn_readfirstlane(min(n_r, ch * len));
        const int hi = __builtin_amdgcn_readfirstlane(min(n_r, lo + len));
        ChunkMap m{1.0, 0.0, 1.0, 0.0};
        if (l >= 0) m = compose_chunk<NT>(g, base, cf, cstep, lo, hi);
        sA[ch * kLanes + lane] = m.A;
        sY[ch * kLanes + lane] = m.y;
        sC[ch * kLanes + lane] = m.P;
        sZ[ch * kLanes + lane] = m.zl;
    }
    __syncthreads();
    if (!active) return;  // after the barrier: every thread must reach it
    for (int ch = row; ch < T; ch += W) {
        const int lo = __builtin_amdgcn_readfirstlane(min(n_r, ch * len));
        const int hi = __builtin_amdgcn_readfirstlane(min(n_r, lo + len));
        double Yin = 0.0, Zin = 0.0;
        for (int c = 0; c < ch; ++c) Yin = sA[c * kLanes + lane] * Yin + sY[c * kLanes + lane];
        for (int c = T - 1; c > ch; --c) Zin = sZ[c * kLanes + lane] + sC[c * kLanes + lane] * Zin;
        if (l < 0) {
            for (int n = lo; n < hi; ++n) {
                store<NT>(g.M + base + (size_t)n * np, 0.0);
                store<NT>(g.Bred + base + (size_t)n * np, 0.0);
                if (g.Ms) {
                    bf16 *o = g.Ms + split_offset_of(f, n, q, n_r, np, g.pp, g.ks2);
                    store<NT>(o, (bf16)0.0f);
                    store<NT>(o + kBlk, (bf16)0.0f);
                    store<NT>(o + 2 * kBlk, (bf16)0.0f);
                }
            }
            continue;
        }
        finish_chunk<NT>(g, base, cf, cstep, f, q, lo, hi, Yin, Zin);
    }
}

}  // namespace scan_detail
}  // namespace mpg
