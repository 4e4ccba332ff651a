// The separable method's contractions (Sec. 4.3 steps 2 and 5, in FP64).
//
// In a patch's own frame the weights of its cell (j, k) factor as in the
// single-grid sums of Eqs. a_ci^lm and a_si^lm: the local moments are
//   A^(lu)_{C,S} = sum_jk w_jk rho_jk s_lu T_j^{lu} {C_k^u, S_k^u},
// and the rotation sums of Eqs. U_C/U_S (the N factors of Eqs. N_CC..N_SC)
// take them to the common frame degree by degree:
//   B^(lm) = sum_patches sum_u X^(l)[(m, .)][(u, .)] A^(lu) (times 2/delta_m).
// The same factors write the common-frame harmonics of Eqs. Q_C/Q_S in a
// patch's local ones, so the expansion runs the steps backwards:
//   L^(lu) = sum_m M^(lm) X^(l)[(m, .)][(u, .)],
//   Phi_jk = sum_lu -G s_lu P_l^u(cos theta_j) {cos, sin}(u phi_k) L^(lu).
// Rows (v, j), v = (field, patch, shell), j the theta row, of the density
// are contiguous runs of n_phi cells.  Five kernels:
//   phi1   F[c][j][v]      = sum_k w_jk rho_(v,j),k f1_k^(c)     (phi transform)
//   theta1 A[slot][v]      = sum_j t1_j^(lu) F[c(u)][j][v]       (per order u)
//   rot1   B[row][lm]      = sum_(patch, u) x1^(l) A             (per degree l)
//   rot2   L[slot][v]      = sum_m M[row][lm] x2^(l)             (per degree, patch)
//   theta2 G[c][j][v]      = sum_l t2_j^(lu) L[slot][v]
//   phi2   Phi_(v,j),k     = sum_c G[c][j][v] f2_k^(c)
// (slot: one per (l, u, C or S), grouped by phi column).  On a phi grid
// symmetric about 0 with an even cell count the transforms fold the mirror
// cells k and n_phi-1-k: C_k^u is even and S_k^u odd in phi, so the C
// columns take the weighted sum of the two cells and the S columns their
// difference over half the cells, and the expansion writes E + O and E - O
// to a point and its mirror image from the cosine (E) and sine (O) sums.
//
// All are v_mfma_f64_16x16x4f64 contractions with 256 threads (four waves)
// per block and 16-deep K slabs staged through LDS, laid out so that every
// global access runs along v.  The phi transforms carry almost all the
// work: phi1 reads the density once (converted, weighted and folded on the
// way into LDS) and keeps every phi column of its 128 rows in registers;
// phi2 keeps the cosine and sine sums of a 128 x 64 tile of rows and
// evaluation points.
#include "mpg_internal.h"

namespace mpg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int SK = 16;       // K slab depth
constexpr int TR = 64;       // rows per block of the rotations
constexpr int VB = 128;      // rows v per block of the transforms and theta contractions
constexpr int PA = VB + 16;  // LDS row pitch of a 128-wide operand (doubles)
constexpr int JB = 4;        // theta rows per block of the expansion's phi transform
constexpr int JR1 = 1;       // and of the moments' (whose registers hold no more state)
constexpr int kMaxTiles = 9; // 16-wide tiles of a degree's 2 lmax + 1 <= 129 entries

__device__ inline v4d mfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// LDS pitch of a slab row of n doubles (n a multiple of 16): an odd multiple
// of 16, so that rows k and k + 1 of a fragment read fall in different bank
// halves
__host__ __device__ constexpr int pitch(int n) { return (n / 16) % 2 ? n : n + 16; }

// The split form keeps the phi columns c >= 1 of its transforms in FP32 (its
// phi transforms sum in FP32 and round their operands to FP32 first, so no
// value changes): column c at [(c - 1) n_theta + j][v] of the FP32 view
// that starts past column 0, which stays FP64 at F[j][v].
__device__ inline float *tf_f32(double *F, int n_theta, int ldv) {
    return reinterpret_cast<float *>(F + (size_t)n_theta * ldv);
}
__device__ inline const float *tf_f32(const double *F, int n_theta, int ldv) {
    return reinterpret_cast<const float *>(F + (size_t)n_theta * ldv);
}

// Lane layout of v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register q of lane l is D[l/16 + 4q][l%16].

// ---------------------------------------------------------------------------
// The transforms keep their columns apart: F and G are [c][j][v] (v =
// (field, patch, shell), ldv of them per (c, j)), the local moments and
// coefficients [slot][v] with slot = coff[c] + l - u (every (l, u, C/S) once).

// Phi transform of the moments.  Block: 128 rows v of one (field, patch)
// group at JR consecutive theta rows j, one after the other; output
// F[c][j][v] = sum_k w_jk rho_(v,j),k f1[k][c] for the order-0 column (a
// row sum) and all NT column tiles of 16 after it (the first NE = NT/2 the
// C columns), as the product f1^T (columns as rows) times
// the folded density slab (rows v as columns), so that a store writes 16
// consecutive v.  K = the kh cells in slabs of 16.  The weight row of the
// current j sits in LDS.  Thread t stages 8 consecutive cells of row t/2
// (from 8 (t%2)), with MIR also their 8 mirror cells, and NT entries of the
// factor slab, into one of two register sets: each slab is loaded two slabs
// ahead of its use (one with eight column tiles, whose registers are full).
template <typename T>
struct PhiStage {
    T a[8], b[8];
};

template <typename T, bool MIR>
__device__ inline void load_phi(PhiStage<T> &st, const T *row, int k, int n_phi, int kh, bool row_ok) {
    if (sizeof(T) == 4 && (n_phi & 3) == 0 && k + 8 <= kh) {
        // 16-byte aligned: rows start at multiples of 4 cells, k and the
        // mirror run n_phi-8-k too
        f32x4 x0 = {0.f, 0.f, 0.f, 0.f}, x1 = x0, y0 = x0, y1 = x0;
        if (row_ok) {
            x0 = *(const f32x4 *)(row + k);
            x1 = *(const f32x4 *)(row + k + 4);
            if (MIR) {
                y0 = *(const f32x4 *)(row + n_phi - 8 - k);
                y1 = *(const f32x4 *)(row + n_phi - 4 - k);
            }
        }
        const float xa[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        const float ya[8] = {y1.w, y1.z, y1.y, y1.x, y0.w, y0.z, y0.y, y0.x};  // cells n_phi-1-k-q
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            st.a[q] = (T)xa[q];
            st.b[q] = (T)ya[q];
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool ok = row_ok && k + q < kh;
        st.a[q] = ok ? row[k + q] : (T)0;
        st.b[q] = (ok && MIR) ? row[n_phi - 1 - k - q] : (T)0;
    }
}

template <typename T, bool MIR, int NT, int JR>
__global__ __launch_bounds__(256, 2) void k_sep_phi1(const T *__restrict__ rho, const double *__restrict__ w,
                                                     size_t w_patch, const double *__restrict__ f1,
                                                     double *__restrict__ F, int ldv, int n_r, int n_patches,
                                                     int n_theta, int n_phi, int kh, int nst) {
    // column tiles: C then S of the orders 1..lmax, NE = NT/2 of each; the
    // order-0 column (factor C_k^0 = dphi for every cell) is a weighted row
    // sum, formed while staging
    constexpr int NC = NT * 16, PB = pitch(NC), NE = NT / 2;
    extern __shared__ double sW[];  // the weight row w_j. of the block's patch
    __shared__ double Ae[SK][PA];
    __shared__ double Ao[MIR ? SK : 1][MIR ? PA : 1];
    __shared__ double Bs[SK][PB];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fg = blockIdx.x / nst, st0 = (blockIdx.x - fg * nst) * VB;
    const int j0 = blockIdx.y * JR, jn = min(JR, n_theta - j0);
    const int nv = min(VB, n_r - st0);
    const size_t v0 = (size_t)fg * n_r + st0;
    const double *wp = w + (size_t)(fg % n_patches) * w_patch;

    // this thread's staging row (v0 + sr, j) and cells
    const int sr = tid >> 1, sk = (tid & 1) * 8;
    const bool row_ok = sr < nv;
    const T *prow0 = rho + ((v0 + (row_ok ? sr : 0)) * n_theta + j0) * n_phi;

    v4d acc[NT][2];
    const int nsl = (kh + SK - 1) / SK;
    // NR register sets: slab s is loaded NR slabs ahead of its use (two for
    // up to six column tiles; the eight-tile variants have no room)
    constexpr int NR = NT <= 6 ? 2 : 1;
    PhiStage<T> stg[NR];
    double bv[NR][NT];
    // slab s of theta row j0 + jj into register set r
    auto load = [&](int r, int jj, int s) {
        load_phi<T, MIR>(stg[r], prow0 + (size_t)jj * n_phi, s * SK + sk, n_phi, kh, row_ok);
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int e = tid + 256 * q;
            bv[r][q] = f1[(size_t)(s * SK + e / NC) * (NC + 1) + 1 + e % NC];
        }
    };
    // after slab s of row jj is staged from set r: the slab NR ahead (in the
    // next row past this row's last) into set r
    auto load_ahead = [&](int r, int jj, int s) {
        const int t = s + NR;
        if (t < nsl) load(r, jj, t);
        else if (jj + 1 < jn && t - nsl < nsl) load(r, jj + 1, t - nsl);
    };
    load(0, 0, 0);
    if (NR == 2) {
        if (nsl > 1) load(NR - 1, 0, 1);
        else if (jn > 1) load(NR - 1, 1, 0);
    }
    const int wv = wave * 32;
    const double c0 = f1[0];  // C_k^0, the same for every cell
    for (int jj = 0; jj < jn; ++jj) {
        const int j = j0 + jj;
        double sum0 = 0.0;  // this thread's cells of the order-0 sum
        // the weight row of theta row j (the previous row's slabs are done)
        for (int k = tid; k < n_phi; k += 256) sW[k] = wp[(size_t)j * n_phi + k];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i) acc[t][i] = v4d{0.0, 0.0, 0.0, 0.0};
        __syncthreads();
        // slab s of this row uses register set (jj * nsl + s) % NR
        auto step = [&](const int r, int s) {
            // stage slab s (weights of cells past kh multiply zeros)
            const int k = s * SK + sk;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool in = k + q < kh;
                const double a = (in ? sW[k + q] : 0.0) * (double)stg[r].a[q];
                const double b = (MIR && in) ? sW[n_phi - 1 - k - q] * (double)stg[r].b[q] : 0.0;
                Ae[sk + q][sr] = a + b;
                if (MIR) Ao[sk + q][sr] = a - b;
                sum0 += a + b;
            }
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int e = tid + 256 * q;
                Bs[e / NC][e % NC] = bv[r][q];
            }
            __syncthreads();
            load_ahead(r, jj, s);
#pragma unroll
            for (int kk = 0; kk < SK / 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                double ae[2], ao[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    ae[i] = Ae[kr][wv + i * 16 + (lane & 15)];
                    ao[i] = MIR ? Ao[kr][wv + i * 16 + (lane & 15)] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const double b = Bs[kr][t * 16 + (lane & 15)];
#pragma unroll
                    for (int i = 0; i < 2; ++i) acc[t][i] = mfma(b, (MIR && t >= NE) ? ao[i] : ae[i], acc[t][i]);
                }
            }
            __syncthreads();
        };
        if (NR == 1) {
            for (int s = 0; s < nsl; ++s) step(0, s);
        } else {
            const int r0 = (jj * nsl) & 1;
            int s = 0;
            for (; s + 1 < nsl; s += 2) {
                if (r0 == 0) {
                    step(0, s);
                    step(NR - 1, s + 1);
                } else {
                    step(NR - 1, s);
                    step(0, s + 1);
                }
            }
            if (s < nsl) {
                if (r0 == 0) step(0, s);
                else step(NR - 1, s);
            }
        }
        // the order-0 column: the row's two staging threads are lanes 2i, 2i+1
        sum0 += __shfl_xor(sum0, 1);
        if (sk == 0 && row_ok) F[(size_t)j * ldv + v0 + sr] = c0 * sum0;
        // register q of lane l: column c = 1 + 16t + l/16 + 4q, row v = wv + 16i + l%16
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = 1 + t * 16 + (lane >> 4) + 4 * q, vv = wv + i * 16 + (lane & 15);
                    if (vv < nv) F[((size_t)c * n_theta + j) * ldv + v0 + vv] = acc[t][i][q];
                }
    }
}

// ---------------------------------------------------------------------------
// Theta contraction of the moments: block (128 rows v from v0 = 128 x, phi
// column c = y): A[coff[c] + s][v] = sum_j t1[c][s][j] F[c][j][v] for the
// degree slots s < lmax + 1 - u (at most five tiles of 16), K = n_theta in
// slabs of 16; slots as rows, v as columns (stores of 16 consecutive v).
// Wave w takes v 32w..32w+31.  v past the last row lie in the zeroed
// padding of the work arrays and are not stored.  F32: the columns c >= 1
// are FP32 (the split form's phi transforms, see tf_f32).
template <bool F32>
__global__ __launch_bounds__(256) void k_sep_theta1(const double *__restrict__ F, int ldv,
                                                    const double *__restrict__ t1, const int *__restrict__ sep_u,
                                                    const int *__restrict__ coff, double *__restrict__ A, int vrows,
                                                    int n_theta, int lp, int L) {
    constexpr int NTM = 5;
    // t1 slab slot-major ([slot][j], odd pitch: its staging writes and the
    // fragment reads of 16 slots x 4 j both spread over the banks)
    __shared__ double As[NTM * 16][SK + 1];
    __shared__ double Bs[SK][PA];
    const int c = blockIdx.y, u = sep_u[c];
    if (u < 0) return;  // padding column (the whole block)
    const int nl = L + 1 - u, ntl = (nl + 15) / 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int v0 = blockIdx.x * VB, wv = wave * 32;
    const double *tc = t1 + (size_t)c * lp * n_theta;
    const bool flt = F32 && c > 0;
    const double *Fc = F + (size_t)c * n_theta * ldv + v0;
    const float *Fs = tf_f32(F, n_theta, ldv) + (size_t)(c - 1) * n_theta * ldv + v0;

    v4d acc[NTM][2];
#pragma unroll
    for (int t = 0; t < NTM; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[t][i] = v4d{0.0, 0.0, 0.0, 0.0};
    // staging: t1 16 j x 80 slots (entry e = tid + 256q: slot e/16, j e%16);
    // F 16 j x 128 v (thread: j tid/16, v tid%16 + 16q); the next slab is
    // loaded into registers while the current one is multiplied
    const int bj = tid >> 4, bv = tid & 15;
    double ra[NTM], rb[8];
    auto load = [&](int j0) {
#pragma unroll
        for (int q = 0; q < NTM; ++q) {
            const int e = tid + 256 * q, sl = e >> 4, j = j0 + (e & 15);
            ra[q] = (sl < nl && j < n_theta) ? tc[(size_t)sl * n_theta + j] : 0.0;
        }
        const bool jok = j0 + bj < n_theta;
        const size_t fo = (size_t)(jok ? j0 + bj : 0) * ldv + bv;
        if (flt) {
            // FP32: v 4 bv + 64 q + e (e < 4) of row j, 16-byte loads
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float4 f = jok ? *(const float4 *)(Fs + fo - bv + 4 * bv + 64 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
                rb[4 * q] = f.x;
                rb[4 * q + 1] = f.y;
                rb[4 * q + 2] = f.z;
                rb[4 * q + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) rb[q] = jok ? Fc[fo + 16 * q] : 0.0;
        }
    };
    load(0);
    for (int j0 = 0; j0 < n_theta; j0 += SK) {
#pragma unroll
        for (int q = 0; q < NTM; ++q) {
            const int e = tid + 256 * q;
            As[e >> 4][e & 15] = ra[q];
        }
        if (flt) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[bj][4 * bv + 64 * q + e] = rb[4 * q + e];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[bj][bv + 16 * q] = rb[q];
        }
        __syncthreads();
        if (j0 + SK < n_theta) load(j0 + SK);
#pragma unroll
        for (int kk = 0; kk < SK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) b[i] = Bs[kr][wv + i * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < NTM; ++t)
                if (t < ntl) {
                    const double a = As[t * 16 + (lane & 15)][kr];
#pragma unroll
                    for (int i = 0; i < 2; ++i) acc[t][i] = mfma(a, b[i], acc[t][i]);
                }
        }
        __syncthreads();
    }
    double *Ac = A + (size_t)coff[c] * ldv + v0;
#pragma unroll
    for (int t = 0; t < NTM; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int sl = t * 16 + (lane >> 4) + 4 * q, vv = wv + i * 16 + (lane & 15);
                if (t < ntl && sl < nl && v0 + vv < vrows) Ac[(size_t)sl * ldv + vv] = acc[t][i][q];
            }
}

// ---------------------------------------------------------------------------
// Rotations of degree l (lmax - blockIdx.y), 64 rows of (field, shell) per block.
//   EXP = false (moments): B[row][perm[l^2 + o]] = sum over kk = (patch g,
//     position i) of A[cslot[l^2 + i]][(f, g, shell)] x1[l][kk][o];  K = P (2l+1)
//   EXP = true (expansion, patch g = blockIdx.z):
//     L[cslot[l^2 + o]][(f, g, shell)] = sum_i M[row][perm[l^2 + i]] x2[l][g][i][o];  K = 2l+1
// N = 2l + 1 in up to nine tiles of 16; wave w takes rows 16w..16w+15.
template <bool EXP>
__global__ __launch_bounds__(256) void k_sep_rot(const double *__restrict__ src, const double *__restrict__ x,
                                                 const long long *__restrict__ xoff, const int *__restrict__ perm,
                                                 const int *__restrict__ cslot, double *__restrict__ dst, int rows,
                                                 int n_r, int P, int ldv, int np) {
    constexpr int NB = kMaxTiles * 16;
    __shared__ double As[SK][pitch(TR)];
    __shared__ double Bs[SK][pitch(NB)];
    // the costliest degrees first (a block's work grows as (2l + 1)^2)
    const int l = gridDim.y - 1 - blockIdx.y, n = 2 * l + 1, nto = (n + 15) / 16, g = EXP ? blockIdx.z : 0;
    const int K = EXP ? n : P * n, l2 = l * l;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = blockIdx.x * TR;
    const double *xl = x + xoff[l] + (EXP ? (size_t)g * n * n : 0);

    v4d acc[kMaxTiles];
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    // staging: A 64 rows x 16 (thread: row tid%64, 4 consecutive kk from
    // 4 (tid/64)); B 16 x 144 (entries tid + 256q); the next slab is loaded
    // into registers while the current one is multiplied
    const int ar = tid & 63, ak = (tid >> 6) * 4;
    const int arow = row0 + ar;
    const bool arow_ok = arow < rows;
    const int af = arow_ok ? arow / n_r : 0, ash = arow_ok ? arow - af * n_r : 0;
    double ra[4], rb[kMaxTiles];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = k0 + ak + q;
            double v = 0.0;
            if (arow_ok && kk < K) {
                if (EXP) {
                    v = src[(size_t)arow * np + perm[l2 + kk]];
                } else {
                    const int gi = kk / n, i = kk - gi * n;
                    v = src[(size_t)cslot[l2 + i] * ldv + (size_t)(af * P + gi) * n_r + ash];
                }
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < kMaxTiles; ++q) {
            const int e = tid + 256 * q, kr = e / NB, o = e - kr * NB, kk = k0 + kr;
            rb[q] = (kk < K && o < n) ? xl[(size_t)kk * n + o] : 0.0;
        }
    };
    load(0);
    for (int k0 = 0; k0 < K; k0 += SK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) As[ak + q][ar] = ra[q];
#pragma unroll
        for (int q = 0; q < kMaxTiles; ++q) {
            const int e = tid + 256 * q, kr = e / NB;
            Bs[kr][e - kr * NB] = rb[q];
        }
        __syncthreads();
        if (k0 + SK < K) load(k0 + SK);
#pragma unroll
        for (int kk = 0; kk < SK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            const double a = As[kr][wave * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < kMaxTiles; ++t)
                if (t < nto) acc[t] = mfma(a, Bs[kr][t * 16 + (lane & 15)], acc[t]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = row0 + wave * 16 + (lane >> 4) + 4 * q, o = t * 16 + (lane & 15);
            if (t >= nto || row >= rows || o >= n) continue;
            if (EXP) {
                const int f = row / n_r, sh = row - f * n_r;
                dst[(size_t)cslot[l2 + o] * ldv + (size_t)(f * P + g) * n_r + sh] = acc[t][q];
            } else {
                dst[(size_t)row * np + perm[l2 + o]] = acc[t][q];
            }
        }
}

// ---------------------------------------------------------------------------
// Theta contraction of the expansion: block (128 v from 128 x, phi column
// c = y, 128 theta rows from 128 z): G[c][j][v] = sum_s t2[c][s][j]
// L[coff[c] + s][v], K = the degree slots in slabs of 16; theta rows as
// rows, v as columns.  Wave w takes theta rows 64(w%2).. and v 64(w/2)..
// F32: the columns c >= 1 are stored in FP32 (see tf_f32).
template <bool F32>
__global__ __launch_bounds__(256, 2) void k_sep_theta2(const double *__restrict__ Lc, const double *__restrict__ t2,
                                                    const int *__restrict__ sep_u, const int *__restrict__ coff,
                                                    double *__restrict__ G, int ldv, int vrows, int n_theta, int lp,
                                                    int L) {
    __shared__ double As[SK][PA];
    __shared__ double Bs[SK][PA];
    const int c = blockIdx.y, u = sep_u[c];
    if (u < 0) return;
    const int nl = L + 1 - u;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int v0 = blockIdx.x * VB, j0 = blockIdx.z * VB;
    const int wj = (wave & 1) * 64, wv = (wave >> 1) * 64;
    const double *tc = t2 + (size_t)c * lp * n_theta;
    const double *lc = Lc + (size_t)coff[c] * ldv + v0;

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[i][t] = v4d{0.0, 0.0, 0.0, 0.0};
    // staging (thread: slot tid/16, theta rows or v tid%16 + 16q); the next
    // slab is loaded into registers while the current one is multiplied
    const int ss = tid >> 4, sx = tid & 15;
    double ra[8], rb[8];
    auto load = [&](int s0) {
        const bool sok = s0 + ss < nl;
        const double *tr = tc + (size_t)(sok ? s0 + ss : 0) * n_theta + j0 + sx;
        const double *lr = lc + (size_t)(sok ? s0 + ss : 0) * ldv + sx;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            ra[q] = (sok && j0 + sx + 16 * q < n_theta) ? tr[16 * q] : 0.0;
            rb[q] = sok ? lr[16 * q] : 0.0;
        }
    };
    load(0);
    for (int s0 = 0; s0 < nl; s0 += SK) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            As[ss][sx + 16 * q] = ra[q];
            Bs[ss][sx + 16 * q] = rb[q];
        }
        __syncthreads();
        if (s0 + SK < nl) load(s0 + SK);
#pragma unroll
        for (int kk = 0; kk < SK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kr][wj + i * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = Bs[kr][wv + t * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[i][t] = mfma(a[i], b[t], acc[i][t]);
        }
        __syncthreads();
    }
    double *Gc = G + (size_t)c * n_theta * ldv + v0;
    float *Gs = tf_f32(G, n_theta, ldv) + (size_t)(c - 1) * n_theta * ldv + v0;
    const bool flt = F32 && c > 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + wj + i * 16 + (lane >> 4) + 4 * q, vv = wv + t * 16 + (lane & 15);
                if (j < n_theta && v0 + vv < vrows) {
                    if (flt) Gs[(size_t)j * ldv + vv] = (float)acc[i][t][q];
                    else Gc[(size_t)j * ldv + vv] = acc[i][t][q];
                }
            }
}

// ---------------------------------------------------------------------------
// Phi transform of the expansion: block (64 evaluation points b, 128 rows v,
// JB theta rows one after the other; the point tiles of the same rows run
// on one XCD and share G in its L2): E = the sum over the C columns plus
// the order-0 column's value (staged in LDS; its factor is cos 0 = 1), O
// the sum over the S columns (with MIR; else all columns go to E);
// Phi[(v, j)][kxy[b].x] = E + O and, with a mirror cell, Phi[(v, j)][kxy[b].y]
// = E - O.  K = the phi columns in slabs of 16.  Wave w takes v 32w.. and
// the block's point tiles (fewer than four in the last), and writes its
// outputs 16 rows at a time through LDS so that each store instruction
// covers one row's 64 consecutive points.  Thread t stages v t%16 + 16q
// (q < 8) of phi column t/16 and points t%16 + 16q (q < 4) of its factor
// row.
template <typename T, bool MIR>
__global__ __launch_bounds__(256, 2) void k_sep_phi2(const double *__restrict__ G, int ldv,
                                                     const double *__restrict__ f2, const int2 *__restrict__ kxy,
                                                     T *__restrict__ phi, int vrows, int n_theta, int n_phi, int kx,
                                                     int ce, int co, int nbt, int nvt, int ngroups) {
    // the slab staging, or (after a theta row's last slab) each wave's 16
    // x 128 tile of outputs on its way to global memory
    constexpr int PO = 144;  // output tile pitch (elements of T): 16 rows x 16 points spread over the banks
    constexpr int STG = SK * PA + SK * pitch(64), OUT = 4 * 16 * PO * (int)sizeof(T) / 8;
    __shared__ double lds[STG > OUT ? STG : OUT];
    double(*As)[PA] = reinterpret_cast<double(*)[PA]>(lds);
    double(*Bs)[pitch(64)] = reinterpret_cast<double(*)[pitch(64)]>(lds + SK * PA);
    // the order-0 column at the current theta row (MIR), by row parity: a
    // row's epilogue reads it while faster waves may already stage the next
    __shared__ double sG0[2][VB];
    // blocks go to the eight XCDs in turn (block id mod 8): the nbt point
    // tiles of one group of rows take ids 8 apart, so they run on one XCD
    // and read their group's G through one L2
    const int id = blockIdx.x, k8 = id >> 3, bt = k8 % nbt, grp = (k8 / nbt) * 8 + (id & 7);
    if (grp >= ngroups) return;  // the whole block, before any barrier
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = bt * 64, v0 = (grp % nvt) * VB, wv = wave * 32;
    const int j0 = (grp / nvt) * JB, jn = min(JB, n_theta - j0);
    const int ntc = min(4, (kx - b0 + 15) / 16);  // point tiles of this block
    const int sc = tid >> 4, sx = tid & 15;
    const int2 kk = b0 + lane < kx ? kxy[b0 + lane] : make_int2(0, -1);  // this lane's output point

    v4d E[2][4], O[2][4];
    // With MIR: E slabs the C columns [1, 1 + ce), O slabs the S columns
    // [1 + ce, nc), and the order-0 column (factor cos 0 = 1 at every
    // point) added to E from LDS.  Without MIR all columns [0, nc) go to
    // E, zero past them in the last slab.
    const int nc = 1 + ce + co;
    const int nse = MIR ? ce / SK : (nc + SK - 1) / SK, nsl = MIR ? nse + co / SK : nse;
    double av[8], bv[4], g0r = 0.0;
    // slab s of theta row j0 + jj into registers (v past the last row lie
    // in the zeroed padding of G and feed only rows that are not stored)
    auto load = [&](int jj, int s) {
        if (MIR && s == 0 && tid < VB) g0r = G[(size_t)(j0 + jj) * ldv + v0 + tid];  // padded rows are zero
        const int c = (MIR ? 1 : 0) + s * SK + sc;
        const bool ok = c < nc;
        const double *g = G + ((size_t)(ok ? c : 0) * n_theta + j0 + jj) * ldv + v0 + sx;
#pragma unroll
        for (int q = 0; q < 8; ++q) av[q] = ok ? g[16 * q] : 0.0;
        const double *f = f2 + (size_t)(ok ? c : 0) * kx + b0 + sx;
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] = (ok && b0 + sx + 16 * q < kx) ? f[16 * q] : 0.0;
    };
    // slabs [s0, s1) of theta row j0 + jj into acc; the first slab's
    // operands are in registers, and the last prefetches the next row's first
    auto run = [&](v4d(&acc)[2][4], int jj, int s0, int s1) {
        for (int s = s0; s < s1; ++s) {
            if (MIR && s == 0 && tid < VB) sG0[jj & 1][tid] = g0r;
#pragma unroll
            for (int q = 0; q < 8; ++q) As[sc][sx + 16 * q] = av[q];
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[sc][sx + 16 * q] = bv[q];
            __syncthreads();
            {
                const bool last = s + 1 == nsl;
                if (!last || jj + 1 < jn) load(last ? jj + 1 : jj, last ? 0 : s + 1);
            }
#pragma unroll
            for (int kk = 0; kk < SK / 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                double a[2], b[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[kr][wv + i * 16 + (lane & 15)];
#pragma unroll
                for (int t = 0; t < 4; ++t) b[t] = Bs[kr][t * 16 + (lane & 15)];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < ntc) {
#pragma unroll
                        for (int i = 0; i < 2; ++i) acc[i][t] = mfma(a[i], b[t], acc[i][t]);
                    }
            }
            __syncthreads();
        }
    };
    load(0, 0);
    for (int jj = 0; jj < jn; ++jj) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) E[i][t] = O[i][t] = v4d{0.0, 0.0, 0.0, 0.0};
        run(E, jj, 0, MIR ? nse : nsl);
        if (MIR) run(O, jj, nse, nsl);
        // outputs through LDS: each lane puts its values at (row, point) of
        // the wave's tile, then a store instruction writes one row's 64
        // points (and their mirror points), consecutive in memory
        T(*ot)[PO] = reinterpret_cast<T(*)[PO]>(lds) + wave * 16;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int bl = t * 16 + (lane & 15);
                const double f0 = MIR ? f2[min(b0 + bl, kx - 1)] : 0.0;  // the order-0 factor
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = (lane >> 4) + 4 * q;
                    const double e = E[i][t][q] + (MIR ? f0 * sG0[jj & 1][wv + i * 16 + r] : 0.0), d = O[i][t][q];
                    ot[r][bl] = (T)(e + d);
                    if (MIR) ot[r][64 + bl] = (T)(e - d);
                }
            }
            __syncthreads();
            if (b0 + lane < kx) {
#pragma unroll 4
                for (int r = 0; r < 16; ++r) {
                    const int v = v0 + wv + i * 16 + r;
                    if (v >= vrows) break;
                    T *o = phi + ((size_t)v * n_theta + j0 + jj) * n_phi;
                    o[kk.x] = ot[r][lane];
                    if (MIR && kk.y >= 0) o[kk.y] = ot[r][64 + lane];
                }
            }
            __syncthreads();  // the tile area is the next round's, then the next row's staging
        }
    }
}

// ---------------------------------------------------------------------------
// Split forms of the two phi transforms (MPG_SPLIT_BF16): the same sums in
// six bf16 piece products (h h, h m, m h, h l, m m, l h of the three pieces
// of each FP32-rounded operand) on v_mfma_f32_32x32x16_bf16, accumulated in
// FP32 over at most n_phi/2 (moments) or 2 ce (expansion) terms.  The
// moments' sums go unchanged to the FP32 columns (tf_f32), the expansion's
// to the potential.  The order-0 column stays an FP64 row sum (moments) and
// an FP64 term added to the cosine sums (expansion).
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int PK = 24;  // LDS pitch (bf16) of a 16-deep row of pieces: 16 rows of a fragment read hit distinct banks

// C/D layout of v_mfma_f32_32x32x16_bf16 (measured): register r of lane l
// holds D[8(r/4) + 4(l/32) + r%4][l%32]; A rows are lane%32 with K elements
// 8(l/32)..+7, B columns lane%32 with the same K elements.
__device__ inline int d_row32(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

__device__ inline v16f mfma32(v8bf a, v8bf b, v16f c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }

// the six partial products of a fragment pair into acc, smallest first
__device__ inline v16f six(const v8bf (&a)[3], const v8bf (&b)[3], v16f acc) {
    acc = mfma32(a[2], b[0], acc);
    acc = mfma32(a[1], b[1], acc);
    acc = mfma32(a[0], b[2], acc);
    acc = mfma32(a[1], b[0], acc);
    acc = mfma32(a[0], b[1], acc);
    return mfma32(a[0], b[0], acc);
}

// three bf16 pieces of an FP32 value (h + m + l exact)
__device__ inline void split3(float v, bf16 &h, bf16 &m, bf16 &l) {
    h = (bf16)v;
    const float r = v - (float)h;
    m = (bf16)r;
    l = (bf16)(r - (float)m);
}

// Moments.  Block: 128 rows v of one (field, patch) group at theta row j;
// output F[c][j][v] for the order-0 column and the 2 NT2 tiles of 32 factor
// rows (C of the orders 1.., then S); K = the kh cells in slabs of 16.  Wave
// w takes v 32w.. and every factor tile.  Thread t stages 8 cells of row t/2
// (as the FP64 kernel) as pieces, and chunks t + 256q of the factor slab.
// Block ids take the theta row fastest, so the blocks in flight read
// neighbouring theta rows of the same density rows.
template <typename T, bool MIR, int NT2>
__global__ __launch_bounds__(256, 2) void k_sep_phi1s(const T *__restrict__ rho, const double *__restrict__ w,
                                                      size_t w_patch, const bf16 *__restrict__ f1s,
                                                      const double *__restrict__ f1, double *__restrict__ F, int ldv,
                                                      int n_r, int n_patches, int n_theta, int n_phi, int kh, int khp,
                                                      int ce, int L, int nst) {
    constexpr int NR = 64 * NT2, NCH = 3 * NR * 2, QF = (NCH + 255) / 256;
    extern __shared__ double sW[];
    __shared__ __attribute__((aligned(16))) bf16 Af[3][NR][PK];
    __shared__ __attribute__((aligned(16))) bf16 Bd[MIR ? 2 : 1][3][VB][PK];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = blockIdx.x % n_theta, fs = blockIdx.x / n_theta;
    const int fg = fs / nst, st0 = (fs - fg * nst) * VB;
    const int nv = min(VB, n_r - st0);
    const size_t v0 = (size_t)fg * n_r + st0;
    const double *wrow = w + (size_t)(fg % n_patches) * w_patch + (size_t)j * n_phi;
    for (int k = tid; k < n_phi; k += 256) sW[k] = wrow[k];

    const int sr = tid >> 1, sk = (tid & 1) * 8;
    const bool row_ok = sr < nv;
    const T *prow = rho + ((v0 + (row_ok ? sr : 0)) * n_theta + j) * n_phi;
    const size_t npc = (size_t)NR * khp;  // one piece of the factor table

    v16f acc[2 * NT2];
#pragma unroll
    for (int t = 0; t < 2 * NT2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
    const int nsl = (kh + SK - 1) / SK;
    PhiStage<T> stg;
    v8bf fc[QF];
    auto load = [&](int s) {
        load_phi<T, MIR>(stg, prow, s * SK + sk, n_phi, kh, row_ok);
#pragma unroll
        for (int q = 0; q < QF; ++q) {
            const int e = tid + 256 * q;
            if (e < NCH) {
                const int pc = e / (NR * 2), rem = e - pc * NR * 2;
                fc[q] = *(const v8bf *)(f1s + pc * npc + (size_t)(rem >> 1) * khp + s * SK + (rem & 1) * 8);
            }
        }
    };
    load(0);
    __syncthreads();  // the weight row
    double sum0 = 0.0;
    for (int s = 0; s < nsl; ++s) {
        const int k = s * SK + sk;
        {
            v8bf ph[3], pd[3];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool in = k + q < kh;
                const double a = (in ? sW[k + q] : 0.0) * (double)stg.a[q];
                const double b = (MIR && in) ? sW[n_phi - 1 - k - q] * (double)stg.b[q] : 0.0;
                sum0 += a + b;
                bf16 h, m, l;
                split3((float)(a + b), h, m, l);
                ph[0][q] = h;
                ph[1][q] = m;
                ph[2][q] = l;
                if (MIR) {
                    split3((float)(a - b), h, m, l);
                    pd[0][q] = h;
                    pd[1][q] = m;
                    pd[2][q] = l;
                }
            }
#pragma unroll
            for (int pc = 0; pc < 3; ++pc) {
                *(v8bf *)&Bd[0][pc][sr][sk] = ph[pc];
                if (MIR) *(v8bf *)&Bd[MIR ? 1 : 0][pc][sr][sk] = pd[pc];
            }
        }
#pragma unroll
        for (int q = 0; q < QF; ++q) {
            const int e = tid + 256 * q;
            if (e < NCH) {
                const int pc = e / (NR * 2), rem = e - pc * NR * 2;
                *(v8bf *)&Af[pc][rem >> 1][(rem & 1) * 8] = fc[q];
            }
        }
        __syncthreads();
        if (s + 1 < nsl) load(s + 1);
        {
            const int kg = (lane >> 5) * 8, row = lane & 31;
            v8bf be[3], bo[3];
#pragma unroll
            for (int pc = 0; pc < 3; ++pc) {
                be[pc] = *(const v8bf *)&Bd[0][pc][wave * 32 + row][kg];
                if (MIR) bo[pc] = *(const v8bf *)&Bd[MIR ? 1 : 0][pc][wave * 32 + row][kg];
            }
#pragma unroll
            for (int t = 0; t < 2 * NT2; ++t) {
                v8bf a[3];
#pragma unroll
                for (int pc = 0; pc < 3; ++pc) a[pc] = *(const v8bf *)&Af[pc][t * 32 + row][kg];
                acc[t] = six(a, (MIR && t >= NT2) ? bo : be, acc[t]);
            }
        }
        __syncthreads();
    }
    // the order-0 column (factor C_k^0 = dphi for every cell), in FP64
    sum0 += __shfl_xor(sum0, 1);
    if (sk == 0 && row_ok) F[(size_t)j * ldv + v0 + sr] = f1[0] * sum0;
    // register r of lane l: factor row 32t + d_row32(l, r), row v = 32w + l%32;
    // the FP32 sums go to the FP32 columns unchanged
    const int vv = wave * 32 + (lane & 31);
    float *Fs = tf_f32(F, n_theta, ldv);
#pragma unroll
    for (int t = 0; t < 2 * NT2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int fr = t * 32 + d_row32(lane, r), o = t < NT2 ? fr : fr - 32 * NT2;  // order - 1
            const int c = 1 + (t < NT2 ? 0 : ce) + o;
            if (o < L && vv < nv) Fs[((size_t)(c - 1) * n_theta + j) * ldv + v0 + vv] = acc[t][r];
        }
}

// Expansion.  Block: 64 points, 128 rows v and JBS theta rows one after
// the other, XCD-aware ids as the FP64 kernel; the block's factor tile (3
// pieces x 64 points x K columns) is loaded into LDS once and serves every
// theta row.  Wave w takes v 32w.. and both 32-point tiles, with the cosine
// sums E and the sine sums O in FP32.  K = the columns 1.. in slabs of 16
// (E: [0, ce), O: [ce, 2 ce) of them; without MIR all into E).  Each wave
// builds its A fragments from its own loads (lane l: row l%32, columns
// 8 (l/32).. of the slab, two 128-byte runs per load) two slabs ahead, so
// the slab loop needs no barrier.  The order-0 column (FP64) is added in
// the epilogue: lane l loads row l%32, and the row of output register r
// (the same for each half-wave) is read from its lane by v_readlane.
constexpr int JBS = 8;
// factor tile row pitch in 16-byte chunks (K + 8 values): the 16 rows of a
// fragment read start on distinct bank groups
__host__ __device__ constexpr int phi2s_pitch8(int K) { return K / 8 + 1; }
constexpr int KMAX2 = 128;  // 2 ce for lmax <= 64
template <typename T, bool MIR, bool O32>
__global__ __launch_bounds__(256, O32 ? 3 : 2) void k_sep_phi2s(const double *__restrict__ G, int ldv,
                                                      const bf16 *__restrict__ f2s, const double *__restrict__ f2,
                                                      const int2 *__restrict__ kxy, T *__restrict__ phi, int vrows,
                                                      int n_theta, int n_phi, int kx, int kxp, int ce, int nbt, int nvt,
                                                      int ngroups) {
    // [3][64][phi2s_pitch8(K)] chunks of 8 values (typed so that every
    // access is a 16-byte one)
    __shared__ v8bf Bf[3 * 64 * phi2s_pitch8(KMAX2)];
    __shared__ int2 sK[64];    // the block's points (kxy), x = -1 past the last
    __shared__ double sF0[64];  // and their order-0 factors
    const int id = blockIdx.x, k8 = id >> 3, bt = k8 % nbt, grp = (k8 / nbt) * 8 + (id & 7);
    if (grp >= ngroups) return;  // the whole block, before any barrier
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = bt * 64, v0 = (grp % nvt) * VB;
    const int j0 = (grp / nvt) * JBS, jn = min(JBS, n_theta - j0);
    const int K = 2 * ce, nsl = K / SK, nse = MIR ? ce / SK : nsl, PF = phi2s_pitch8(K);
    const size_t npc = (size_t)kxp * K;  // one piece of the factor table
    const int kg = (lane >> 5) * 8, row = lane & 31;
    const size_t cstr = (size_t)n_theta * ldv;  // one column of the FP32 transforms
    // this lane's A row: v = v0 + 32w + row, columns 1 + s SK + kg + q
    const float *ga = tf_f32(G, n_theta, ldv) + (size_t)kg * cstr + (size_t)j0 * ldv + v0 + wave * 32 + row;
    const double *g0p = G + (size_t)j0 * ldv + v0 + wave * 32 + row;

    for (int e = tid; e < 3 * 64 * (K / 8); e += 256) {
        const int pc = e / (64 * (K / 8)), rem = e - pc * 64 * (K / 8), pt = rem / (K / 8), kc = (rem % (K / 8)) * 8;
        Bf[(pc * 64 + pt) * PF + kc / 8] = *(const v8bf *)(f2s + pc * npc + (size_t)(b0 + pt) * K + kc);
    }
    if (tid < 64) {
        const int b = b0 + tid;
        sK[tid] = b < kx ? kxy[b] : make_int2(-1, -1);
        sF0[tid] = b < kx ? f2[b] : 0.0;
    }
    __syncthreads();  // the factor tile and point tables; no barrier follows

    const int total = jn * nsl;
    float gv[2][8];
    auto load = [&](float(&g)[8], int i) {
        if (i < total) {
            const int jj = i / nsl, s = i - jj * nsl;
            const float *p = ga + (size_t)(s * SK) * cstr + (size_t)jj * ldv;
#pragma unroll
            for (int q = 0; q < 8; ++q) g[q] = p[(size_t)q * cstr];
        }
    };
    v16f E[2], O[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) E[t][r] = O[t][r] = 0.f;
    double g0 = 0.0;
    // slab s of theta row jj from register set g, which then loads the slab
    // two ahead
    auto body = [&](float(&g)[8], int jj, int s) {
        if (s == 0) g0 = g0p[(size_t)jj * ldv];  // padded rows are zero
        v8bf a[3];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            bf16 h, m, l;
            split3(g[q], h, m, l);
            a[0][q] = h;
            a[1][q] = m;
            a[2][q] = l;
        }
        load(g, jj * nsl + s + 2);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            v8bf b[3];
#pragma unroll
            for (int pc = 0; pc < 3; ++pc) b[pc] = Bf[(pc * 64 + t * 32 + row) * PF + (s * SK + kg) / 8];
            if (!MIR || s < nse) E[t] = six(a, b, E[t]);
            else O[t] = six(a, b, O[t]);
        }
    };
    // the theta row's outputs: register r of lane l holds row v = 32w +
    // d_row32(l, r) at point 32t + l%32.  Stores take byte offsets from the
    // wave's first row, in 32 bits when its 32 rows span less than 4 GiB.
    using Off = typename std::conditional<O32, unsigned, size_t>::type;
    auto epilogue = [&](int jj) {
        char *o0 = reinterpret_cast<char *>(phi + ((size_t)(v0 + wave * 32) * n_theta + j0 + jj) * n_phi);
        const Off rb = (Off)((size_t)n_theta * n_phi * sizeof(T));
        const int vlim = vrows - v0 - wave * 32;  // rows of this wave inside the call
        const int g0lo = __double2loint(g0), g0hi = __double2hiint(g0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int vl = d_row32(lane, r), r0 = d_row32(0, r);  // vl = r0 or r0 + 4
            const double ga0 = __hiloint2double(__builtin_amdgcn_readlane(g0hi, r0), __builtin_amdgcn_readlane(g0lo, r0));
            const double ga1 = __hiloint2double(__builtin_amdgcn_readlane(g0hi, r0 + 4),
                                                __builtin_amdgcn_readlane(g0lo, r0 + 4));
            const double g0v = lane < 32 ? ga0 : ga1;
            if (vl >= vlim) continue;
            const Off ro = (Off)vl * rb;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int2 kk = sK[t * 32 + row];  // LDS broadcast reads, kept out of registers
                if (kk.x < 0) continue;
                const double e = (double)E[t][r] + sF0[t * 32 + row] * g0v, d = (double)O[t][r];
                *reinterpret_cast<T *>(o0 + (ro + (Off)kk.x * (Off)sizeof(T))) = (T)(e + d);
                if (MIR && kk.y >= 0) *reinterpret_cast<T *>(o0 + (ro + (Off)kk.y * (Off)sizeof(T))) = (T)(e - d);
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) E[t][r] = O[t][r] = 0.f;
    };
    load(gv[0], 0);
    load(gv[1], 1);
    for (int jj = 0; jj < jn; ++jj) {
        for (int s = 0; s < nsl; s += 2) {  // nsl = ce / 8 is even
            body(gv[0], jj, s);
            body(gv[1], jj, s + 1);
        }
        epilogue(jj);
    }
}

template <typename T, bool MIR>
hipError_t launch_phi1(const Plan &p, int n_fields, const T *rho) {
    const int nt = (p.sep_nc() - 1) / 16, nst = (p.n_r + VB - 1) / VB;
    if (p.sep_ce != p.sep_co || p.sep_ce / 16 != nt / 2) return hipErrorInvalidValue;
    const size_t w_patch = p.npat == 1 ? 0 : (size_t)p.n_ang;
    const dim3 grid(n_fields * p.n_patches * nst, (p.n_theta + JR1 - 1) / JR1);
    const size_t lds = sizeof(double) * p.n_phi;
#define MPG_PHI1(N)                                                                                                 \
    case N:                                                                                                         \
        hipLaunchKernelGGL((k_sep_phi1<T, MIR, N, JR1>), grid, dim3(256), lds, p.stream, rho, p.w, w_patch, p.sep_f1,    \
                           p.sep_F, p.sep_ldv(), p.n_r, p.n_patches, p.n_theta, p.n_phi, p.sep_kh, nst);         \
        break;
    switch (nt) {
        MPG_PHI1(2)
        MPG_PHI1(4)
        MPG_PHI1(6)
        MPG_PHI1(8)
    default:
        return hipErrorInvalidValue;
    }
#undef MPG_PHI1
    return hipGetLastError();
}

template <typename T, bool MIR>
void launch_phi2(const Plan &p, int vrows, T *phi) {
    // groups of rows = (128 v, JB theta rows); nbt point tiles per group
    const int nbt = (p.sep_kx + 63) / 64, nvt = (vrows + VB - 1) / VB, ng = nvt * ((p.n_theta + JB - 1) / JB);
    const dim3 grid((unsigned)((ng + 7) / 8 * 8 * nbt));
    hipLaunchKernelGGL((k_sep_phi2<T, MIR>), grid, dim3(256), 0, p.stream, p.sep_F, p.sep_ldv(), p.sep_f2,
                       p.sep_kxy, phi, vrows, p.n_theta, p.n_phi, p.sep_kx, p.sep_ce, p.sep_co, nbt, nvt, ng);
}

}  // namespace

template <typename T, bool MIR>
hipError_t launch_phi1s(const Plan &p, int n_fields, const T *rho) {
    const int nst = (p.n_r + VB - 1) / VB;
    const size_t w_patch = p.npat == 1 ? 0 : (size_t)p.n_ang;
    const size_t nb = (size_t)n_fields * p.n_patches * nst * p.n_theta;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;  // one grid axis
    const dim3 grid((unsigned)nb);
    const size_t lds = sizeof(double) * p.n_phi;
    if (p.sep_nt2 == 1)
        hipLaunchKernelGGL((k_sep_phi1s<T, MIR, 1>), grid, dim3(256), lds, p.stream, rho, p.w, w_patch, p.sep_f1s,
                           p.sep_f1, p.sep_F, p.sep_ldv(), p.n_r, p.n_patches, p.n_theta, p.n_phi, p.sep_kh, p.sep_khp,
                           p.sep_ce, p.lmax, nst);
    else if (p.sep_nt2 == 2)
        hipLaunchKernelGGL((k_sep_phi1s<T, MIR, 2>), grid, dim3(256), lds, p.stream, rho, p.w, w_patch, p.sep_f1s,
                           p.sep_f1, p.sep_F, p.sep_ldv(), p.n_r, p.n_patches, p.n_theta, p.n_phi, p.sep_kh, p.sep_khp,
                           p.sep_ce, p.lmax, nst);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T, bool MIR>
void launch_phi2s(const Plan &p, int vrows, T *phi) {
    const int nbt = (p.sep_kx + 63) / 64, nvt = (vrows + VB - 1) / VB, ng = nvt * ((p.n_theta + JBS - 1) / JBS);
    const dim3 grid((unsigned)((ng + 7) / 8 * 8 * nbt));
    if (2 * p.sep_ce > KMAX2) return;  // lmax <= 64 (checked at plan creation)
    if ((size_t)32 * p.n_theta * p.n_phi * sizeof(T) <= 0xffffffffu)
        hipLaunchKernelGGL((k_sep_phi2s<T, MIR, true>), grid, dim3(256), 0, p.stream, p.sep_F, p.sep_ldv(), p.sep_f2s,
                           p.sep_f2, p.sep_kxy, phi, vrows, p.n_theta, p.n_phi, p.sep_kx, p.sep_kxp, p.sep_ce, nbt, nvt,
                           ng);
    else
        hipLaunchKernelGGL((k_sep_phi2s<T, MIR, false>), grid, dim3(256), 0, p.stream, p.sep_F, p.sep_ldv(), p.sep_f2s,
                           p.sep_f2, p.sep_kxy, phi, vrows, p.n_theta, p.n_phi, p.sep_kx, p.sep_kxp, p.sep_ce, nbt, nvt,
                           ng);
}

hipError_t sep_phi_moments(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    if (n_fields > p.max_fields) return hipErrorInvalidValue;
    if (p.split()) {
        if (rho_dtype == MPG_F64)
            return p.sep_mir ? launch_phi1s<double, true>(p, n_fields, (const double *)rho)
                             : launch_phi1s<double, false>(p, n_fields, (const double *)rho);
        return p.sep_mir ? launch_phi1s<float, true>(p, n_fields, (const float *)rho)
                         : launch_phi1s<float, false>(p, n_fields, (const float *)rho);
    }
    if (rho_dtype == MPG_F64)
        return p.sep_mir ? launch_phi1<double, true>(p, n_fields, (const double *)rho)
                         : launch_phi1<double, false>(p, n_fields, (const double *)rho);
    return p.sep_mir ? launch_phi1<float, true>(p, n_fields, (const float *)rho)
                     : launch_phi1<float, false>(p, n_fields, (const float *)rho);
}

hipError_t sep_theta_moments(const Plan &p, int n_fields) {
    const int vrows = n_fields * p.n_patches * p.n_r, rows = n_fields * p.n_r;
    if (p.sep_lp > 80 || p.lmax > 64) return hipErrorInvalidValue;  // five slot tiles, nine degree tiles
    if (p.split())
        hipLaunchKernelGGL(k_sep_theta1<true>, dim3((vrows + VB - 1) / VB, p.sep_nc()), dim3(256), 0, p.stream,
                           p.sep_F, p.sep_ldv(), p.sep_t1, p.sep_m, p.sep_coff, p.sep_A, vrows, p.n_theta, p.sep_lp,
                           p.lmax);
    else
        hipLaunchKernelGGL(k_sep_theta1<false>, dim3((vrows + VB - 1) / VB, p.sep_nc()), dim3(256), 0, p.stream,
                           p.sep_F, p.sep_ldv(), p.sep_t1, p.sep_m, p.sep_coff, p.sep_A, vrows, p.n_theta, p.sep_lp,
                           p.lmax);
    hipLaunchKernelGGL(k_sep_rot<false>, dim3((rows + TR - 1) / TR, p.lmax + 1), dim3(256), 0, p.stream, p.sep_A,
                       p.sep_x1, p.sep_xoff, p.sep_perm, p.sep_cslot, p.Bpart, rows, p.n_r, p.n_patches,
                       p.sep_ldv(), p.np);
    return hipGetLastError();
}

hipError_t sep_theta_expansion(const Plan &p, int n_fields) {
    const int vrows = n_fields * p.n_patches * p.n_r, rows = n_fields * p.n_r;
    if (n_fields > p.max_fields || p.lmax > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sep_rot<true>, dim3((rows + TR - 1) / TR, p.lmax + 1, p.n_patches), dim3(256), 0,
                       p.stream, p.M, p.sep_x2, p.sep_xoff, p.sep_perm, p.sep_cslot, p.sep_A, rows, p.n_r,
                       p.n_patches, p.sep_ldv(), p.np);
    const dim3 g2((vrows + VB - 1) / VB, p.sep_nc(), (p.n_theta + VB - 1) / VB);
    if (p.split())
        hipLaunchKernelGGL(k_sep_theta2<true>, g2, dim3(256), 0, p.stream, p.sep_A, p.sep_t2, p.sep_m, p.sep_coff,
                           p.sep_F, p.sep_ldv(), vrows, p.n_theta, p.sep_lp, p.lmax);
    else
        hipLaunchKernelGGL(k_sep_theta2<false>, g2, dim3(256), 0, p.stream, p.sep_A, p.sep_t2, p.sep_m, p.sep_coff,
                           p.sep_F, p.sep_ldv(), vrows, p.n_theta, p.sep_lp, p.lmax);
    return hipGetLastError();
}

hipError_t sep_phi_expansion(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    const int vrows = n_fields * p.n_patches * p.n_r;
    if (n_fields > p.max_fields) return hipErrorInvalidValue;
    if (p.split()) {
        if (phi_dtype == MPG_F64) {
            if (p.sep_mir) launch_phi2s<double, true>(p, vrows, (double *)phi);
            else launch_phi2s<double, false>(p, vrows, (double *)phi);
        } else {
            if (p.sep_mir) launch_phi2s<float, true>(p, vrows, (float *)phi);
            else launch_phi2s<float, false>(p, vrows, (float *)phi);
        }
        return hipGetLastError();
    }
    if (phi_dtype == MPG_F64) {
        if (p.sep_mir) launch_phi2<double, true>(p, vrows, (double *)phi);
        else launch_phi2<double, false>(p, vrows, (double *)phi);
    } else {
        if (p.sep_mir) launch_phi2<float, true>(p, vrows, (float *)phi);
        else launch_phi2<float, false>(p, vrows, (float *)phi);
    }
    return hipGetLastError();
}

}  // namespace mpg
