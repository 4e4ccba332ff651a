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
// Rows r = (field, patch, shell, theta row j) of the density are
// contiguous runs of n_phi cells.  Five kernels:
//   phi1   F[c][r]      = sum_k w_jk rho_r,k f_k^(c)          (phi transform)
//   theta1 A[v][lu]     = sum_j t1_j^(lu) F[c(u)][v, j]         (per order u)
//   rot1   B[row][lm]   = sum_(patch, u) x1^(l) A               (per degree l)
//   rot2   L[v][lu]     = sum_m M[row][lm] x2^(l)               (per degree, patch)
//   theta2 G[c][v, j]   = sum_l t2_j^(lu) L[v][lu]
//   phi2   Phi_r,k      = sum_c G[c][r] f2_k^(c)
// (v = (field, patch, shell)).  On a phi grid symmetric about 0 with an even
// cell count the transforms fold the mirror cells k and n_phi-1-k: C_k^u is
// even and S_k^u odd in phi, so the C columns take the weighted sum of the
// two cells and the S columns their difference over half the cells, and the
// expansion writes E + O and E - O to a point and its mirror image from the
// cosine (E) and sine (O) sums.
//
// All are v_mfma_f64_16x16x4f64 contractions with 256 threads (four waves)
// per block and 16-deep K slabs staged through LDS.  The phi transforms
// carry almost all the work: phi1 reads the density once (converted,
// weighted and folded on the way into LDS) and keeps every phi column of its
// 128 rows in registers; phi2 keeps the cosine and sine sums of a 128 x 64
// tile of rows and evaluation points.
#include "mpg_internal.h"

namespace mpg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int SK = 16;       // K slab depth
constexpr int RB = 128;      // rows per block of the phi transforms
constexpr int PA = RB + 16;  // LDS row pitch of a 128-row operand (doubles)
constexpr int TR = 64;       // rows per block of the theta contractions and rotations
constexpr int kMaxTiles = 9; // 16-wide tiles of a degree's 2 lmax + 1 <= 129 entries

__device__ inline v4d mfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// LDS pitch of a slab row of n doubles (n a multiple of 16): an odd multiple
// of 16, so that rows k and k + 1 of a fragment read fall in different bank
// halves
__host__ __device__ constexpr int pitch(int n) { return (n / 16) % 2 ? n : n + 16; }

// Lane layout of v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register q of lane l is D[l/16 + 4q][l%16].

// ---------------------------------------------------------------------------
// Phi transform of the moments.  Block: 128 rows x all NT column tiles of 16
// (the first NE the C columns), K = the kh cells (mirrored: the first half)
// in slabs of 16.  Thread t stages 8 consecutive cells of row t/2 (from
// (t%2)*8), and with MIR their 8 mirror cells, with their weights; and NT
// entries of the factor slab.  The next slab is loaded into registers while
// the current one is multiplied.
template <typename T>
struct PhiStage {
    T a[8], b[8];
    double wa[8], wb[8];
};

template <typename T, bool MIR>
__device__ inline void load_phi(PhiStage<T> &st, const T *row, const double *wr, int k, int n_phi, int kh,
                                bool row_ok) {
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
            st.wa[q] = row_ok ? wr[k + q] : 0.0;
            st.wb[q] = (MIR && row_ok) ? wr[n_phi - 1 - k - q] : 0.0;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool ok = row_ok && k + q < kh;
        st.a[q] = ok ? row[k + q] : (T)0;
        st.b[q] = (ok && MIR) ? row[n_phi - 1 - k - q] : (T)0;
        st.wa[q] = ok ? wr[k + q] : 0.0;
        st.wb[q] = (ok && MIR) ? wr[n_phi - 1 - k - q] : 0.0;
    }
}

template <typename T, bool MIR, int NT>
__global__ __launch_bounds__(256) void k_sep_phi1(const T *__restrict__ rho, const double *__restrict__ w,
                                                  size_t w_patch, const double *__restrict__ f1,
                                                  double *__restrict__ F, size_t ldF, size_t n_rows,
                                                  int rows_per_patch, int n_patches, int n_theta, int n_phi, int kh,
                                                  int ne) {
    constexpr int NC = NT * 16, PB = pitch(NC);
    __shared__ double Ae[SK][PA];
    __shared__ double Ao[MIR ? SK : 1][MIR ? PA : 1];
    __shared__ double Bs[SK][PB];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const size_t r0 = (size_t)blockIdx.x * RB;

    // this thread's staging row and cells
    const int sr = tid >> 1, sk = (tid & 1) * 8;
    const size_t r = r0 + sr;
    const bool row_ok = r < n_rows;
    const size_t rr = row_ok ? r : 0;
    const T *prow = rho + rr * n_phi;
    const double *wr = w + (rr / rows_per_patch % n_patches) * w_patch + (rr % n_theta) * n_phi;

    v4d acc[2][NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = v4d{0.0, 0.0, 0.0, 0.0};

    const int nsl = (kh + SK - 1) / SK;
    PhiStage<T> st;
    double bv[NT];
    auto load = [&](int s) {
        load_phi<T, MIR>(st, prow, wr, s * SK + sk, n_phi, kh, row_ok);
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int e = tid + 256 * q;
            bv[q] = f1[(size_t)(s * SK + e / NC) * NC + e % NC];
        }
    };
    load(0);
    const int wm = wave * 32;
    for (int s = 0; s < nsl; ++s) {
        // stage slab s
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double a = st.wa[q] * (double)st.a[q], b = st.wb[q] * (double)st.b[q];
            Ae[sk + q][sr] = a + b;
            if (MIR) Ao[sk + q][sr] = a - b;
        }
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int e = tid + 256 * q;
            Bs[e / NC][e % NC] = bv[q];
        }
        __syncthreads();
        if (s + 1 < nsl) load(s + 1);
#pragma unroll
        for (int kk = 0; kk < SK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double ae[2], ao[2], b[NT];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ae[i] = Ae[kr][wm + i * 16 + (lane & 15)];
                ao[i] = MIR ? Ao[kr][wm + i * 16 + (lane & 15)] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = Bs[kr][t * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[i][t] = mfma((MIR && t >= ne) ? ao[i] : ae[i], b[t], acc[i][t]);
        }
        __syncthreads();
    }

    // F[c][r]: register q of lane l is row l/16 + 4q of the 16-row tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const size_t row = r0 + wm + i * 16 + (lane >> 4) + 4 * q;
                if (row < n_rows) F[(size_t)(t * 16 + (lane & 15)) * ldF + row] = acc[i][t][q];
            }
}

// ---------------------------------------------------------------------------
// Theta contraction of the moments: block (64 rows v, phi column c):
// A[v][col(c, s)] = sum_j F[c][v * n_theta + j] t1[c][s][j] for the degree
// slots s < lmax + 1 - u (at most five tiles of 16), K = n_theta in slabs of
// 16.  Wave w takes rows 16w..16w+15.
__global__ __launch_bounds__(256) void k_sep_theta1(const double *__restrict__ F, size_t ldF,
                                                    const double *__restrict__ t1, const int *__restrict__ sep_u,
                                                    const int *__restrict__ sep_col, double *__restrict__ A, int rows,
                                                    int n_theta, int lp, int L, int lda) {
    constexpr int NTM = 5, PB = pitch(NTM * 16);
    __shared__ double As[SK][pitch(TR)];
    __shared__ double Bs[SK][PB];
    const int c = blockIdx.y, u = sep_u[c];
    if (u < 0) return;  // padding column (the whole block)
    const int nl = L + 1 - u, ntl = (nl + 15) / 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = blockIdx.x * TR;
    const double *Fc = F + (size_t)c * ldF;
    const double *tc = t1 + (size_t)c * lp * n_theta;

    v4d acc[NTM];
#pragma unroll
    for (int t = 0; t < NTM; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    // staging: A 64 rows x 16 (thread: row tid/4, 4 consecutive j);
    // B 16 x 80 (thread: slots tid/16 + 16q, j tid%16)
    const int ar = tid >> 2, aj = (tid & 3) * 4;
    const bool arow_ok = row0 + ar < rows;
    const double *fa = Fc + (size_t)(arow_ok ? row0 + ar : 0) * n_theta;
    for (int j0 = 0; j0 < n_theta; j0 += SK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + aj + q;
            As[aj + q][ar] = (arow_ok && j < n_theta) ? fa[j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NTM; ++q) {
            const int sl = (tid >> 4) + 16 * q, j = j0 + (tid & 15);
            Bs[tid & 15][sl] = (sl < lp && j < n_theta) ? tc[(size_t)sl * n_theta + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            const double a = As[kr][wave * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < NTM; ++t)
                if (t < ntl) acc[t] = mfma(a, Bs[kr][t * 16 + (lane & 15)], acc[t]);
        }
        __syncthreads();
    }
    const int *cols = sep_col + (size_t)c * lp;
#pragma unroll
    for (int t = 0; t < NTM; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = row0 + wave * 16 + (lane >> 4) + 4 * q, sl = t * 16 + (lane & 15);
            if (t < ntl && row < rows && sl < nl) A[(size_t)row * lda + cols[sl]] = acc[t][q];
        }
}

// ---------------------------------------------------------------------------
// Rotations of degree l (blockIdx.y), 64 rows of (field, shell) per block.
//   EXP = false (moments): B[row][perm[l^2 + o]] = sum over kk = (patch g,
//     position i) of A[(f, g, shell)][l^2 + i] x1[l][kk][o];  K = P (2l+1)
//   EXP = true (expansion, patch g = blockIdx.z):
//     L[(f, g, shell)][l^2 + o] = sum_i M[row][perm[l^2 + i]] x2[l][g][i][o];  K = 2l+1
// N = 2l + 1 in up to nine tiles of 16; wave w takes rows 16w..16w+15.
template <bool EXP>
__global__ __launch_bounds__(256) void k_sep_rot(const double *__restrict__ src, const double *__restrict__ x,
                                                 const long long *__restrict__ xoff, const int *__restrict__ perm,
                                                 double *__restrict__ dst, int rows, int n_r, int P, int n_lm,
                                                 int np) {
    constexpr int NB = kMaxTiles * 16;
    __shared__ double As[SK][pitch(TR)];
    __shared__ double Bs[SK][pitch(NB)];
    const int l = blockIdx.y, n = 2 * l + 1, nto = (n + 15) / 16, g = EXP ? blockIdx.z : 0;
    const int K = EXP ? n : P * n, l2 = l * l;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = blockIdx.x * TR;
    const double *xl = x + xoff[l] + (EXP ? (size_t)g * n * n : 0);

    v4d acc[kMaxTiles];
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    // staging: A 64 rows x 16 (thread: row tid/4, 4 consecutive kk); B 16 x
    // 144 (thread: entries tid + 256q)
    const int ar = tid >> 2, ak = (tid & 3) * 4;
    const int arow = row0 + ar;
    const bool arow_ok = arow < rows;
    const int af = arow_ok ? arow / n_r : 0, ash = arow_ok ? arow - af * n_r : 0;
    for (int k0 = 0; k0 < K; k0 += SK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = k0 + ak + q;
            double v = 0.0;
            if (arow_ok && kk < K) {
                if (EXP) {
                    v = src[(size_t)arow * np + perm[l2 + kk]];
                } else {
                    const int gi = kk / n, i = kk - gi * n;
                    v = src[((size_t)(af * P + gi) * n_r + ash) * n_lm + l2 + i];
                }
            }
            As[ak + q][ar] = v;
        }
#pragma unroll
        for (int q = 0; q < kMaxTiles; ++q) {
            const int e = tid + 256 * q, kr = e / NB, o = e - kr * NB, kk = k0 + kr;
            Bs[kr][o] = (kk < K && o < n) ? xl[(size_t)kk * n + o] : 0.0;
        }
        __syncthreads();
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
                dst[((size_t)(f * P + g) * n_r + sh) * n_lm + l2 + o] = acc[t][q];
            } else {
                dst[(size_t)row * np + perm[l2 + o]] = acc[t][q];
            }
        }
}

// ---------------------------------------------------------------------------
// Theta contraction of the expansion: block (64 rows v, 64 theta rows, phi
// column c): G[c][v * n_theta + j] = sum_s L[v][col(c, s)] t2[c][s][j], K =
// the degree slots in slabs of 16.  Wave w takes rows 32(w%2).. and theta
// rows 32(w/2)..
__global__ __launch_bounds__(256) void k_sep_theta2(const double *__restrict__ Lc, const double *__restrict__ t2,
                                                    const int *__restrict__ sep_u, const int *__restrict__ sep_col,
                                                    double *__restrict__ G, size_t ldF, int rows, int n_theta, int lp,
                                                    int L, int lda) {
    __shared__ double As[SK][pitch(TR)];
    __shared__ double Bs[SK][pitch(TR)];
    const int c = blockIdx.z, u = sep_u[c];
    if (u < 0) return;
    const int nl = L + 1 - u;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = blockIdx.x * TR, j0 = blockIdx.y * TR;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int *cols = sep_col + (size_t)c * lp;
    const double *tc = t2 + (size_t)c * lp * n_theta;

    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[i][t] = v4d{0.0, 0.0, 0.0, 0.0};
    // staging: A 64 rows x 16 slots (thread: row tid/4, slots 4(tid%4)..);
    // B 16 slots x 64 theta rows (thread: slot tid/16, rows 4(tid%16)..)
    const int ar = tid >> 2, as = (tid & 3) * 4, bs = tid >> 4, bj = (tid & 15) * 4;
    const bool arow_ok = row0 + ar < rows;
    const double *la = Lc + (size_t)(arow_ok ? row0 + ar : 0) * lda;
    for (int s0 = 0; s0 < nl; s0 += SK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sl = s0 + as + q;
            As[as + q][ar] = (arow_ok && sl < nl) ? la[cols[sl]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sl = s0 + bs, j = j0 + bj + q;
            Bs[bs][bj + q] = (sl < nl && j < n_theta) ? tc[(size_t)sl * n_theta + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 2; ++t) b[t] = Bs[kr][wn + t * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int t = 0; t < 2; ++t) acc[i][t] = mfma(a[i], b[t], acc[i][t]);
        }
        __syncthreads();
    }
    double *Gc = G + (size_t)c * ldF;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = row0 + wm + i * 16 + (lane >> 4) + 4 * q, j = j0 + wn + t * 16 + (lane & 15);
                if (row < rows && j < n_theta) Gc[(size_t)row * n_theta + j] = acc[i][t][q];
            }
}

// ---------------------------------------------------------------------------
// Phi transform of the expansion: block (128 rows, 64 evaluation points b):
// E = the sum over the C columns, O over the S columns (with MIR; else all
// columns go to E); Phi[r][kxy[b].x] = E + O and, with a mirror cell,
// Phi[r][kxy[b].y] = E - O.  K = the phi columns in slabs of 16.  Wave w
// takes rows 32w.. and all 64 points.  Thread t stages 8 rows of phi column
// t/16 (from (t%16)*8) and 4 points of factor row t/16.
template <typename T, bool MIR>
__global__ __launch_bounds__(256) void k_sep_phi2(const double *__restrict__ G, size_t ldF,
                                                  const double *__restrict__ f2, const int2 *__restrict__ kxy,
                                                  T *__restrict__ phi, size_t n_rows, int n_phi, int kx, int ce,
                                                  int co) {
    __shared__ double As[SK][PA];
    __shared__ double Bs[SK][pitch(64)];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const size_t r0 = (size_t)blockIdx.x * RB;
    const int b0 = blockIdx.y * 64, wm = wave * 32;
    const int sc = tid >> 4, sr = (tid & 15) * 8, sb = (tid & 15) * 4;

    v4d E[2][4], O[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) E[i][t] = O[i][t] = v4d{0.0, 0.0, 0.0, 0.0};

    const int nsl = (ce + co) / SK, nse = ce / SK;
    double av[8], bv[4];
    auto load = [&](int s) {
        // G rows past n_rows lie inside the padded work array and feed only
        // output rows that are not stored
        const double *g = G + (size_t)(s * SK + sc) * ldF + r0 + sr;
#pragma unroll
        for (int q = 0; q < 8; ++q) av[q] = g[q];
        const double *f = f2 + (size_t)(s * SK + sc) * kx;
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] = b0 + sb + q < kx ? f[b0 + sb + q] : 0.0;
    };
    // slabs [s0, s1) into acc; the first slab's operands are in registers
    auto run = [&](v4d(&acc)[2][4], int s0, int s1) {
        for (int s = s0; s < s1; ++s) {
#pragma unroll
            for (int q = 0; q < 8; ++q) As[sc][sr + q] = av[q];
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[sc][sb + q] = bv[q];
            __syncthreads();
            if (s + 1 < nsl) load(s + 1);
#pragma unroll
            for (int kk = 0; kk < SK / 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                double a[2], b[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
                for (int t = 0; t < 4; ++t) b[t] = Bs[kr][t * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[i][t] = mfma(a[i], b[t], acc[i][t]);
            }
            __syncthreads();
        }
    };
    load(0);
    run(E, 0, MIR ? nse : nsl);
    if (MIR) run(O, nse, nsl);

#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int b = b0 + t * 16 + (lane & 15);
        if (b >= kx) continue;
        const int2 kk = kxy[b];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const size_t row = r0 + wm + i * 16 + (lane >> 4) + 4 * q;
                if (row >= n_rows) continue;
                T *o = phi + row * n_phi;
                const double e = E[i][t][q], d = O[i][t][q];
                o[kk.x] = (T)(e + d);
                if (MIR && kk.y >= 0) o[kk.y] = (T)(e - d);
            }
    }
}

template <typename T, bool MIR>
hipError_t launch_phi1(const Plan &p, dim3 grid, const T *rho, size_t n_rows) {
    const int nt = p.sep_nc() / 16, ne = p.sep_ce / 16, rpp = p.n_r * p.n_theta;
    const size_t w_patch = p.npat == 1 ? 0 : (size_t)p.n_ang;
#define MPG_PHI1(N)                                                                                                 \
    case N:                                                                                                         \
        hipLaunchKernelGGL((k_sep_phi1<T, MIR, N>), grid, dim3(256), 0, p.stream, rho, p.w, w_patch, p.sep_f1,      \
                           p.sep_F, p.sep_rows(), n_rows, rpp, p.n_patches, p.n_theta, p.n_phi, p.sep_kh, ne);       \
        break;
    switch (nt) {
        MPG_PHI1(1)
        MPG_PHI1(2)
        MPG_PHI1(3)
        MPG_PHI1(4)
        MPG_PHI1(5)
        MPG_PHI1(6)
        MPG_PHI1(7)
        MPG_PHI1(8)
        MPG_PHI1(9)
    default:
        return hipErrorInvalidValue;
    }
#undef MPG_PHI1
    return hipGetLastError();
}

template <typename T, bool MIR>
void launch_phi2(const Plan &p, dim3 grid, T *phi, size_t n_rows) {
    hipLaunchKernelGGL((k_sep_phi2<T, MIR>), grid, dim3(256), 0, p.stream, p.sep_F, p.sep_rows(), p.sep_f2,
                       p.sep_kxy, phi, n_rows, p.n_phi, p.sep_kx, p.sep_ce, p.sep_co);
}

}  // namespace

hipError_t sep_phi_moments(const Plan &p, int n_fields, const void *rho, int rho_dtype) {
    const size_t n_rows = (size_t)n_fields * p.n_patches * p.n_r * p.n_theta;
    if (n_rows > p.sep_rows()) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n_rows + RB - 1) / RB));
    if (rho_dtype == MPG_F64)
        return p.sep_mir ? launch_phi1<double, true>(p, grid, (const double *)rho, n_rows)
                         : launch_phi1<double, false>(p, grid, (const double *)rho, n_rows);
    return p.sep_mir ? launch_phi1<float, true>(p, grid, (const float *)rho, n_rows)
                     : launch_phi1<float, false>(p, grid, (const float *)rho, n_rows);
}

hipError_t sep_theta_moments(const Plan &p, int n_fields) {
    const int vrows = n_fields * p.n_patches * p.n_r, rows = n_fields * p.n_r;
    if (p.sep_lp > 80 || p.lmax > 64) return hipErrorInvalidValue;  // five slot tiles, nine degree tiles
    hipLaunchKernelGGL(k_sep_theta1, dim3((vrows + TR - 1) / TR, p.sep_nc()), dim3(256), 0, p.stream, p.sep_F,
                       p.sep_rows(), p.sep_t1, p.sep_m, p.sep_col, p.sep_A, vrows, p.n_theta, p.sep_lp, p.lmax,
                       p.n_lm);
    hipLaunchKernelGGL(k_sep_rot<false>, dim3((rows + TR - 1) / TR, p.lmax + 1), dim3(256), 0, p.stream, p.sep_A,
                       p.sep_x1, p.sep_xoff, p.sep_perm, p.Bpart, rows, p.n_r, p.n_patches, p.n_lm, p.np);
    return hipGetLastError();
}

hipError_t sep_expansion(const Plan &p, int n_fields, void *phi, int phi_dtype) {
    const int vrows = n_fields * p.n_patches * p.n_r, rows = n_fields * p.n_r;
    const size_t n_rows = (size_t)vrows * p.n_theta;
    if (n_rows > p.sep_rows() || p.lmax > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sep_rot<true>, dim3((rows + TR - 1) / TR, p.lmax + 1, p.n_patches), dim3(256), 0,
                       p.stream, p.M, p.sep_x2, p.sep_xoff, p.sep_perm, p.sep_A, rows, p.n_r, p.n_patches, p.n_lm,
                       p.np);
    hipLaunchKernelGGL(k_sep_theta2, dim3((vrows + TR - 1) / TR, (p.n_theta + TR - 1) / TR, p.sep_nc()), dim3(256),
                       0, p.stream, p.sep_A, p.sep_t2, p.sep_m, p.sep_col, p.sep_F, p.sep_rows(), vrows, p.n_theta,
                       p.sep_lp, p.lmax, p.n_lm);
    dim3 grid((unsigned)((n_rows + RB - 1) / RB), (p.sep_kx + 63) / 64);
    if (phi_dtype == MPG_F64) {
        if (p.sep_mir) launch_phi2<double, true>(p, grid, (double *)phi, n_rows);
        else launch_phi2<double, false>(p, grid, (double *)phi, n_rows);
    } else {
        if (p.sep_mir) launch_phi2<float, true>(p, grid, (float *)phi, n_rows);
        else launch_phi2<float, false>(p, grid, (float *)phi, n_rows);
    }
    return hipGetLastError();
}

}  // namespace mpg
