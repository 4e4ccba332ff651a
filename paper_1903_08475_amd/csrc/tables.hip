// FP64 table build of a plan (Sec. 4.3 step 1): Wigner d at pi/2 by the
// recursions of Sec. 3, d(beta) by their Fourier sum, the angular integrals
// T, C, S (Eqs. T_lm, C_k^m, S_k^m), the normalisation factors
// (Eqs. N_CC..N_SC), the angular weights U (Eqs. U_C/U_S), the prefactors Q
// (Eqs. Q_C/Q_S), the overlap weights w (Sec. 4.2) and the radial
// recurrence coefficients of Eq. M_C.  Everything runs on the device in
// FP64; the host only validates, lays out columns and launches.
#include <cmath>
#include <vector>

#include "mpg_internal.h"

namespace mpg {
namespace {

__host__ __device__ inline int off_dh(int l) { return (l - 1) * l * (2 * l - 1) / 3 + 3 * l * (l - 1) / 2 + l; }
__host__ __device__ inline int off_sq(int l) { return l * (l + 1) * (2 * l + 1) / 6; }
__host__ __device__ inline int off_tri(int l) { return l * (l + 1) / 2; }

__device__ inline int tri_row(int t) {
    int l = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (off_tri(l + 1) <= t) ++l;
    while (off_tri(l) > t) --l;
    return l;
}

// d^l_{m'm}(pi/2) for -l <= m' <= l, 0 <= m <= l, stored at
// dh[off_dh(l) + (m'+l)(l+1) + m].  Apex d^0_00 = 1; the diagonal seeds
// d^l_{l0} = -sqrt((2l-1)/(2l)) d^{l-1}_{l-1,0} and
// d^l_{lm} = +sqrt(l(2l-1)/(2(l+m)(l+m-1))) d^{l-1}_{l-1,m-1} (m >= 1; the
// sign printed with this recursion in Sec. 3 gives the wrong sign of
// d^1_11(pi/2) = 1/2 and is not used); the three-term recursion runs down
// in m' only to m' = 0, and m' < 0 is filled from
// d_{-m',m}(pi/2) = (-1)^{l+m} d_{m'm}(pi/2) (the second symmetry of
// Sec. 3 at beta = pi/2), since continuing the recursion below 0 loses
// all accuracy at high l.
__global__ void k_dhalf(int L, double *dh) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= off_tri(L + 1)) return;
    int l = tri_row(t), m = t - off_tri(l);
    double v = 1.0;
    for (int lp = 1; lp <= l - m; ++lp) v *= -sqrt((2.0 * lp - 1.0) / (2.0 * lp));
    for (int k = 1; k <= m; ++k) {
        int lp = l - m + k;
        v *= sqrt(lp * (2.0 * lp - 1.0) / (2.0 * (lp + k) * (lp + k - 1.0)));
    }
    double *d = dh + off_dh(l);
    const int W = l + 1;
    d[(2 * l) * W + m] = v;
    double n1 = v, n2 = 0.0;
    for (int j = l - 1; j >= 0; --j) {
        double q = (double)(l - j) * (l + j + 1);
        double val = 2.0 * m / sqrt(q) * n1 - sqrt((double)(l - j - 1) * (l + j + 2) / q) * n2;
        d[(j + l) * W + m] = val;
        n2 = n1;
        n1 = val;
    }
    double sgn = ((l + m) & 1) ? -1.0 : 1.0;
    for (int j = 1; j <= l; ++j) d[(l - j) * W + m] = sgn * d[(l + j) * W + m];
}

// Re[i^n (x + i y)]
__device__ inline double re_ipow(int n, double x, double y) {
    n &= 3;
    return n == 0 ? x : n == 1 ? -y : n == 2 ? -x : y;
}

// d^l_{m'm}(beta) = i^{m-m'} sum_u d_{u m'}(pi/2) d_{u m}(pi/2) e^{i u beta}
// for 0 <= m', m <= l at two angles; db[b][off_sq(l) + m'(l+1) + m].
__global__ void k_dbeta(int L, const double *dh, double beta0, double beta1, double *db) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int per = off_sq(L + 1);
    if (t >= 2 * per) return;
    int b = t / per, r = t - b * per;
    int l = 0;
    while (off_sq(l + 1) <= r) ++l;
    int rr = r - off_sq(l), mp = rr / (l + 1), m = rr - mp * (l + 1);
    double beta = b ? beta1 : beta0;
    const double *d = dh + off_dh(l);
    const int W = l + 1;
    double x = 0.0, y = 0.0;
    for (int u = -l; u <= l; ++u) {
        double p = d[(u + l) * W + mp] * d[(u + l) * W + m];
        double s, c;
        sincos(u * beta, &s, &c);
        x += p * c;
        y += p * s;
    }
    db[b * per + r] = re_ipow(m - mp, x, y);
}

// Bracketed parts of Eqs. N_CC..N_SC (without 2/delta_m, mu_m and the
// factor s_lu, which the T table carries): N4[(off_sq(l) + m(l+1) + u)*4 + c]
// with c = CC, CS, SS, SC.
__global__ void k_ncoef(int L, const double *db, double alpha, double gamma, double *N4) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int per = off_sq(L + 1);
    if (t >= per) return;
    int l = 0;
    while (off_sq(l + 1) <= t) ++l;
    int rr = t - off_sq(l), m = rr / (l + 1), u = rr - m * (l + 1);
    double d0 = db[off_sq(l) + u * (l + 1) + m];        // d_{um}(beta)
    double d1 = db[per + off_sq(l) + u * (l + 1) + m];  // d_{um}(pi - beta)
    double mu = u > 0 ? 1.0 : 0.0;
    double sg = ((l + m + u) & 1) ? -1.0 : 1.0;
    double sp, cp, sm, cm;
    sincos(m * gamma + u * alpha, &sp, &cp);
    sincos(m * gamma - u * alpha, &sm, &cm);
    double *o = N4 + 4 * (size_t)t;
    o[0] = cp * d0 + mu * sg * cm * d1;
    o[1] = sp * d0 - mu * sg * sm * d1;
    o[2] = cp * d0 - mu * sg * cm * d1;
    o[3] = sp * d0 + mu * sg * sm * d1;
}

// s_lu T_j^{lu} = int_{theta_j^-}^{theta_j^+} sin t d^l_{u0}(t) dt, with
// d_{u0}(t) = s_lu P_l^u(cos t) written as its Fourier sum; each
// int sin t e^{ivt} dt is closed form.  Tt[j][off_tri(l) + u].
__global__ void k_ttilde(int L, const double *dh, int n_theta, double theta0, double dtheta, double *Tt) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int per = off_tri(L + 1);
    if (t >= n_theta * per) return;
    int j = t / per, r = t - j * per;
    int l = tri_row(r), u = r - off_tri(l);
    double h = 0.5 * dtheta, tm = theta0 + (j + 0.5) * dtheta;
    const double *d = dh + off_dh(l);
    const int W = l + 1;
    double sx = 0.0, sy = 0.0;
    for (int v = -l; v <= l; ++v) {
        // E(k) = int e^{ikt} dt = e^{ik tm} 2 sin(kh)/k ; J = (E(v+1)-E(v-1))/(2i)
        double er[2], ei[2];
        for (int q = 0; q < 2; ++q) {
            int k = q ? v - 1 : v + 1;
            double amp = (k == 0) ? 2.0 * h : 2.0 * sin(k * h) / k;
            double s, c;
            sincos(k * tm, &s, &c);
            er[q] = amp * c;
            ei[q] = amp * s;
        }
        double jr = 0.5 * (ei[0] - ei[1]), ji = -0.5 * (er[0] - er[1]);
        double p = d[(v + l) * W + u] * d[(v + l) * W + 0];
        sx += p * jr;
        sy += p * ji;
    }
    Tt[t] = re_ipow(-u, sx, sy);
}

// C_k^u and S_k^u (Eqs. C_k^m, S_k^m): CS[(k(L+1)+u)*2 + {0,1}]
__global__ void k_cs(int L, int n_phi, double phi0, double dphi, double *CS) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_phi * (L + 1)) return;
    int k = t / (L + 1), u = t - k * (L + 1);
    double h = 0.5 * dphi, pm = phi0 + (k + 0.5) * dphi;
    double c = dphi, s = 0.0;
    if (u > 0) {
        double a = 2.0 * sin(u * h) / u, sn, cs;
        sincos(u * pm, &sn, &cs);
        c = a * cs;
        s = a * sn;
    }
    CS[2 * t] = c;
    CS[2 * t + 1] = s;
}

__device__ inline void decode_col(int src, int &l, int &m, int &is_s) {
    l = (int)sqrt((double)src);
    while ((l + 1) * (l + 1) <= src) ++l;
    while (l * l > src) --l;
    int rem = src - l * l;
    m = (rem + 1) / 2;
    is_s = (rem > 0 && (rem & 1) == 0);
}

// Eqs. U_C/U_S with the prefactor 2/delta_m of Eq. del_m:
//   U_C = (2/delta_m) w sum_u (N_CC C_k^u + N_CS S_k^u) s_lu T_j^{lu}
//   U_S = 2 w sum_u (N_SS S_k^u - N_SC C_k^u) s_lu T_j^{lu}   (m >= 1)
// (the text prints 2/lambda_{m'm}, which is 2 also for m = 0, m' > 0 and
// then doubles those terms; 2/delta_m is what the real form of
// Eq. phispherical requires).  Ut[q][off + jk] (row length ld), zero on
// padding; w holds the n_ang weights of this patch.
__global__ void k_U(int L, int np_alloc, int n_angp, int n_ang, int n_phi, const int *col_src,
                    const double *Tt, const double *CS, const double *N4, const double *w, size_t ld,
                    size_t off, double *Ut) {
    int jk = blockIdx.x * blockDim.x + threadIdx.x;
    int q = blockIdx.y;
    if (jk >= n_angp || q >= np_alloc) return;
    int src = col_src[q];
    double val = 0.0;
    if (src >= 0 && jk < n_ang) {
        int l, m, is_s;
        decode_col(src, l, m, is_s);
        int j = jk / n_phi, k = jk - j * n_phi;
        const double *T = Tt + (size_t)j * off_tri(L + 1) + off_tri(l);
        const double *cs = CS + (size_t)k * (L + 1) * 2;
        const double *N = N4 + 4 * (size_t)(off_sq(l) + m * (l + 1));
        double s = 0.0;
        for (int u = 0; u <= l; ++u) {
            double c = cs[2 * u], sn = cs[2 * u + 1];
            double f = is_s ? (N[4 * u + 2] * sn - N[4 * u + 3] * c) : (N[4 * u + 0] * c + N[4 * u + 1] * sn);
            s += f * T[u];
        }
        val = (m == 0 ? 1.0 : 2.0) * w[jk] * s;
    }
    Ut[(size_t)q * ld + off + jk] = val;
}

struct Rot {
    double r[9];
};

// Eqs. Q_C/Q_S at the upper vertex of every cell of patch 0 (ev = 1), or at
// its angular centre (ev = 1/2):
//   Q = -G s_lm P_l^m(cos theta) {cos, sin}(m phi)
// with (theta, phi) the global angles of x = R xi.  The normalised
// functions s_lm P_l^m come from the recurrences of the normalised
// associated Legendre functions (Condon-Shortley phase).  Qt[jk][perm].
__global__ void k_Q(int L, int np, int n_angp, int n_ang, int n_phi, double theta0, double phi0,
                    double dtheta, double dphi, double ev, Rot R, double G, const int *perm_of, size_t ld,
                    double *Qt) {
    int jk = blockIdx.x * blockDim.x + threadIdx.x;
    if (jk >= n_angp) return;
    double *row = Qt + (size_t)jk * ld;
    if (jk >= n_ang) {
        for (int q = 0; q < np; ++q) row[q] = 0.0;
        return;
    }
    int j = jk / n_phi, k = jk - j * n_phi;
    double st, ct, sp, cp;
    sincos(theta0 + (j + ev) * dtheta, &st, &ct);
    sincos(phi0 + (k + ev) * dphi, &sp, &cp);
    double xi = st * cp, et = st * sp, ze = ct;
    double x = R.r[0] * xi + R.r[1] * et + R.r[2] * ze;
    double y = R.r[3] * xi + R.r[4] * et + R.r[5] * ze;
    double z = R.r[6] * xi + R.r[7] * et + R.r[8] * ze;
    double rho = sqrt(x * x + y * y), rr = sqrt(rho * rho + z * z);
    double cth = z / rr, sth = rho / rr, ph = atan2(y, x);
    double pmm = 1.0;
    for (int m = 0; m <= L; ++m) {
        if (m > 0) pmm *= -sqrt((2.0 * m - 1.0) / (2.0 * m)) * sth;
        double sm, cm;
        sincos(m * ph, &sm, &cm);
        double p2 = 0.0, p1 = pmm;
        for (int l = m; l <= L; ++l) {
            double p;
            if (l == m) p = pmm;
            else if (l == m + 1) p = cth * sqrt(2.0 * m + 1.0) * pmm;
            else p = (cth * (2.0 * l - 1.0) * p1 - sqrt((double)(l - 1) * (l - 1) - (double)m * m) * p2) /
                     sqrt((double)l * l - (double)m * m);
            if (l > m) { p2 = p1; p1 = p; }
            if (m == 0) {
                row[perm_of[l * l]] = -G * p;
            } else {
                row[perm_of[l * l + 2 * m - 1]] = -G * p * cm;
                row[perm_of[l * l + 2 * m]] = -G * p * sm;
            }
        }
    }
}

// ---- overlap weights -----------------------------------------------------
// For a Yin point at local (theta, phi), the other patch's local
// coordinates are (-xi, zeta, eta) (Eq. caryytransform).  For patches
// spanning [pi/2-c, pi/2+c] x [-phe, phe] it is covered iff
//   sin theta |sin phi| <= sc           (sc = cos(pi/2 - c))
//   sin theta cos phi   <= kap |cos theta|   (kap = cot(pi - phe))
// At fixed phi the covered colatitudes are [0, X] u [pi - X, pi] with
// cos X = max(g1(phi), g2(phi)),
//   g1 = sqrt(max(0, 1 - sc^2/sin^2 phi)),  g2 = max(0, cos phi)/sqrt(cos^2 phi + kap^2).
// The covered area of a cell is the phi-integral of a piecewise function of
// cos X, split where its form changes, each piece integrated in closed form:
//   int g1 dphi = -+ G(cos phi),  G(u) = pi/2 - psi - sc atan2(sc cos psi, sin psi),
//                                  u = a cos psi, a^2 = 1 - sc^2  (sign: -sin phi)
//   int g2 dphi = asin(sin phi / sqrt(1 + kap^2)).
struct OvlGeom {
    double sc, kap;
    int kap_inf;
};

__device__ inline double ovl_g1(double p, double sc) {
    double s = sin(p);
    double v = (s == 0.0) ? -1.0 : 1.0 - sc * sc / (s * s);
    return v > 0.0 ? sqrt(v) : 0.0;
}
__device__ inline double ovl_g2(double p, const OvlGeom &o) {
    if (o.kap_inf) return 0.0;
    double c = cos(p);
    return c > 0.0 ? c / sqrt(c * c + o.kap * o.kap) : 0.0;
}
__device__ inline double ovl_F1(double p, double sc) {
    double a = sqrt(1.0 - sc * sc);
    double u = cos(p) / a;
    u = u > 1.0 ? 1.0 : (u < -1.0 ? -1.0 : u);
    double psi = acos(u);
    double G = 0.5 * M_PI - psi - sc * atan2(sc * cos(psi), sin(psi));
    return sin(p) > 0.0 ? -G : G;
}
__device__ inline double ovl_F2(double p, double kap) { return asin(sin(p) / sqrt(1.0 + kap * kap)); }

__device__ inline void push_s(double s, double *c, int &n) {
    if (s >= 0.0 && s <= 1.0) {
        double b = asin(s);
        c[n++] = b; c[n++] = -b; c[n++] = M_PI - b; c[n++] = -M_PI + b;
    }
}
__device__ inline void push_c(double v, double *c, int &n) {
    if (v >= -1.0 && v <= 1.0) {
        double b = acos(v);
        c[n++] = b; c[n++] = -b;
    }
}

__global__ void k_overlap(int n_theta, int n_phi, double theta0, double phi0, double dtheta, double dphi,
                          OvlGeom o, double *w) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_theta * n_phi) return;
    int j = t / n_phi, k = t - j * n_phi;
    double t1 = theta0 + j * dtheta, t2 = t1 + dtheta;
    double p1 = phi0 + k * dphi, p2 = p1 + dphi;
    double c1 = cos(t1), c2 = cos(t2);
    double cand[48];
    int n = 0;
    cand[n++] = p1;
    cand[n++] = p2;
    push_s(o.sc, cand, n);
    push_c(0.0, cand, n);
    if (!o.kap_inf) push_s(sqrt(o.sc * o.sc * (1.0 + o.kap * o.kap) / (o.kap * o.kap + o.sc * o.sc)), cand, n);
    double vs[4] = {c1, c2, -c1, -c2};
    for (int q = 0; q < 4; ++q) {
        double v = vs[q];
        if (v > 0.0 && v < 1.0) {
            push_s(o.sc / sqrt(1.0 - v * v), cand, n);
            if (!o.kap_inf) push_c(v * o.kap / sqrt(1.0 - v * v), cand, n);
        }
    }
    // keep points inside [p1, p2], sort
    int m = 0;
    for (int q = 0; q < n; ++q)
        if (cand[q] >= p1 && cand[q] <= p2) cand[m++] = cand[q];
    for (int a = 1; a < m; ++a)
        for (int b = a; b > 0 && cand[b - 1] > cand[b]; --b) {
            double tmp = cand[b]; cand[b] = cand[b - 1]; cand[b - 1] = tmp;
        }
    double area = 0.0;
    for (int q = 0; q + 1 < m; ++q) {
        double pa = cand[q], pb = cand[q + 1];
        if (!(pb > pa)) continue;
        double pm = 0.5 * (pa + pb);
        double x1 = ovl_g1(pm, o.sc), x2 = ovl_g2(pm, o);
        int act = (x1 == 0.0 && x2 == 0.0) ? 0 : (x1 >= x2 ? 1 : 2);
        double cx = x1 > x2 ? x1 : x2;
        double C0 = 0.0;
        int cnt = 0;
        // [cos t1 - clamp(cX, c2, c1)] + [clamp(-cX, c2, c1) - cos t2]
        if (cx < c2) C0 += c1 - c2;
        else if (cx <= c1) { C0 += c1; ++cnt; }
        if (-cx > c1) C0 += c1 - c2;
        else if (-cx >= c2) { C0 += -c2; ++cnt; }
        double I = 0.0;
        if (cnt && act == 1) I = ovl_F1(pb, o.sc) - ovl_F1(pa, o.sc);
        else if (cnt && act == 2) I = ovl_F2(pb, o.kap) - ovl_F2(pa, o.kap);
        area += C0 * (pb - pa) - cnt * I;
    }
    w[t] = 1.0 - 0.5 * area / ((p2 - p1) * (c1 - c2));
}

__global__ void k_fill(double *p, size_t n, double v) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// Radial recurrence coefficients (Eq. M_C written with ratios <= 1):
//   y_n = a_n y_{n-1} + b_n B_n,   z_n = c_n z_{n+1} + e_n B_{n+1},  M_n = y_n + z_n
//   a_n = (r_{n-1}^+/r_n^+)^{l+1},          b_n = R_in,n/(r_n^+)^{l+1}
//   c_n = (r_n^+/r_{n+1}^+)^l,               e_n = (r_n^+)^l R_out,n+1
// (Eqs. R_in, R_out; l = 2 gives the logarithm).  coef[(n(L+1)+l)*4 + .]
__global__ void k_coef(int n_r, int L, const double *re, double *coef) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_r * (L + 1)) return;
    int n = t / (L + 1), l = t - n * (L + 1);
    double rm = re[n], rp = re[n + 1];
    double ratio = rm / rp;
    double a = pow(ratio, (double)(l + 1));
    double b = (ratio == 0.0) ? rp * rp / (l + 3.0) : -rp * rp * expm1((l + 3.0) * log(ratio)) / (l + 3.0);
    double c = 0.0, e = 0.0;
    if (n + 1 < n_r) {
        double rn = rp, rq = re[n + 2];
        c = pow(rn / rq, (double)l);
        double lg = log(rq / rn);
        e = (l == 2) ? rn * rn * lg : rn * rn * expm1((2.0 - l) * lg) / (2.0 - l);
    }
    double *o = coef + 4 * (size_t)t;
    o[0] = a; o[1] = b; o[2] = c; o[3] = e;
}

// x = hi + mid + lo, each piece the round-to-nearest bf16 of the remaining
// FP64 residual (24 significant bits in all), written as tile-slab blocks.
// Thread = one 16-byte chunk (8 consecutive K) of one row of a block.  Tile
// t < tiles_e holds source rows t*128 .. (end e_end), tile t >= tiles_e
// rows o0 + (t - tiles_e)*128 .. (end o_end); rows past a tile's end are 0.
__global__ void k_tile_split(const double *__restrict__ src, size_t ld, int slabs, int tiles_e, int e_end, int o0,
                             int o_end, size_t n_threads, bf16 *__restrict__ dst) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_threads) return;
    const size_t blk = t / 512;
    const int c = (int)(t - blk * 512);
    const int tile = (int)(blk / slabs), slab = (int)(blk - (size_t)tile * slabs);
    const int r = c >> 2, kc = (c & 3) ^ ((r >> 2) & 3);
    const int row = (tile < tiles_e ? tile * kSplitTile : o0 + (tile - tiles_e) * kSplitTile) + r;
    const int end = tile < tiles_e ? e_end : o_end;
    const double *x = src + (size_t)row * ld + (size_t)slab * kSlabK + kc * 8;
    uint32_t hm[3][4];
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        uint32_t w[3] = {0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const double v = row < end ? x[q + u] : 0.0;
            const bf16 h = (bf16)(float)v;
            const double r1 = v - (double)(float)h;
            const bf16 m = (bf16)(float)r1;
            const bf16 l = (bf16)(float)(r1 - (double)(float)m);
            w[0] |= (uint32_t)__builtin_bit_cast(uint16_t, h) << (16 * u);
            w[1] |= (uint32_t)__builtin_bit_cast(uint16_t, m) << (16 * u);
            w[2] |= (uint32_t)__builtin_bit_cast(uint16_t, l) << (16 * u);
        }
        hm[0][q / 2] = w[0];
        hm[1][q / 2] = w[1];
        hm[2][q / 2] = w[2];
    }
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    bf16 *o = dst + blk * 3 * kBlk + (size_t)c * 8;
#pragma unroll
    for (int pc = 0; pc < 3; ++pc) *(u32x4 *)(o + pc * kBlk) = (u32x4){hm[pc][0], hm[pc][1], hm[pc][2], hm[pc][3]};
}

// Tables of every patch in the real index (patch 1 = (-1)^m patch 0 under
// the fold): U[g][jk][n_lm] from Ut[q][jk], Q[g][jk][n_lm] from Qt[jk][q].
// Under the fold patch 1 is (-1)^m patch 0; on the general path patch g
// is column block g of Ut and row block g of Qt; for the per-patch method
// every patch has the one local U, and its Q in its own frame sits at row
// block g, column block g.
__global__ void k_export(const double *Ut, const double *Qt, int np, int n_angp, int n_ang, int n_lm,
                         int n_patches, int npat, int fold, int per_patch, size_t ldq, const int *col_src,
                         double *U, double *Q) {
    int jk = blockIdx.x * blockDim.x + threadIdx.x;
    int q = blockIdx.y;
    if (jk >= n_ang || q >= np) return;
    int src = col_src[q];
    if (src < 0) return;
    int l = (int)sqrt((double)src);
    while ((l + 1) * (l + 1) <= src) ++l;
    while (l * l > src) --l;
    int m = (src - l * l + 1) / 2;
    const size_t ldu = (size_t)npat * n_angp;
    for (int g = 0; g < n_patches; ++g) {
        const int ub = npat == 1 ? 0 : g, qr = (npat > 1 || per_patch) ? g : 0, qc = per_patch ? g : 0;
        double sg = (fold && g == 1 && (m & 1)) ? -1.0 : 1.0;
        double u = Ut[(size_t)q * ldu + (size_t)ub * n_angp + jk];
        double v = Qt[((size_t)qr * n_angp + jk) * ldq + (size_t)qc * np + q];
        size_t o = ((size_t)g * n_ang + jk) * n_lm + src;
        if (U) U[o] = sg * u;
        if (Q) Q[o] = sg * v;
    }
}

// ---- factors of the separable method ------------------------------------
// In each patch's own frame its cell weights factor over (theta, phi) (Eqs.
// a_ci^lm, a_si^lm): the local moments are A^(lu) = sum_jk w_jk rho_jk
// s_lu T_j^{lu} {C_k^u, S_k^u}, and the rotation sums of Eqs. U_C/U_S take
// them to the common frame degree by degree.  A phi column c has
// code[c] = 2 u + (0 for C, 1 for S), -1 on padding: the order-0 column,
// the C columns of u = 1..lmax, then the S columns of u = 1..lmax.

// f1[k][c] = C_k^u or S_k^u for the first kh cells (zero past them)
__global__ void k_sep_f1(int L, int kh, int khp, int nc, const int *code, const double *CS, double *f1) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= khp * nc) return;
    int k = t / nc, c = t - k * nc, cd = code[c];
    f1[t] = (cd < 0 || k >= kh) ? 0.0 : CS[((size_t)k * (L + 1) + (cd >> 1)) * 2 + (cd & 1)];
}

// f2[c][b] = cos or sin of u phi at the evaluation point of the cell kx[b]
__global__ void k_sep_f2(int kxn, int nc, double phi0, double dphi, double ev, const int *code, const int2 *kx,
                         double *f2) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc * kxn) return;
    int c = t / kxn, b = t - c * kxn, cd = code[c];
    double v = 0.0;
    if (cd >= 0) {
        double s, co;
        sincos((cd >> 1) * (phi0 + (kx[b].x + ev) * dphi), &s, &co);
        v = (cd & 1) ? s : co;
    }
    f2[t] = v;
}

// t1[c][l - u][j] = s_lu T_j^{lu}, zero past lmax and on padding
__global__ void k_sep_t1(int L, int n_theta, int nc, int lp, const int *code, const double *Tt, double *t1) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nc * lp * n_theta) return;
    int j = (int)(t % n_theta), r = (int)(t / n_theta), slot = r % lp, c = r / lp, cd = code[c];
    double v = 0.0;
    if (cd >= 0) {
        int u = cd >> 1, l = u + slot;
        if (l <= L) v = Tt[(size_t)j * off_tri(L + 1) + off_tri(l) + u];
    }
    t1[t] = v;
}

// t2[c][l - u][j] = -G s_lu P_l^u(cos theta) at the evaluation colatitude of
// row j (normalised associated Legendre recurrences, Condon-Shortley phase,
// as for Eqs. Q_C/Q_S); one thread per (column, row)
__global__ void k_sep_t2(int L, int n_theta, int nc, int lp, double theta0, double dtheta, double ev, double G,
                         const int *code, double *t2) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc * n_theta) return;
    int c = t / n_theta, j = t - c * n_theta, cd = code[c];
    double *o = t2 + (size_t)c * lp * n_theta + j;
    for (int slot = 0; slot < lp; ++slot) o[(size_t)slot * n_theta] = 0.0;
    if (cd < 0) return;
    const int m = cd >> 1;
    double sth, cth;
    sincos(theta0 + (j + ev) * dtheta, &sth, &cth);
    double pmm = 1.0;
    for (int u = 1; u <= m; ++u) pmm *= -sqrt((2.0 * u - 1.0) / (2.0 * u)) * sth;
    double p2 = 0.0, p1 = pmm;
    for (int l = m; l <= L; ++l) {
        double pl;
        if (l == m) pl = pmm;
        else if (l == m + 1) pl = cth * sqrt(2.0 * m + 1.0) * pmm;
        else pl = (cth * (2.0 * l - 1.0) * p1 - sqrt((double)(l - 1) * (l - 1) - (double)m * m) * p2) /
                  sqrt((double)l * l - (double)m * m);
        if (l > m) {
            p2 = p1;
            p1 = pl;
        }
        o[(size_t)(l - m) * n_theta] = -G * pl;
    }
}

// Rotation of degree l for patch g, from the patch's N factors (Eqs.
// N_CC..N_SC): with i, o positions inside the degree's 2l + 1 real-index
// entries (pos(m, C) = 2m - 1 or 0 for m = 0, pos(m, S) = 2m),
//   X[(m, C)][(u, C)] = N_CC, X[(m, C)][(u, S)] = N_CS,
//   X[(m, S)][(u, S)] = N_SS, X[(m, S)][(u, C)] = -N_SC.
// Moments (Eqs. U_C/U_S): B[(m, .)] = f_m sum_g sum_(u, .) X A^g[(u, .)] with
// f_m = 2/delta_m for C and 2 for S, stored x1[l][g (2l+1) + pos(u)][pos(m)].
// Expansion: the common-frame moments M give the patch's local ones
// L^g[(u, .)] = sum_(m, .) M[(m, .)] X[(m, .)][(u, .)] (the same factors
// write the common-frame harmonics in local ones), x2[l][g][pos(m)][pos(u)].
__device__ inline void pos_decode(int p, int &m, int &s) {
    m = (p + 1) >> 1;
    s = p > 0 && (p & 1) == 0;
}

__global__ void k_sep_x(int L, int n_patches, int g, const double *N4, const long long *xoff, double *x1,
                        double *x2) {
    // t runs over (l, pos(m), pos(u)) of all degrees: find l
    const long long tt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long acc = 0;
    int l;
    for (l = 0; l <= L; ++l) {
        const long long n2 = (long long)(2 * l + 1) * (2 * l + 1);
        if (tt < acc + n2) break;
        acc += n2;
    }
    if (l > L) return;
    const int n = 2 * l + 1, r = (int)(tt - acc), pm = r / n, pu = r - pm * n;
    int m, sm, u, su;
    pos_decode(pm, m, sm);
    pos_decode(pu, u, su);
    const double *N = N4 + 4 * (size_t)(off_sq(l) + m * (l + 1) + u);
    double x;
    if (!sm) x = su ? N[1] : N[0];
    else x = su ? N[2] : -N[3];
    const double f = (!sm && m == 0) ? 1.0 : 2.0;
    x1[xoff[l] + ((size_t)g * n + pu) * n + pm] = f * x;
    x2[xoff[l] + ((size_t)g * n + pm) * n + pu] = x;
}

// three bf16 pieces of an FP64 factor (through FP32: 24 significant bits)
__device__ inline void split3d(double x, bf16 &h, bf16 &m, bf16 &l) {
    const float v = (float)x;
    h = (bf16)v;
    const float r = v - (float)h;
    m = (bf16)r;
    l = (bf16)(r - (float)m);
}

// f1s[p][row][k]: row < 32 nt2 is the C column of order row + 1, row >= 32
// nt2 the S column of order row - 32 nt2 + 1 (zero past lmax); its phi
// factor at column index 1 + (C: row, S: ce + row - 32 nt2) of f1
__global__ void k_sep_f1s(int L, int nt2, int khp, int nc, int ce, const double *f1, bf16 *f1s) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x, R = 64 * nt2;
    if (t >= R * khp) return;
    const int row = t / khp, k = t - row * khp;
    const bool s = row >= 32 * nt2;
    const int o = s ? row - 32 * nt2 : row;  // order - 1
    double x = 0.0;
    if (o < L) x = f1[(size_t)k * nc + 1 + (s ? ce : 0) + o];
    bf16 h, m, l;
    split3d(x, h, m, l);
    const size_t n = (size_t)R * khp;
    f1s[t] = h;
    f1s[n + t] = m;
    f1s[2 * n + t] = l;
}

// f2s[p][b][cc] = pieces of f2[1 + cc][b] (cc < 2 ce; zero past kx)
__global__ void k_sep_f2s(int kx, int kxp, int ce, const double *f2, bf16 *f2s) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x, K = 2 * ce;
    if (t >= kxp * K) return;
    const int b = t / K, cc = t - b * K;
    const double x = b < kx ? f2[(size_t)(1 + cc) * kx + b] : 0.0;
    bf16 h, m, l;
    split3d(x, h, m, l);
    const size_t n = (size_t)kxp * K;
    f2s[t] = h;
    f2s[n + t] = m;
    f2s[2 * n + t] = l;
}

inline unsigned blocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

static void rotation(double a, double b, double g, double R[9]) {
    // Eq. rottransmatrix, x = R xi
    double ca = cos(a), sa = sin(a), cb = cos(b), sb = sin(b), cg = cos(g), sg = sin(g);
    R[0] = ca * cb * cg - sa * sg;  R[1] = sa * cb * cg + ca * sg;  R[2] = -sb * cg;
    R[3] = -ca * cb * sg - sa * cg; R[4] = -sa * cb * sg + ca * cg; R[5] = sb * sg;
    R[6] = ca * sb;                 R[7] = sa * sb;                 R[8] = cb;
}

hipError_t build_tables(Plan &p, const double *euler, const double *r_edges, const double *host_w,
                        int w_per_patch) {
    const int L = p.lmax;
    hipStream_t s = p.stream;

    // column layout: even-m block first, odd-m block second (fold only)
    std::vector<int> col_src(p.np_alloc, -1), col_l(p.np_alloc, -1), perm_of(p.n_lm, -1);
    {
        int qe = 0, qo = p.ne_p;
        for (int l = 0; l <= L; ++l)
            for (int m = 0; m <= l; ++m) {
                int srcs[2] = {m == 0 ? l * l : l * l + 2 * m - 1, l * l + 2 * m};
                for (int c = 0; c < (m == 0 ? 1 : 2); ++c) {
                    int &q = (!p.fold || (m % 2 == 0)) ? qe : qo;
                    col_src[q] = srcs[c];
                    col_l[q] = l;
                    perm_of[srcs[c]] = q;
                    ++q;
                }
            }
    }
    hipError_t err = hipSuccess;
    int *d_perm = nullptr, *d_code = nullptr;
    int2 *d_kx = nullptr;
    double *d_re = nullptr, *dh = nullptr, *db = nullptr, *N4 = nullptr, *Tt = nullptr, *CS = nullptr;
    const size_t kang = (size_t)p.kang();
    const size_t nU = (size_t)p.np_alloc * kang, nQ = (size_t)p.n2() * p.kq();
#define STEP(x)                             \
    do {                                    \
        err = (x);                          \
        if (err != hipSuccess) goto done;   \
    } while (0)
    STEP(hipMalloc(&p.col_src, sizeof(int) * p.np_alloc));
    STEP(hipMalloc(&p.col_l, sizeof(int) * p.np_alloc));
    STEP(hipMalloc(&d_perm, sizeof(int) * p.n_lm));
    STEP(hipMemcpyAsync(p.col_src, col_src.data(), sizeof(int) * p.np_alloc, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(p.col_l, col_l.data(), sizeof(int) * p.np_alloc, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(d_perm, perm_of.data(), sizeof(int) * p.n_lm, hipMemcpyHostToDevice, s));

    // overlap weights w_jk (Sec. 4.2), one row per patch block
    STEP(hipMalloc(&p.w, sizeof(double) * p.npat * p.n_ang));
    for (int b = 0; b < p.npat; ++b) {
        double *wb = p.w + (size_t)b * p.n_ang;
        if (host_w) {
            const double *src = host_w + (w_per_patch ? (size_t)b * p.n_ang : 0);
            STEP(hipMemcpyAsync(wb, src, sizeof(double) * p.n_ang, hipMemcpyHostToDevice, s));
        } else if (p.n_patches == 1) {
            hipLaunchKernelGGL(k_fill, dim3(blocks(p.n_ang, 256)), dim3(256), 0, s, wb, (size_t)p.n_ang, 1.0);
        } else {
            OvlGeom o;
            o.sc = p.ovl_sc;
            o.kap = p.ovl_kap;
            o.kap_inf = p.ovl_kap_inf;
            hipLaunchKernelGGL(k_overlap, dim3(blocks(p.n_ang, 64)), dim3(64), 0, s, p.n_theta, p.n_phi,
                               p.theta0, p.phi0, p.dtheta, p.dphi, o, wb);
        }
    }
    STEP(hipGetLastError());

    // radial recurrence coefficients
    STEP(hipMalloc(&d_re, sizeof(double) * (p.n_r + 1)));
    STEP(hipMemcpyAsync(d_re, r_edges, sizeof(double) * (p.n_r + 1), hipMemcpyHostToDevice, s));
    STEP(hipMalloc(&p.coef, sizeof(double) * 4 * (size_t)p.n_r * (L + 1)));
    hipLaunchKernelGGL(k_coef, dim3(blocks((size_t)p.n_r * (L + 1), 128)), dim3(128), 0, s, p.n_r, L, d_re, p.coef);
    STEP(hipGetLastError());

    // Wigner d at pi/2, T and C/S (the same for every patch: they depend on
    // the local extents only)
    STEP(hipMalloc(&dh, sizeof(double) * off_dh(L + 1)));
    STEP(hipMalloc(&db, sizeof(double) * 2 * off_sq(L + 1)));
    STEP(hipMalloc(&N4, sizeof(double) * 4 * off_sq(L + 1)));
    STEP(hipMalloc(&Tt, sizeof(double) * (size_t)p.n_theta * off_tri(L + 1)));
    STEP(hipMalloc(&CS, sizeof(double) * 2 * (size_t)p.n_phi * (L + 1)));
    hipLaunchKernelGGL(k_dhalf, dim3(blocks(off_tri(L + 1), 64)), dim3(64), 0, s, L, dh);
    hipLaunchKernelGGL(k_ttilde, dim3(blocks((size_t)p.n_theta * off_tri(L + 1), 128)), dim3(128), 0, s, L, dh,
                       p.n_theta, p.theta0, p.dtheta, Tt);
    hipLaunchKernelGGL(k_cs, dim3(blocks((size_t)p.n_phi * (L + 1), 128)), dim3(128), 0, s, L, p.n_phi, p.phi0,
                       p.dphi, CS);
    STEP(hipGetLastError());

    if (p.sep) {
        // phi columns: order 0, then C of u = 1..L (padded to 16), then S
        const int nc = p.sep_nc(), lp = p.sep_lp, P = p.n_patches, n = p.n_phi;
        std::vector<int> code(nc, -1), ucol(nc, -1), coff(nc, 0), cslot(p.n_lm, -1);
        for (int u = 0; u <= L; ++u)
            for (int cs = 0; cs < (u == 0 ? 1 : 2); ++cs) {
                const int c = cs ? 1 + p.sep_ce + u - 1 : u;
                code[c] = 2 * u + cs;
                ucol[c] = u;
            }
        // slots: the degrees u..L of every column, column after column
        for (int c = 0, o = 0; c < nc; ++c) {
            if (code[c] < 0) continue;
            const int u = code[c] >> 1, cs = code[c] & 1;
            coff[c] = o;
            for (int l = u; l <= L; ++l) cslot[cs ? l * l + 2 * u : (u == 0 ? l * l : l * l + 2 * u - 1)] = o++;
        }
        // expansion points: cell kx[b].x, and its mirror image kx[b].y (-1: none)
        std::vector<int2> kx(p.sep_kx);
        for (int b = 0; b < p.sep_kx; ++b) {
            if (!p.sep_mir) kx[b] = make_int2(b, -1);
            else if (p.eval_centre) kx[b] = make_int2(b, n - 1 - b);
            else if (b < n / 2 - 1) kx[b] = make_int2(b, n - 2 - b);
            else kx[b] = make_int2(b == n / 2 - 1 ? b : n - 1, -1);
        }
        std::vector<long long> xoff(L + 2, 0);
        for (int l = 0; l <= L; ++l) xoff[l + 1] = xoff[l] + (long long)P * (2 * l + 1) * (2 * l + 1);
        const double ev = p.eval_centre ? 0.5 : 1.0;
        STEP(hipMalloc(&d_code, sizeof(int) * nc));
        STEP(hipMalloc(&d_kx, sizeof(int2) * p.sep_kx));
        STEP(hipMalloc(&p.sep_m, sizeof(int) * nc));
        STEP(hipMalloc(&p.sep_coff, sizeof(int) * nc));
        STEP(hipMalloc(&p.sep_cslot, sizeof(int) * p.n_lm));
        STEP(hipMalloc(&p.sep_kxy, sizeof(int2) * p.sep_kx));
        STEP(hipMalloc(&p.sep_xoff, sizeof(long long) * (L + 2)));
        STEP(hipMalloc(&p.sep_perm, sizeof(int) * p.n_lm));
        STEP(hipMalloc(&p.sep_f1, sizeof(double) * p.sep_khp * nc));
        STEP(hipMalloc(&p.sep_f2, sizeof(double) * nc * p.sep_kx));
        STEP(hipMalloc(&p.sep_t1, sizeof(double) * nc * lp * p.n_theta));
        STEP(hipMalloc(&p.sep_t2, sizeof(double) * nc * lp * p.n_theta));
        STEP(hipMalloc(&p.sep_x1, sizeof(double) * xoff[L + 1]));
        STEP(hipMalloc(&p.sep_x2, sizeof(double) * xoff[L + 1]));
        STEP(hipMemcpyAsync(d_code, code.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(d_kx, kx.data(), sizeof(int2) * p.sep_kx, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(p.sep_kxy, kx.data(), sizeof(int2) * p.sep_kx, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(p.sep_m, ucol.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(p.sep_coff, coff.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(p.sep_cslot, cslot.data(), sizeof(int) * p.n_lm, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(p.sep_xoff, xoff.data(), sizeof(long long) * (L + 2), hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(p.sep_perm, perm_of.data(), sizeof(int) * p.n_lm, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_sep_f1, dim3(blocks((size_t)p.sep_khp * nc, 128)), dim3(128), 0, s, L, p.sep_kh,
                           p.sep_khp, nc, d_code, CS, p.sep_f1);
        hipLaunchKernelGGL(k_sep_f2, dim3(blocks((size_t)nc * p.sep_kx, 128)), dim3(128), 0, s, p.sep_kx, nc,
                           p.phi0, p.dphi, ev, d_code, d_kx, p.sep_f2);
        hipLaunchKernelGGL(k_sep_t1, dim3(blocks((size_t)nc * lp * p.n_theta, 128)), dim3(128), 0, s, L,
                           p.n_theta, nc, lp, d_code, Tt, p.sep_t1);
        hipLaunchKernelGGL(k_sep_t2, dim3(blocks((size_t)nc * p.n_theta, 64)), dim3(64), 0, s, L, p.n_theta, nc,
                           lp, p.theta0, p.dtheta, ev, p.G, d_code, p.sep_t2);
        STEP(hipGetLastError());
        if (p.split()) {
            const size_t n1 = (size_t)64 * p.sep_nt2 * p.sep_khp, n2 = (size_t)p.sep_kxp * 2 * p.sep_ce;
            STEP(hipMalloc(&p.sep_f1s, sizeof(bf16) * 3 * n1));
            STEP(hipMalloc(&p.sep_f2s, sizeof(bf16) * 3 * n2));
            hipLaunchKernelGGL(k_sep_f1s, dim3(blocks(n1, 128)), dim3(128), 0, s, L, p.sep_nt2, p.sep_khp, nc,
                               p.sep_ce, p.sep_f1, p.sep_f1s);
            hipLaunchKernelGGL(k_sep_f2s, dim3(blocks(n2, 128)), dim3(128), 0, s, p.sep_kx, p.sep_kxp, p.sep_ce,
                               p.sep_f2, p.sep_f2s);
            STEP(hipGetLastError());
        }
        // every patch's N factors from its own Euler angles
        for (int g = 0; g < P; ++g) {
            const double *e = euler + 3 * g;
            hipLaunchKernelGGL(k_dbeta, dim3(blocks(2 * off_sq(L + 1), 128)), dim3(128), 0, s, L, dh, e[1],
                               M_PI - e[1], db);
            hipLaunchKernelGGL(k_ncoef, dim3(blocks(off_sq(L + 1), 128)), dim3(128), 0, s, L, db, e[0], e[2], N4);
            hipLaunchKernelGGL(k_sep_x, dim3(blocks((size_t)(xoff[L + 1] / P), 128)), dim3(128), 0, s, L, P, g, N4,
                               p.sep_xoff, p.sep_x1, p.sep_x2);
            STEP(hipGetLastError());
        }
    }

    // U and Q of every patch block (under the fold, patch 0 only: patch 1
    // is derived from it); d at beta and pi - beta and the N factors come
    // from the block's own Euler angles
    STEP(hipMalloc(&p.Ut, sizeof(double) * nU));
    STEP(hipMalloc(&p.Qt, sizeof(double) * nQ));
    STEP(hipMemsetAsync(p.Qt, 0, sizeof(double) * nQ, s));
    for (int b = 0; b < p.npat; ++b) {
        // the per-patch method takes every patch's harmonics in its own frame
        const double ident[3] = {0.0, 0.0, 0.0};
        const double *e = p.per_patch ? ident : euler + 3 * b;
        hipLaunchKernelGGL(k_dbeta, dim3(blocks(2 * off_sq(L + 1), 128)), dim3(128), 0, s, L, dh, e[1],
                           M_PI - e[1], db);
        hipLaunchKernelGGL(k_ncoef, dim3(blocks(off_sq(L + 1), 128)), dim3(128), 0, s, L, db, e[0], e[2], N4);
        hipLaunchKernelGGL(k_U, dim3(blocks(p.n_angp, 128), p.np_alloc), dim3(128), 0, s, L, p.np_alloc, p.n_angp,
                           p.n_ang, p.n_phi, p.col_src, Tt, CS, N4, p.w + (size_t)b * p.n_ang, kang,
                           (size_t)b * p.n_angp, p.Ut);
        STEP(hipGetLastError());
    }
    // Q at the cells of patch b in the frame of patch c: xi_c = R_c^T R_b xi_b
    // (per-patch method, all pairs); else in the common frame, x = R_b xi_b
    for (int b = 0; b < (p.per_patch ? p.n_patches : p.npat); ++b)
        for (int c = 0; c < p.nq(); ++c) {
            double Rb[9], Rc[9];
            rotation(euler[3 * b], euler[3 * b + 1], euler[3 * b + 2], Rb);
            Rot R;
            if (p.per_patch) {
                rotation(euler[3 * c], euler[3 * c + 1], euler[3 * c + 2], Rc);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double v = 0.0;
                        for (int k = 0; k < 3; ++k) v += Rc[3 * k + i] * Rb[3 * k + j];
                        R.r[3 * i + j] = v;
                    }
            } else {
                for (int i = 0; i < 9; ++i) R.r[i] = Rb[i];
            }
            const size_t ldq = (size_t)p.kq();
            hipLaunchKernelGGL(k_Q, dim3(blocks(p.n_angp, 64)), dim3(64), 0, s, L, p.np, p.n_angp, p.n_ang, p.n_phi,
                               p.theta0, p.phi0, p.dtheta, p.dphi, p.eval_centre ? 0.5 : 1.0, R, p.G, d_perm, ldq,
                               p.Qt + (size_t)b * p.n_angp * ldq + (size_t)c * p.np);
            STEP(hipGetLastError());
        }

    // split-BF16 copies
    if (p.split()) {
        // U: GEMM1 column tiles over the K = n_angp slabs
        const int ks1 = (int)(kang / kSlabK), ks2 = p.kq() / kSlabK;
        const size_t tU = (size_t)(p.tiles_e() + p.tiles_o()) * ks1 * 512;
        const size_t tQ = (size_t)(p.n2() / kSplitTile) * ks2 * 512;
        STEP(hipMalloc(&p.Us, sizeof(bf16) * tU * 24));
        STEP(hipMalloc(&p.Qs, sizeof(bf16) * tQ * 24));
        hipLaunchKernelGGL(k_tile_split, dim3(blocks(tU, 256)), dim3(256), 0, s, p.Ut, kang, ks1,
                           p.tiles_e(), p.fold ? p.ne_p : p.np, p.ne_p, p.np, tU, p.Us);
        // Q: angular tiles over the K = np slabs
        hipLaunchKernelGGL(k_tile_split, dim3(blocks(tQ, 256)), dim3(256), 0, s, p.Qt, (size_t)p.kq(), ks2,
                           p.n2() / kSplitTile, p.n2(), 0, p.n2(), tQ, p.Qs);
        STEP(hipGetLastError());
    }
    STEP(hipStreamSynchronize(s));
done:
#undef STEP
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_perm);
    (void)hipFree(d_re);
    (void)hipFree(d_code);
    (void)hipFree(d_kx);
    (void)hipFree(dh);
    (void)hipFree(db);
    (void)hipFree(N4);
    (void)hipFree(Tt);
    (void)hipFree(CS);
    return err;
}

hipError_t export_tables(const Plan &p, double *U, double *Q, double *w) {
    if (U || Q)
        hipLaunchKernelGGL(k_export, dim3(blocks(p.n_ang, 128), p.np), dim3(128), 0, p.stream, p.Ut, p.Qt, p.np,
                           p.n_angp, p.n_ang, p.n_lm, p.n_patches, p.npat, (int)p.fold, (int)p.per_patch,
                           (size_t)p.kq(), p.col_src, U, Q);
    hipError_t e = hipGetLastError();
    for (int g = 0; w && e == hipSuccess && g < p.n_patches; ++g)
        e = hipMemcpyAsync(w + (size_t)g * p.n_ang, p.w + (size_t)(p.npat == 1 ? 0 : g) * p.n_ang,
                           sizeof(double) * p.n_ang, hipMemcpyDeviceToDevice, p.stream);
    return e;
}

}  // namespace mpg
