/*
 * oracle.c -- plain FP64 reference of the multipole gravity solver.
 * TEST INFRASTRUCTURE ONLY (see oracle.h): used by tests, the smoke check
 * and the CPU baseline of the benchmark, never by the product library.
 *
 * Every routine follows the definition it cites; nothing is blocked, fused
 * or reordered beyond it.  Build: plain C99, -O2, no fast-math, no FMA
 * contraction.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_LMAX_CAP 84 /* (2*84)! still fits a double */

static int lm_count(int lmax) { return (lmax + 1) * (lmax + 1); }
static int idx_c(int l, int m) { return m == 0 ? l * l : l * l + 2 * m - 1; }
static int idx_s(int l, int m) { return l * l + 2 * m; }

/* ---------------------------------------------------------------------- */
/* Eq. rottransmatrix (z-y'-z'' convention).  Row-major R, x = R xi.       */
void orc_rotation(double a, double b, double g, double R[9]) {
    double ca = cos(a), sa = sin(a), cb = cos(b), sb = sin(b);
    double cg = cos(g), sg = sin(g);
    R[0] = ca * cb * cg - sa * sg;  R[1] = sa * cb * cg + ca * sg;  R[2] = -sb * cg;
    R[3] = -ca * cb * sg - sa * cg; R[4] = -sa * cb * sg + ca * cg; R[5] = sb * sg;
    R[6] = ca * sb;                 R[7] = sa * sb;                 R[8] = cb;
}

/* ---------------------------------------------------------------------- */
/* Eq. Y_l^m: associated Legendre functions with the Condon-Shortley phase,
 * by the textbook recurrences on the unnormalised P_l^m, times
 * s_lm = sqrt((l-m)!/(l+m)!).  out[l(l+1)/2 + m]. */
int orc_legendre(int lmax, double x, double *out) {
    if (lmax < 0 || lmax > ORC_LMAX_CAP || !(x >= -1.0 && x <= 1.0)) return -1;
    double somx2 = sqrt((1.0 - x) * (1.0 + x));
    double pmm = 1.0, fact = 1.0;
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) { pmm *= -fact * somx2; fact += 2.0; }
        double p_lm2 = 0.0, p_lm1 = pmm;
        for (int l = m; l <= lmax; ++l) {
            double p;
            if (l == m) p = pmm;
            else if (l == m + 1) p = x * (2.0 * m + 1.0) * pmm;
            else p = (x * (2.0 * l - 1.0) * p_lm1 - (l + m - 1.0) * p_lm2) / (double)(l - m);
            if (l > m) { p_lm2 = p_lm1; p_lm1 = p; }
            double prod = 1.0; /* (l+m)!/(l-m)! */
            for (int k = l - m + 1; k <= l + m; ++k) prod *= (double)k;
            out[l * (l + 1) / 2 + m] = p / sqrt(prod);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Gauss-Legendre rule by Newton iteration on P_n. */
int orc_gauss_legendre(int n, double *x, double *wt) {
    if (n < 1 || n > 512) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        {   /* final derivative at the converged node */
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Adaptive Gauss-Legendre (rule of 10 nodes against two halves), absolute
 * tolerance per accepted piece. */
typedef double (*orc_fn)(double, const void *);

static double gl_x10[10], gl_w10[10];
static int gl10_ready = 0;
static void gl10_init(void) {
    if (!gl10_ready) { orc_gauss_legendre(10, gl_x10, gl_w10); gl10_ready = 1; }
}
static double gl10(orc_fn f, const void *ctx, double a, double b) {
    double h = 0.5 * (b - a), m = 0.5 * (a + b), s = 0.0;
    for (int i = 0; i < 10; ++i) s += gl_w10[i] * f(m + h * gl_x10[i], ctx);
    return s * h;
}
static double adapt_rec(orc_fn f, const void *ctx, double a, double b,
                        double whole, double tol, int depth) {
    double m = 0.5 * (a + b);
    double l = gl10(f, ctx, a, m), r = gl10(f, ctx, m, b);
    if (depth <= 0 || fabs(l + r - whole) <= tol) return l + r;
    return adapt_rec(f, ctx, a, m, l, tol, depth - 1) +
           adapt_rec(f, ctx, m, b, r, tol, depth - 1);
}
static double adapt_int(orc_fn f, const void *ctx, double a, double b, double tol) {
    gl10_init();
    return adapt_rec(f, ctx, a, b, gl10(f, ctx, a, b), tol, 60);
}

/* ---------------------------------------------------------------------- */
/* Overlap weights (Sec. 4.2, w_jk = 1 - alpha_jk/2).
 * A Yin point with local unit vector (xi,eta,zeta) has Yang-local
 * coordinates (-xi, zeta, eta) (Eq. caryytransform, P is its own inverse).
 * With both patches spanning [pi/2-c, pi/2+c] x [-phe, phe]:
 *   |cos theta_Yang| <= sin c   <=>  |sin phi| <= sin c / sin theta
 *   |phi_Yang| <= phe           <=>  cos phi <= cot(pi-phe) |cot theta|
 * (the second for phe in [pi/2, pi]; always true for phe = pi). */
typedef struct { double sc, tau; int tau_inf; double p1, p2; } ovl_ctx;

static double seg_overlap(double a0, double a1, double b0, double b1) {
    double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
    return hi > lo ? hi - lo : 0.0;
}

/* covered phi-length inside [p1, p2] at colatitude th, times sin th */
static double ovl_integrand(double th, const void *vctx) {
    const ovl_ctx *c = (const ovl_ctx *)vctx;
    double st = sin(th), ct = cos(th);
    double s1[3][2], s2[2][2];
    int n1 = 0, n2 = 0;
    double A = c->sc / st;
    if (A >= 1.0) { s1[0][0] = -ORC_PI; s1[0][1] = ORC_PI; n1 = 1; }
    else {
        double a = asin(A);
        s1[0][0] = -ORC_PI;     s1[0][1] = -ORC_PI + a;
        s1[1][0] = -a;          s1[1][1] = a;
        s1[2][0] = ORC_PI - a;  s1[2][1] = ORC_PI;
        n1 = 3;
    }
    double Bv = c->tau_inf ? 2.0 : c->tau * fabs(ct / st);
    if (Bv >= 1.0) { s2[0][0] = -ORC_PI; s2[0][1] = ORC_PI; n2 = 1; }
    else {
        double b = acos(Bv);
        s2[0][0] = -ORC_PI; s2[0][1] = -b;
        s2[1][0] = b;       s2[1][1] = ORC_PI;
        n2 = 2;
    }
    double len = 0.0;
    for (int u = 0; u < n1; ++u)
        for (int v = 0; v < n2; ++v) {
            double lo = s1[u][0] > s2[v][0] ? s1[u][0] : s2[v][0];
            double hi = s1[u][1] < s2[v][1] ? s1[u][1] : s2[v][1];
            if (hi > lo) len += seg_overlap(lo, hi, c->p1, c->p2);
        }
    return st * len;
}

int orc_overlap_weights(const orc_grid *g, double *w) {
    if (!g || !w || g->n_patches != 2 || g->n_theta < 1 || g->n_phi < 1) return -1;
    double th_lo = g->theta0, th_hi = g->theta0 + g->n_theta * g->dtheta;
    double ph_lo = g->phi0, ph_hi = g->phi0 + g->n_phi * g->dphi;
    if (fabs(th_lo + th_hi - ORC_PI) > 1e-12 || fabs(ph_lo + ph_hi) > 1e-12) return -2;
    if (th_lo < 0.0 || th_lo >= 0.5 * ORC_PI) return -3;
    if (ph_hi < 0.5 * ORC_PI || ph_hi > ORC_PI + 1e-15) return -4;
    ovl_ctx ctx;
    ctx.sc = cos(th_lo);
    ctx.tau_inf = ph_hi >= ORC_PI;
    ctx.tau = ctx.tau_inf ? 0.0 : 1.0 / tan(ORC_PI - ph_hi);
    for (int j = 0; j < g->n_theta; ++j) {
        double t1 = g->theta0 + j * g->dtheta, t2 = t1 + g->dtheta;
        for (int k = 0; k < g->n_phi; ++k) {
            ctx.p1 = g->phi0 + k * g->dphi;
            ctx.p2 = ctx.p1 + g->dphi;
            double area = g->dphi * (cos(t1) - cos(t2));
            /* Split [t1, t2] wherever the covered length changes its formula:
             * a boundary curve meets the cell edge phi = p1 or p2, the
             * curves meet each other, or a condition starts to bind.
             * Between these points the integrand is smooth. */
            double br[32];
            int nb = 0;
            br[nb++] = t1;
            br[nb++] = t2;
            double ps[2] = {ctx.p1, ctx.p2};
            for (int e = 0; e < 2; ++e) {
                double sp = fabs(sin(ps[e])), cpv = cos(ps[e]);
                if (sp > 0.0 && ctx.sc / sp <= 1.0) {
                    double t = asin(ctx.sc / sp);
                    br[nb++] = t; br[nb++] = ORC_PI - t;
                }
                if (!ctx.tau_inf && cpv > 0.0) {
                    double t = atan2(ctx.tau, cpv);
                    br[nb++] = t; br[nb++] = ORC_PI - t;
                }
            }
            { double t = asin(ctx.sc); br[nb++] = t; br[nb++] = ORC_PI - t; }
            if (!ctx.tau_inf) {
                double t = atan(ctx.tau);
                br[nb++] = t; br[nb++] = ORC_PI - t;
                double cc = sqrt((1.0 - ctx.sc * ctx.sc) / (1.0 + ctx.tau * ctx.tau));
                br[nb++] = acos(cc); br[nb++] = acos(-cc);
            }
            br[nb++] = 0.5 * ORC_PI;
            /* sort (insertion) and integrate piece by piece inside [t1, t2] */
            for (int u = 1; u < nb; ++u)
                for (int v = u; v > 0 && br[v - 1] > br[v]; --v) {
                    double tmp = br[v]; br[v] = br[v - 1]; br[v - 1] = tmp;
                }
            double cov = 0.0;
            for (int u = 0; u + 1 < nb; ++u) {
                double a = br[u] < t1 ? t1 : br[u], b = br[u + 1] > t2 ? t2 : br[u + 1];
                if (b > a) cov += adapt_int(ovl_integrand, &ctx, a, b, 1e-18 * area);
            }
            w[j * g->n_phi + k] = 1.0 - 0.5 * (cov / area);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Angular weights U (Eqs. A_lm_mult/B_lm_mult in the real form of
 * Eq. phimulti, with the 2/delta_m of Eq. del_m) and prefactors Q
 * (Eqs. Q_C/Q_S), both in the global frame, straight from the definition. */
#define ORC_NQ 12

static int check_grid(const orc_grid *g, int lmax) {
    if (!g || g->n_patches < 1 || g->n_r < 1 || g->n_theta < 1 || g->n_phi < 1) return -1;
    if (!g->r_edges || !g->euler || lmax < 0 || lmax > ORC_LMAX_CAP) return -1;
    if (g->r_edges[0] < 0.0) return -1;
    for (int i = 0; i < g->n_r; ++i)
        if (!(g->r_edges[i + 1] > g->r_edges[i])) return -1;
    return 0;
}

static void global_angles(const double R[9], double th, double ph,
                          double *cth, double *phg) {
    double xi = sin(th) * cos(ph), et = sin(th) * sin(ph), ze = cos(th);
    double x = R[0] * xi + R[1] * et + R[2] * ze;
    double y = R[3] * xi + R[4] * et + R[5] * ze;
    double z = R[6] * xi + R[7] * et + R[8] * ze;
    double r = sqrt(x * x + y * y + z * z);
    double c = z / r;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    *cth = c;
    *phg = atan2(y, x);
}

int orc_tables_range(const orc_grid *g, int lmax, const double *w,
                     int c0, int c1, double *U, double *Q) {
    if (check_grid(g, lmax)) return -1;
    int n_ang = g->n_theta * g->n_phi, nlm = lm_count(lmax);
    if (c0 < 0 || c1 > n_ang || c0 > c1) return -1;
    double qx[ORC_NQ], qw[ORC_NQ];
    orc_gauss_legendre(ORC_NQ, qx, qw);
    int ntri = (lmax + 1) * (lmax + 2) / 2;
    double *P = (double *)malloc(sizeof(double) * ntri);
    double *acc = (double *)malloc(sizeof(double) * nlm);
    double *cm = (double *)malloc(sizeof(double) * (lmax + 1));
    double *sm = (double *)malloc(sizeof(double) * (lmax + 1));
    if (!P || !acc || !cm || !sm) { free(P); free(acc); free(cm); free(sm); return -5; }
    for (int p = 0; p < g->n_patches; ++p) {
        double R[9];
        orc_rotation(g->euler[3 * p], g->euler[3 * p + 1], g->euler[3 * p + 2], R);
        for (int c = c0; c < c1; ++c) {
            int j = c / g->n_phi, k = c % g->n_phi;
            double t1 = g->theta0 + j * g->dtheta, f1 = g->phi0 + k * g->dphi;
            if (U) {
                memset(acc, 0, sizeof(double) * nlm);
                for (int a = 0; a < ORC_NQ; ++a) {
                    double th = t1 + 0.5 * g->dtheta * (qx[a] + 1.0);
                    for (int b = 0; b < ORC_NQ; ++b) {
                        double ph = f1 + 0.5 * g->dphi * (qx[b] + 1.0);
                        double wt = qw[a] * qw[b] * 0.25 * g->dtheta * g->dphi * sin(th);
                        double cth, phg;
                        global_angles(R, th, ph, &cth, &phg);
                        orc_legendre(lmax, cth, P);
                        for (int m = 0; m <= lmax; ++m) { cm[m] = cos(m * phg); sm[m] = sin(m * phg); }
                        for (int l = 0; l <= lmax; ++l) {
                            acc[idx_c(l, 0)] += wt * P[l * (l + 1) / 2];
                            for (int m = 1; m <= l; ++m) {
                                double v = wt * P[l * (l + 1) / 2 + m];
                                acc[idx_c(l, m)] += v * cm[m];
                                acc[idx_s(l, m)] += v * sm[m];
                            }
                        }
                    }
                }
                double wc = w ? w[(size_t)p * g->w_stride + c] : 1.0;
                double *row = U + ((size_t)p * n_ang + c) * nlm;
                for (int l = 0; l <= lmax; ++l) {
                    row[idx_c(l, 0)] = wc * acc[idx_c(l, 0)];          /* 2/delta_0 = 1 */
                    for (int m = 1; m <= l; ++m) {
                        row[idx_c(l, m)] = 2.0 * wc * acc[idx_c(l, m)];
                        row[idx_s(l, m)] = 2.0 * wc * acc[idx_s(l, m)];
                    }
                }
            }
            if (Q) {
                double cth, phg;
                const double ev = g->eval_centre ? 0.5 : 1.0;  /* evaluation point in the cell */
                global_angles(R, t1 + ev * g->dtheta, f1 + ev * g->dphi, &cth, &phg);
                orc_legendre(lmax, cth, P);
                double *row = Q + ((size_t)p * n_ang + c) * nlm;
                for (int l = 0; l <= lmax; ++l) {
                    row[idx_c(l, 0)] = -g->G * P[l * (l + 1) / 2];
                    for (int m = 1; m <= l; ++m) {
                        row[idx_c(l, m)] = -g->G * P[l * (l + 1) / 2 + m] * cos(m * phg);
                        row[idx_s(l, m)] = -g->G * P[l * (l + 1) / 2 + m] * sin(m * phg);
                    }
                }
            }
        }
    }
    free(P); free(acc); free(cm); free(sm);
    return 0;
}

int orc_tables(const orc_grid *g, int lmax, const double *w, double *U, double *Q) {
    if (check_grid(g, lmax)) return -1;
    return orc_tables_range(g, lmax, w, 0, g->n_theta * g->n_phi, U, Q);
}

/* ---------------------------------------------------------------------- */
/* Neumaier's compensated summation, the oracle's stand-in for the two-sum
 * the paper uses for its angular sums (Sec. 4.3). */
static void neu_add(double *s, double *comp, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *comp += (*s - t) + x;
    else *comp += (x - t) + *s;
    *s = t;
}

int orc_moments(const orc_grid *g, int lmax, const double *U,
                const double *rho, int n_sh, const int *shells, double *B) {
    if (check_grid(g, lmax) || !U || !rho || !B) return -1;
    int n_ang = g->n_theta * g->n_phi, nlm = lm_count(lmax);
    int cnt = shells ? n_sh : g->n_r;
    double *s = (double *)malloc(sizeof(double) * nlm);
    double *cp = (double *)malloc(sizeof(double) * nlm);
    if (!s || !cp) { free(s); free(cp); return -5; }
    for (int t = 0; t < cnt; ++t) {
        int i = shells ? shells[t] : t;
        if (i < 0 || i >= g->n_r) { free(s); free(cp); return -1; }
        memset(s, 0, sizeof(double) * nlm);
        memset(cp, 0, sizeof(double) * nlm);
        for (int p = 0; p < g->n_patches; ++p)
            for (int c = 0; c < n_ang; ++c) {
                double r = rho[((size_t)p * g->n_r + i) * n_ang + c];
                if (r == 0.0) continue;
                const double *u = U + ((size_t)p * n_ang + c) * nlm;
                for (int q = 0; q < nlm; ++q) neu_add(&s[q], &cp[q], r * u[q]);
            }
        for (int q = 0; q < nlm; ++q) B[(size_t)i * nlm + q] = s[q] + cp[q];
    }
    free(s); free(cp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Radial factors of Eq. M_C at the interface r_n^+ for shell i, degree l:
 *   i <= n :  R_in,i / (r_n)^{l+1} = r_n^2 [ (r_i^+/r_n)^{l+3} - (r_i^-/r_n)^{l+3} ] / (l+3)
 *   i >  n :  (r_n)^l R_out,i      = [ (r_i^+)^2 (r_n/r_i^+)^l - (r_i^-)^2 (r_n/r_i^-)^l ] / (2-l)
 *                                    (r_n^2 ln(r_i^+/r_i^-) at l = 2)
 * (Eqs. R_in, R_out); each difference of powers via expm1. */
double orc_radial_factor(const double *r_edges, int n, int i, int l) {
    double rn = r_edges[n + 1], rp = r_edges[i + 1], rm = r_edges[i];
    if (i <= n) {
        double p = l + 3.0, a = rp / rn, b = rm / rn;
        double ap = pow(a, p);
        double diff = (b == 0.0) ? ap : -ap * expm1(p * log(b / a));
        return rn * rn * diff / p;
    } else {
        if (l == 2) return rn * rn * log(rp / rm);
        double q = 2.0 - l;
        double y = rm * rm * pow(rn / rm, (double)l);
        return y * expm1(q * log(rp / rm)) / q;
    }
}

int orc_radial(const orc_grid *g, int lmax, const double *B,
               int n_sh, const int *shells, double *M) {
    if (check_grid(g, lmax) || !B || !M) return -1;
    int nlm = lm_count(lmax), nr = g->n_r;
    int cnt = shells ? n_sh : nr;
    double *f = (double *)malloc(sizeof(double) * nr);
    double *s = (double *)malloc(sizeof(double) * nlm);
    double *cp = (double *)malloc(sizeof(double) * nlm);
    if (!f || !s || !cp) { free(f); free(s); free(cp); return -5; }
    for (int t = 0; t < cnt; ++t) {
        int n = shells ? shells[t] : t;
        if (n < 0 || n >= nr) { free(f); free(s); free(cp); return -1; }
        memset(s, 0, sizeof(double) * nlm);
        memset(cp, 0, sizeof(double) * nlm);
        for (int l = 0; l <= lmax; ++l) {
            for (int i = 0; i < nr; ++i) f[i] = orc_radial_factor(g->r_edges, n, i, l);
            for (int q = l * l; q < (l + 1) * (l + 1); ++q)
                for (int i = 0; i < nr; ++i)
                    neu_add(&s[q], &cp[q], f[i] * B[(size_t)i * nlm + q]);
        }
        for (int q = 0; q < nlm; ++q) M[(size_t)n * nlm + q] = s[q] + cp[q];
    }
    free(f); free(s); free(cp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Eq. gravpotmult. */
int orc_expand(const orc_grid *g, int lmax, const double *Q,
               const double *M, int n_sh, const int *shells, double *phi) {
    if (check_grid(g, lmax) || !Q || !M || !phi) return -1;
    int n_ang = g->n_theta * g->n_phi, nlm = lm_count(lmax);
    int cnt = shells ? n_sh : g->n_r;
    for (int t = 0; t < cnt; ++t) {
        int n = shells ? shells[t] : t;
        if (n < 0 || n >= g->n_r) return -1;
        const double *m = M + (size_t)n * nlm;
        for (int p = 0; p < g->n_patches; ++p)
            for (int c = 0; c < n_ang; ++c) {
                const double *q = Q + ((size_t)p * n_ang + c) * nlm;
                double s = 0.0, cp = 0.0;
                for (int k = 0; k < nlm; ++k) neu_add(&s, &cp, q[k] * m[k]);
                phi[((size_t)p * g->n_r + n) * n_ang + c] = s + cp;
            }
    }
    return 0;
}

int orc_phi_points(const orc_grid *g, int lmax, const double *M, int n,
                   const int *pp, const int *ii, const int *cc, double *out) {
    if (check_grid(g, lmax) || !M || !out || n < 0) return -1;
    int n_ang = g->n_theta * g->n_phi, nlm = lm_count(lmax);
    double *Q = (double *)malloc(sizeof(double) * nlm);
    if (!Q) return -5;
    for (int t = 0; t < n; ++t) {
        if (pp[t] < 0 || pp[t] >= g->n_patches || ii[t] < 0 || ii[t] >= g->n_r ||
            cc[t] < 0 || cc[t] >= n_ang) { free(Q); return -1; }
        /* the one-row table of this point, from the same definition */
        orc_grid one = *g;
        int j = cc[t] / g->n_phi, k = cc[t] % g->n_phi;
        one.n_patches = 1;
        one.euler = g->euler + 3 * pp[t];
        one.n_theta = 1; one.n_phi = 1;
        one.theta0 = g->theta0 + j * g->dtheta;
        one.phi0 = g->phi0 + k * g->dphi;
        orc_tables_range(&one, lmax, NULL, 0, 1, NULL, Q);
        const double *m = M + (size_t)ii[t] * nlm;
        double s = 0.0, cp = 0.0;
        for (int q = 0; q < nlm; ++q) neu_add(&s, &cp, Q[q] * m[q]);
        out[t] = s + cp;
    }
    free(Q);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Brute force through the addition theorem, sum_m Y Y* = (2l+1)/(4 pi) P_l,
 * on the Green's function expansion of Eq. integralpoisson. */
static void local_dir(double th, double ph, int patch, double v[3]) {
    double xi = sin(th) * cos(ph), et = sin(th) * sin(ph), ze = cos(th);
    if (patch == 0) { v[0] = xi; v[1] = et; v[2] = ze; }
    else { v[0] = -xi; v[1] = ze; v[2] = et; } /* Yang -> Yin frame */
}

int orc_brute_phi(const orc_grid *g, int lmax, const double *w,
                  const double *rho, int nq, int n, const int *pp,
                  const int *ii, const int *cc, double *out) {
    if (check_grid(g, lmax) || !rho || !out || g->n_patches > 2 || nq < 1 || nq > 64) return -1;
    int n_ang = g->n_theta * g->n_phi, nr = g->n_r;
    double qx[64], qw[64];
    orc_gauss_legendre(nq, qx, qw);
    double *I = (double *)malloc(sizeof(double) * (lmax + 1));
    double *K = (double *)malloc(sizeof(double) * (lmax + 1) * nr);
    if (!I || !K) { free(I); free(K); return -5; }
    for (int t = 0; t < n; ++t) {
        int pt = pp[t], nt = ii[t], ct = cc[t];
        if (pt < 0 || pt >= g->n_patches || nt < 0 || nt >= nr || ct < 0 || ct >= n_ang) {
            free(I); free(K); return -1;
        }
        for (int l = 0; l <= lmax; ++l)
            for (int i = 0; i < nr; ++i) K[l * nr + i] = orc_radial_factor(g->r_edges, nt, i, l);
        double tv[3];
        const double ev = g->eval_centre ? 0.5 : 1.0;  /* evaluation point in the cell */
        local_dir(g->theta0 + (ct / g->n_phi + ev) * g->dtheta,
                  g->phi0 + (ct % g->n_phi + ev) * g->dphi, pt, tv);
        double s = 0.0, cp = 0.0;
        for (int p = 0; p < g->n_patches; ++p)
            for (int c = 0; c < n_ang; ++c) {
                int j = c / g->n_phi, k = c % g->n_phi;
                double t1 = g->theta0 + j * g->dtheta, f1 = g->phi0 + k * g->dphi;
                for (int l = 0; l <= lmax; ++l) I[l] = 0.0;
                for (int a = 0; a < nq; ++a) {
                    double th = t1 + 0.5 * g->dtheta * (qx[a] + 1.0);
                    for (int b = 0; b < nq; ++b) {
                        double ph = f1 + 0.5 * g->dphi * (qx[b] + 1.0);
                        double wt = qw[a] * qw[b] * 0.25 * g->dtheta * g->dphi * sin(th);
                        double sv[3];
                        local_dir(th, ph, p, sv);
                        double x = tv[0] * sv[0] + tv[1] * sv[1] + tv[2] * sv[2];
                        double p0 = 1.0, p1 = x;
                        I[0] += wt;
                        if (lmax >= 1) I[1] += wt * x;
                        for (int l = 2; l <= lmax; ++l) {
                            double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
                            I[l] += wt * p2;
                            p0 = p1; p1 = p2;
                        }
                    }
                }
                double wc = w ? w[(size_t)p * g->w_stride + c] : 1.0;
                for (int i = 0; i < nr; ++i) {
                    double r = rho[((size_t)p * nr + i) * n_ang + c];
                    if (r == 0.0) continue;
                    for (int l = 0; l <= lmax; ++l)
                        neu_add(&s, &cp, -g->G * r * wc * K[l * nr + i] * I[l]);
                }
            }
        out[t] = s + cp;
    }
    free(I); free(K);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Eq. phiana with Eq. u0.  The lower limit u0 is 0 for a point inside the
 * ellipsoid and the positive root of Eq. u0 outside (the text states the
 * two cases the other way round; only this assignment gives -GM/r far
 * away and a root that exists).  The last function integrates
 * [(a^2+u)(b^2+u)(c^2+u)]^{-1/2}. */
typedef struct { double a2, b2, c2, u0, L; int ka, kb, kc; } ell_ctx;

static double ell_integrand(double psi, const void *vctx) {
    const ell_ctx *e = (const ell_ctx *)vctx;
    double t = tan(psi), sc = 1.0 / cos(psi);
    double u = e->u0 + e->L * t * t;
    double du = 2.0 * e->L * t * sc * sc;
    double A = e->a2 + u, B = e->b2 + u, C = e->c2 + u;
    double f = 1.0 / sqrt(A * B * C);
    if (e->ka) f /= A;
    if (e->kb) f /= B;
    if (e->kc) f /= C;
    return f * du;
}

static double ell_int(ell_ctx e, int ka, int kb, int kc) {
    e.ka = ka; e.kb = kb; e.kc = kc;
    double scale = ell_integrand(0.25 * ORC_PI, &e);
    return adapt_int(ell_integrand, &e, 0.0, 0.5 * ORC_PI, 1e-17 * fabs(scale));
}

double orc_ellipsoid_phi(double a, double b, double c, double rho0, double G,
                         double X, double Y, double Z) {
    ell_ctx e;
    e.a2 = a * a; e.b2 = b * b; e.c2 = c * c;
    double s = X * X / e.a2 + Y * Y / e.b2 + Z * Z / e.c2;
    double u0 = 0.0;
    if (s > 1.0) {
        double lo = 0.0, hi = 1.0;
        for (;;) {
            double f = X * X / (e.a2 + hi) + Y * Y / (e.b2 + hi) + Z * Z / (e.c2 + hi) - 1.0;
            if (f < 0.0) break;
            hi *= 2.0;
        }
        for (int it = 0; it < 400; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double f = X * X / (e.a2 + mid) + Y * Y / (e.b2 + mid) + Z * Z / (e.c2 + mid) - 1.0;
            if (f > 0.0) lo = mid; else hi = mid;
        }
        u0 = 0.5 * (lo + hi);
    }
    e.u0 = u0;
    e.L = u0 + (e.a2 > e.b2 ? (e.a2 > e.c2 ? e.a2 : e.c2) : (e.b2 > e.c2 ? e.b2 : e.c2));
    double IA = ell_int(e, 1, 0, 0), IB = ell_int(e, 0, 1, 0);
    double IC = ell_int(e, 0, 0, 1), ID = ell_int(e, 0, 0, 0);
    return ORC_PI * G * rho0 * a * b * c * (IA * X * X + IB * Y * Y + IC * Z * Z - ID);
}
