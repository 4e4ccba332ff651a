/*
 * oracle.h -- plain, slow, single-threaded FP64 CPU reference for the
 * multipole gravity solver on multi-patch spherical grids
 * (Wongwathanarat, "A Generalized Solution Method for Parallelized
 * Computation of the Three-dimensional Gravitational Potential on a
 * Multi-patch grid in Spherical Geometry", arXiv:1903.08475).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links,
 * includes or calls this code; only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no source with
 * the GPU path.
 *
 * What it computes is the discretised result of Sec. 2.2 and Sec. 4.2
 * written out from its definition, without the paper's factorisation:
 *
 *   U^{C/S}_{g,jk,lm} = (2/delta_m) s_lm w_jk  Int_cell P_l^m(cos th) {cos,sin}(m ph) dOmega
 *   B_{i,lm}          = sum_g sum_jk rho_{g,i,jk} U_{g,jk,lm}                 (Eq. B_CS)
 *   M_{n,lm}          = sum_{i<=n} R_in,i/(r_n)^{l+1} B_i + sum_{i>n} (r_n)^l R_out,i B_i   (Eq. M_C)
 *   Phi_{g,n,jk}      = sum_lm Q_{g,jk,lm} M_{n,lm}                             (Eq. gravpotmult)
 *
 * with s_lm = sqrt((l-m)!/(l+m)!), P_l^m including the Condon-Shortley
 * phase, (th, ph) the global angles of a point of patch g under
 * x = R^(g) xi (Eq. rottransmatrix), the cell integral taken in the
 * patch's local (theta, phi) by tensor Gauss-Legendre quadrature, and Q
 * the prefactors of Eqs. Q_C/Q_S at the upper cell vertex (or, with
 * eval_centre, at the cell's angular centre on the same outer radius).  No Wigner d,
 * no T/C/S integrals, no (-1)^m sharing between patches and no radial
 * recurrence is used.
 *
 * Real column index of a moment: idx(l,0) = l^2, idx(l,m,C) = l^2+2m-1,
 * idx(l,m,S) = l^2+2m  (m >= 1);  n_lm = (lmax+1)^2.
 *
 * Array layouts (row-major, last index fastest):
 *   rho, phi : [n_patches][n_r][n_theta][n_phi]
 *   U, Q     : [n_patches][n_theta*n_phi][n_lm]
 *   B, M     : [n_r][n_lm]
 *   w        : [n_theta*n_phi]
 * All functions return 0 on success and a negative value on bad arguments.
 */
#ifndef MPG_ORACLE_H
#define MPG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n_patches;          /* number of grid patches N_g                   */
    int n_r, n_theta, n_phi;
    const double *r_edges;  /* n_r+1 radial interfaces, increasing, >= 0    */
    double theta0, phi0;    /* local lower corner of every patch            */
    double dtheta, dphi;    /* local angular spacing                        */
    const double *euler;    /* n_patches*3 Euler angles (alpha,beta,gamma)  */
    double G;               /* gravitational constant                       */
    int w_stride;           /* overlap weights of patch p start at
                               w + p*w_stride (0: one set for all patches) */
    int eval_centre;        /* 0: Phi at the upper cell vertex (Eq.
                               gravpotmult); 1: at the cell's angular centre,
                               still at the outer radius of its shell      */
} orc_grid;

/* Eq. rottransmatrix: R = R_z''(gamma) R_y'(beta) R_z(alpha), x = R xi. */
void orc_rotation(double alpha, double beta, double gamma, double R[9]);

/* s_lm P_l^m(x) for 0<=m<=l<=lmax (Condon-Shortley phase), stored at
 * out[l(l+1)/2+m].  Textbook unnormalised recurrence times s_lm. */
int orc_legendre(int lmax, double x, double *out);

/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration. */
int orc_gauss_legendre(int n, double *x, double *wt);

/* Cell-averaged overlap weight w_jk = 1 - alpha_jk/2 (Sec. 4.2) for the
 * two-patch Yin-Yang grid whose patches both span
 * [pi/2-c, pi/2+c] x [-phe, phe] locally (c in (0,pi/2], phe in (pi/2,pi]),
 * given as the grid's own extent.  alpha_jk is the area fraction of the
 * cell that the other patch covers, integrated over theta by adaptive
 * Gauss-Legendre quadrature of the covered phi-length. */
int orc_overlap_weights(const orc_grid *g, double *w);

/* Angular weights U and prefactors Q of every patch, directly from the
 * definitions above; w may be NULL (w = 1). */
int orc_tables(const orc_grid *g, int lmax, const double *w,
               double *U, double *Q);
/* Same for the cell range [c0, c1) of every patch only (rows outside the
 * range are left untouched). */
int orc_tables_range(const orc_grid *g, int lmax, const double *w,
                     int c0, int c1, double *U, double *Q);

/* Eq. B_CS with Neumaier-compensated sums; only the shells listed in
 * shells[0..n_sh) are computed (shells == NULL: all). */
int orc_moments(const orc_grid *g, int lmax, const double *U,
                const double *rho, int n_sh, const int *shells, double *B);

/* Radial factor of Eq. M_C for target interface r_{n}^+ (0-based shell n)
 * and source shell i at degree l: R_in,i/(r_n)^{l+1} for i <= n,
 * (r_n)^l R_out,i for i > n (Eqs. R_in, R_out). */
double orc_radial_factor(const double *r_edges, int n, int i, int l);

/* Eq. M_C by the direct double sum over shells, every radial factor written
 * as a ratio <= 1; rows listed in shells (NULL: all) are computed. */
int orc_radial(const orc_grid *g, int lmax, const double *B,
               int n_sh, const int *shells, double *M);

/* Eq. gravpotmult at every vertex of the shells listed (NULL: all). */
int orc_expand(const orc_grid *g, int lmax, const double *Q,
               const double *M, int n_sh, const int *shells, double *phi);

/* Eq. gravpotmult at n points (patch p[t], shell i[t], cell c[t]), with Q
 * evaluated on the fly. */
int orc_phi_points(const orc_grid *g, int lmax, const double *M, int n,
                   const int *p, const int *i, const int *c, double *out);

/* Brute force through the addition theorem: for target points
 * (patch p[t], shell i[t], cell c[t]) at the upper vertex,
 *   Phi = -G sum_cells rho w sum_{l<=lmax} K_l(r_n, shell)
 *                 Int_cell P_l(xhat . xhat') dOmega'
 * where all directions are expressed in patch 0's frame through the
 * Yin<->Yang map of Eq. caryytransform (two patches) -- no Euler angle,
 * no Y_lm, no rotation of harmonics.  Only n_patches 1 or 2. */
int orc_brute_phi(const orc_grid *g, int lmax, const double *w,
                  const double *rho, int nq, int n, const int *p,
                  const int *i, const int *c, double *out);

/* Potential of a homogeneous tri-axial ellipsoid (Eq. phiana) with
 * semi-axes a,b,c along X,Y,Z, density rho0, at (X,Y,Z). */
double orc_ellipsoid_phi(double a, double b, double c, double rho0, double G,
                         double X, double Y, double Z);

#ifdef __cplusplus
}
#endif
#endif
