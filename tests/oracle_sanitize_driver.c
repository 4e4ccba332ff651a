/*
 * Runs every routine of the CPU oracle on small grids, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).
 * Exit status 0 when every call succeeds, every result is finite, the
 * expansion agrees with the point evaluation, bad arguments are rejected,
 * and the monopole of a uniform density is exact.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/oracle.h"

static int fails = 0;

#define CHECK(cond, what)                                \
    do {                                                 \
        if (!(cond)) {                                   \
            fprintf(stderr, "check failed: %s\n", what); \
            ++fails;                                     \
        }                                                \
    } while (0)

static int all_finite(const double *x, size_t n) {
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(x[k])) return 0;
    return 1;
}

/* one grid through tables, moments, radial sums, expansion, point values
 * and (one or two patches) the brute-force sum */
static void run_grid(const orc_grid *g, int lmax, const double *w, unsigned seed) {
    const int n_ang = g->n_theta * g->n_phi, n_lm = (lmax + 1) * (lmax + 1);
    const size_t cells = (size_t)g->n_patches * g->n_r * n_ang;
    double *U = malloc(sizeof(double) * g->n_patches * n_ang * n_lm);
    double *Q = malloc(sizeof(double) * g->n_patches * n_ang * n_lm);
    double *rho = malloc(sizeof(double) * cells);
    double *B = malloc(sizeof(double) * g->n_r * n_lm);
    double *M = malloc(sizeof(double) * g->n_r * n_lm);
    double *phi = malloc(sizeof(double) * cells);
    srand(seed);
    for (size_t k = 0; k < cells; ++k) rho[k] = (double)rand() / RAND_MAX;
    CHECK(orc_tables(g, lmax, w, U, Q) == 0, "tables");
    CHECK(orc_moments(g, lmax, U, rho, 0, NULL, B) == 0, "moments");
    CHECK(orc_radial(g, lmax, B, 0, NULL, M) == 0, "radial");
    CHECK(orc_expand(g, lmax, Q, M, 0, NULL, phi) == 0, "expand");
    CHECK(all_finite(U, (size_t)g->n_patches * n_ang * n_lm) && all_finite(M, (size_t)g->n_r * n_lm) &&
              all_finite(phi, cells),
          "finite results");
    int p[3] = {0, g->n_patches - 1, 0}, i[3] = {0, g->n_r - 1, g->n_r / 2}, c[3] = {0, n_ang - 1, n_ang / 2};
    double pt[3], bf[3];
    CHECK(orc_phi_points(g, lmax, M, 3, p, i, c, pt) == 0, "phi_points");
    for (int t = 0; t < 3; ++t) {
        double ref = phi[((size_t)p[t] * g->n_r + i[t]) * n_ang + c[t]];
        CHECK(fabs(pt[t] - ref) <= 1e-12 * fabs(ref), "phi_points equals the expansion");
    }
    if (g->n_patches <= 2) {
        CHECK(orc_brute_phi(g, lmax, w, rho, 4, 3, p, i, c, bf) == 0, "brute_phi");
        CHECK(all_finite(bf, 3), "finite brute force");
    }
    /* shell subsets */
    int sh[2] = {g->n_r - 1, 0};
    CHECK(orc_moments(g, lmax, U, rho, 2, sh, B) == 0, "moments on a shell subset");
    CHECK(orc_radial(g, lmax, B, 2, sh, M) == 0, "radial on a shell subset");
    CHECK(orc_expand(g, lmax, Q, M, 2, sh, phi) == 0, "expand on a shell subset");
    free(U);
    free(Q);
    free(rho);
    free(B);
    free(M);
    free(phi);
}

int main(void) {
    const double pi = acos(-1.0);
    double r[5] = {0.0, 0.3, 0.5, 0.8, 1.0};

    /* Yin-Yang at pi/8: 2 x 6 cells per patch, no buffer */
    double eul[6] = {pi / 2, pi / 4, 3 * pi / 2, pi / 2, pi / 4, pi / 2};
    orc_grid yy = {2, 4, 2, 6, r, pi / 4, -3 * pi / 4, pi / 4, pi / 4, eul, 1.0, 0};
    double w[12];
    CHECK(orc_overlap_weights(&yy, w) == 0, "overlap weights");
    double area = 0.0;
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 6; ++k) {
            double t0 = pi / 4 + j * pi / 4;
            area += 2.0 * w[j * 6 + k] * (pi / 4) * (cos(t0) - cos(t0 + pi / 4));
        }
    CHECK(fabs(area - 4 * pi) < 1e-12, "weighted area of both patches is 4 pi");
    run_grid(&yy, 5, w, 1u);

    /* full polar grid, one patch, turned */
    double e1[3] = {0.4, 0.9, -1.3};
    orc_grid po = {1, 4, 4, 8, r, 0.0, -pi, pi / 4, pi / 4, e1, 1.0, 0};
    run_grid(&po, 4, NULL, 2u);

    /* a uniform density on the polar grid has only the monopole */
    {
        const int lmax = 2, n_lm = 9, n_ang = 32;
        double U[32 * 9], Q[32 * 9], rho[4 * 32], B[4 * 9];
        for (int k = 0; k < 4 * 32; ++k) rho[k] = 1.0;
        CHECK(orc_tables(&po, lmax, NULL, U, Q) == 0, "tables (uniform)");
        CHECK(orc_moments(&po, lmax, U, rho, 0, NULL, B) == 0, "moments (uniform)");
        for (int i = 0; i < 4; ++i) {
            CHECK(fabs(B[i * n_lm] - 4 * pi) < 1e-12, "monopole moment is 4 pi");
            for (int q = 1; q < n_lm; ++q) CHECK(fabs(B[i * n_lm + q]) < 1e-13, "higher moments vanish");
        }
        (void)n_ang;
    }

    /* three patches with their own weights (general path) */
    double e3[9] = {0.1, 0.7, 0.2, 1.9, 1.1, -0.4, -2.2, 2.3, 0.9};
    double w3[3 * 12];
    for (int k = 0; k < 36; ++k) w3[k] = 1.0 / 3.0;
    orc_grid three = {3, 4, 2, 6, r, pi / 4, -3 * pi / 4, pi / 4, pi / 4, e3, 1.0, 12};
    run_grid(&three, 3, w3, 3u);

    /* special functions */
    double pl[15], x[16], wt[16], R[9];
    CHECK(orc_legendre(4, 0.3, pl) == 0 && all_finite(pl, 15), "legendre");
    CHECK(orc_gauss_legendre(16, x, wt) == 0 && all_finite(x, 16) && all_finite(wt, 16), "gauss-legendre");
    orc_rotation(0.3, 1.2, -0.7, R);
    CHECK(all_finite(R, 9), "rotation");
    CHECK(isfinite(orc_radial_factor(r, 2, 1, 3)) && isfinite(orc_radial_factor(r, 1, 3, 2)), "radial factor");
    double inside = orc_ellipsoid_phi(0.5, 0.4, 0.3, 1.0, 1.0, 0.1, 0.0, 0.05);
    double outside = orc_ellipsoid_phi(0.5, 0.4, 0.3, 1.0, 1.0, 2.0, 1.0, -1.0);
    CHECK(isfinite(inside) && isfinite(outside) && inside < outside && outside < 0.0, "ellipsoid potential");

    /* bad arguments are rejected */
    CHECK(orc_legendre(-1, 0.3, pl) < 0, "negative lmax rejected");
    orc_grid bad = yy;
    bad.n_r = 0;
    CHECK(orc_tables(&bad, 2, NULL, x, wt) < 0, "empty grid rejected");

    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("oracle sanitize driver: all checks passed\n");
    return fails ? 1 : 0;
}
