"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), textbook library routines, closed forms,
invariants, special cases and brute force on tiny inputs.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import lpmv

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
S = 1.0 / math.sqrt(2.0)


def read_golden(name):
    blocks, cur = {}, None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line[0].isalpha() and " " not in line:
            cur = blocks.setdefault(line, [])
            continue
        cur.append([S if t == "s" else -S if t == "-s" else float(t) for t in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def m_parity(lmax):
    v = np.zeros((lmax + 1) ** 2)
    for l in range(lmax + 1):
        v[l * l] = 1.0
        for m in range(1, l + 1):
            v[l * l + 2 * m - 1] = v[l * l + 2 * m] = (-1.0) ** m
    return v


def shell_areas(g):
    th = g.theta0 + np.arange(g.n_theta) * g.dtheta
    return np.repeat(g.dphi * (np.cos(th) - np.cos(th + g.dtheta)), g.n_phi)


# --- Eq. rottransmatrix, Eq. yintoxyz, Eq. caryytransform, Sec. 4.1 -----------

def test_euler_angles_give_printed_frames():
    gd = read_golden("yinyang_frames.txt")
    R_yin = O.rotation(*(np.pi * gd["EULER_YIN"][0]))
    R_yang = O.rotation(*(np.pi * gd["EULER_YANG"][0]))
    assert np.abs(R_yin - gd["M_YIN"]).max() < 1e-15
    assert np.abs(R_yang - gd["M_YIN"] @ gd["P"]).max() < 1e-15
    # Yang = Yin rotated by pi about the common polar axis (global z)
    assert np.abs(R_yang - np.diag([-1.0, -1.0, 1.0]) @ R_yin).max() < 1e-15
    # the axis S is global z in both frames
    assert np.abs(R_yin @ gd["AXIS_S"][0] - [0, 0, 1]).max() < 1e-15


def test_rotation_is_orthonormal_and_composes():
    rng = np.random.default_rng(1)
    for a, b, c in rng.uniform(-3, 3, size=(5, 3)):
        R = O.rotation(a, b, c)
        assert np.abs(R @ R.T - np.eye(3)).max() < 1e-15
        Rz = lambda t: np.array([[np.cos(t), np.sin(t), 0], [-np.sin(t), np.cos(t), 0], [0, 0, 1]])
        Ry = lambda t: np.array([[np.cos(t), 0, -np.sin(t)], [0, 1, 0], [np.sin(t), 0, np.cos(t)]])
        assert np.abs(R - Rz(c) @ Ry(b) @ Rz(a)).max() < 1e-15


# --- Eq. Y_l^m: associated Legendre with Condon-Shortley phase -----------------

@pytest.mark.parametrize("x", [-0.97, -0.4, 0.0, 0.31, 0.77, 0.999])
def test_legendre_matches_scipy(x):
    L = 40
    P = O.legendre(L, x)
    for l in range(L + 1):
        for m in range(l + 1):
            ref = lpmv(m, l, x) * math.sqrt(math.factorial(l - m) / math.factorial(l + m))
            assert abs(P[l * (l + 1) // 2 + m] - ref) <= 1e-13 * max(1.0, abs(ref)), (l, m)


def test_gauss_legendre_exact_for_polynomials():
    x, w = O.gauss_legendre(12)
    for k in range(24):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-15


# --- Eqs. R_in, R_out and the radial factors of Eq. M_C ------------------------

def test_radial_factors_match_direct_integration():
    e = W.geometric_edges(12, 1.3)
    x, wq = O.gauss_legendre(40)
    for n in (0, 3, 11):
        rn = e[n + 1]
        for i in range(12):
            a, b = e[i], e[i + 1]
            r = 0.5 * (b - a) * x + 0.5 * (a + b)
            for l in (0, 1, 2, 3, 7, 25):
                if i <= n:
                    ref = 0.5 * (b - a) * np.sum(wq * r ** (l + 2)) / rn ** (l + 1)
                else:
                    ref = 0.5 * (b - a) * np.sum(wq * r ** (1 - l)) * rn ** l
                got = O.radial_factor(e, n, i, l)
                assert abs(got - ref) <= 1e-13 * abs(ref), (n, i, l, got, ref)


# --- Sec. 4.2 overlap weights ---------------------------------------------------

def test_overlap_weights_area_invariants():
    g = W.config1()
    w = O.overlap_weights(g)
    A = shell_areas(g)
    # Eq. after A_lm_mult: sum_g int w dOmega = 4 pi
    assert abs(2 * np.sum(w * A) - 4 * math.pi) < 1e-13
    # the doubly covered area of the unbuffered Yin-Yang grid is 3 sqrt2 pi - 4 pi
    assert abs(np.sum((1 - w) * 2 * A) - (3 * math.sqrt(2) - 4) * math.pi) < 1e-13
    assert w.min() >= 0.5 - 1e-15 and w.max() <= 1.0
    wg = w.reshape(g.n_theta, g.n_phi)
    assert np.abs(wg - wg[::-1, :]).max() < 1e-14 and np.abs(wg - wg[:, ::-1]).max() < 1e-14


def _covered_fraction_by_rule(g, j, k, n=1200):
    """Midpoint rule in (theta, phi) of the indicator 'inside the other patch',
    the patch membership tested through the Yin/Yang Euler rotations."""
    R0 = O.rotation(*g.euler[0])
    R1 = O.rotation(*g.euler[1])
    t = g.theta0 + (j + (np.arange(n) + 0.5) / n) * g.dtheta
    p = g.phi0 + (k + (np.arange(n) + 0.5) / n) * g.dphi
    T, Pp = np.meshgrid(t, p, indexing="ij")
    v = np.stack([np.sin(T) * np.cos(Pp), np.sin(T) * np.sin(Pp), np.cos(T)])
    x = np.tensordot(R0, v, 1)
    loc = np.tensordot(R1.T, x, 1)
    th1 = np.arccos(np.clip(loc[2], -1, 1))
    ph1 = np.arctan2(loc[1], loc[0])
    th_hi = g.theta0 + g.n_theta * g.dtheta
    ph_hi = g.phi0 + g.n_phi * g.dphi
    inside = (th1 >= g.theta0) & (th1 <= th_hi) & (ph1 >= g.phi0) & (ph1 <= ph_hi)
    return np.sum(inside * np.sin(T)) / np.sum(np.sin(T))


def test_overlap_weights_match_point_membership():
    g = W.config1()
    w = O.overlap_weights(g).reshape(g.n_theta, g.n_phi)
    cut = [(j, k) for j in range(g.n_theta) for k in range(g.n_phi) if 0.5 < w[j, k] < 1.0]
    assert len(cut) > 10
    for j, k in cut[:: max(1, len(cut) // 6)]:
        alpha = _covered_fraction_by_rule(g, j, k)
        assert abs((1 - 0.5 * alpha) - w[j, k]) < 2e-3, (j, k)


# --- closed forms ---------------------------------------------------------------

def test_ellipsoid_closed_form_limits():
    G = 1.0
    # homogeneous sphere: inside -2 pi G rho (R^2 - r^2/3), outside -G M / r
    for r in (0.0, 0.3, 0.99):
        assert abs(O.ellipsoid_phi(1, 1, 1, 1, G, r, 0, 0) + 2 * math.pi * (1 - r * r / 3)) < 1e-13
    for r in (1.5, 4.0, 30.0):
        assert abs(O.ellipsoid_phi(1, 1, 1, 1, G, 0, r, 0) + 4 * math.pi / 3 / r) < 1e-13 / r
    # far field of a tri-axial body tends to -G M / r
    a, b, c = 0.5, 0.4, 0.3
    M = 4 * math.pi / 3 * a * b * c
    for d in ([1, 0, 0], [0, 1, 1], [1, -2, 0.5]):
        d = np.array(d) / np.linalg.norm(d)
        r = 200.0
        assert abs(O.ellipsoid_phi(a, b, c, 1, G, *(r * d)) * r / M + 1) < 1e-5
    # interior potential is a quadratic form: second differences are constant
    h = 0.05
    f = lambda x: O.ellipsoid_phi(a, b, c, 1, G, x, 0.02, 0.01)
    d2 = [(f(x + h) - 2 * f(x) + f(x - h)) / h ** 2 for x in (-0.2, 0.0, 0.2)]
    assert max(d2) - min(d2) < 1e-8
    # Poisson: the Laplacian inside is 4 pi G rho
    lap = 0.0
    for e in np.eye(3):
        p0 = np.array([0.05, 0.02, 0.01])
        lap += (O.ellipsoid_phi(a, b, c, 1, G, *(p0 + h * e)) - 2 * O.ellipsoid_phi(a, b, c, 1, G, *p0)
                + O.ellipsoid_phi(a, b, c, 1, G, *(p0 - h * e))) / h ** 2
    assert abs(lap - 4 * math.pi) < 1e-7


def _sphere_rho(g, n_in):
    rho = np.zeros(g.shape)
    rho[:, :n_in] = 1.0
    return rho


def test_homogeneous_sphere_monopole_on_yinyang():
    g = W.yinyang(8, W.uniform_edges(10), 0)
    w = O.overlap_weights(g)
    R = g.r_edges[6]
    phi, *_ = O.potential(g, 0, _sphere_rho(g, 6), w)
    r = g.r_edges[1:]
    exact = np.where(r >= R, -4 * math.pi / 3 * R ** 3 / r, -2 * math.pi * (R * R - r * r / 3))
    for p in range(2):
        got = phi[p].reshape(g.n_r, -1)
        assert np.abs(got - exact[:, None]).max() < 1e-13


def test_homogeneous_sphere_all_degrees_on_polar_grid():
    g = W.polar(8, 16, W.uniform_edges(9), 6)
    R = g.r_edges[4]
    phi, B, *_ = O.potential(g, 6, _sphere_rho(g, 4))
    assert np.abs(B[:, 1:]).max() < 1e-14
    r = g.r_edges[1:]
    exact = np.where(r >= R, -4 * math.pi / 3 * R ** 3 / r, -2 * math.pi * (R * R - r * r / 3))
    assert np.abs(phi[0].reshape(g.n_r, -1) - exact[:, None]).max() < 1e-13


# --- special cases of the method ------------------------------------------------

def test_polar_grid_weights_reduce_to_T_C_S():
    """N_g = 1, Euler angles 0: U = (2/delta_m) s_lm T_j C_k (or S_k) of
    Eqs. T_lm, C_k^m, S_k^m (Sec. 2.2), integrated here by scipy."""
    g = W.polar(6, 10, W.uniform_edges(2), 7)
    U, _ = O.tables(g, 7)
    for j in (0, 2, 5):
        t1, t2 = g.theta0 + j * g.dtheta, g.theta0 + (j + 1) * g.dtheta
        for k in (0, 3, 9):
            p1, p2 = g.phi0 + k * g.dphi, g.phi0 + (k + 1) * g.dphi
            for l in range(8):
                for m in range(l + 1):
                    s = math.sqrt(math.factorial(l - m) / math.factorial(l + m))
                    T = integrate.quad(lambda t: math.sin(t) * lpmv(m, l, math.cos(t)), t1, t2,
                                       epsabs=1e-15, epsrel=1e-14)[0]
                    if m == 0:
                        ref = s * T * (p2 - p1)
                        got = U[0, j * g.n_phi + k, l * l]
                        assert abs(got - ref) < 1e-14, (l, m)
                    else:
                        Ck = (math.sin(m * p2) - math.sin(m * p1)) / m
                        Sk = (math.cos(m * p1) - math.cos(m * p2)) / m
                        assert abs(U[0, j * g.n_phi + k, l * l + 2 * m - 1] - 2 * s * T * Ck) < 1e-14
                        assert abs(U[0, j * g.n_phi + k, l * l + 2 * m] - 2 * s * T * Sk) < 1e-14


def test_discrete_orthogonality_on_polar_grid():
    g = W.polar(8, 16, W.uniform_edges(3), 7)
    U, _ = O.tables(g, 7)
    th = g.theta0 + (np.arange(g.n_theta) + 0.5) * g.dtheta
    ph = g.phi0 + (np.arange(g.n_phi) + 0.5) * g.dphi
    for mp in range(0, 5):
        for kind in ("c", "s"):
            if kind == "s" and mp == 0:
                continue
            f = np.cos(mp * ph) if kind == "c" else np.sin(mp * ph)
            rho = np.broadcast_to((1.0 + th[:, None] ** 2) * f[None, :], g.shape[1:]).copy()[None]
            B = O.moments(g, 7, U, rho)
            for l in range(8):
                for m in range(l + 1):
                    for col, kk in ([(l * l, "c")] if m == 0 else [(l * l + 2 * m - 1, "c"), (l * l + 2 * m, "s")]):
                        if (m, kk) != (mp, kind):
                            assert np.abs(B[:, col]).max() < 1e-13, (mp, kind, l, m, kk)


def test_oracle_matches_addition_theorem_brute_force():
    g = W.yinyang(4, W.geometric_edges(6, 1.5), 8)
    w = O.overlap_weights(g)
    rho = W.random_rho(g, 7)
    phi, *_ = O.potential(g, 8, rho, w)
    pts = [(p, i, c) for p in range(2) for i in (0, 2, 5) for c in (0, 7, 23, 47)]
    p, i, c = map(np.array, zip(*pts))
    bf = O.brute_phi(g, 8, w, rho, p, i, c, nq=12)
    got = phi.reshape(2, g.n_r, -1)[p, i, c]
    assert np.abs(got - bf).max() <= 1e-13 * np.abs(bf).max()


@pytest.mark.slow
def test_oracle_matches_brute_force_high_degree():
    g = W.yinyang(8, W.uniform_edges(5), 24)
    w = O.overlap_weights(g)
    rho = W.random_rho(g, 8, positive=False)
    phi, *_ = O.potential(g, 24, rho, w)
    pts = [(p, i, c) for p in range(2) for i in (1, 4) for c in (5, 100, 191)]
    p, i, c = map(np.array, zip(*pts))
    bf = O.brute_phi(g, 24, w, rho, p, i, c, nq=16)
    got = phi.reshape(2, g.n_r, -1)[p, i, c]
    assert np.abs(got - bf).max() <= 1e-12 * np.abs(bf).max()


def test_yang_tables_are_parity_images_of_yin():
    """Sec. 4.2: theta equal, phi shifted by pi, so Q_Yang = (-1)^m Q_Yin; the
    same holds for the cell integrals U."""
    g = W.yinyang(8, W.uniform_edges(2), 12)
    U, Q = O.tables(g, 12, O.overlap_weights(g))
    par = m_parity(12)
    assert np.abs(U[1] - U[0] * par).max() < 1e-14 * np.abs(U).max()
    assert np.abs(Q[1] - Q[0] * par).max() < 1e-14 * np.abs(Q).max()


def test_frame_independence():
    """Global frame aligned with Yin (Yin (0,0,0), Yang (pi/2,pi/2,pi/2), whose
    matrix is the Yin<->Yang map) gives the same physical potential."""
    g1 = W.yinyang(8, W.uniform_edges(6), 10)
    g2 = W.yinyang(8, W.uniform_edges(6), 10)
    g2.euler = np.array([[0.0, 0.0, 0.0], [np.pi / 2, np.pi / 2, np.pi / 2]])
    assert np.abs(O.rotation(*g2.euler[1]) - W.YY_SWAP).max() < 1e-15
    w = O.overlap_weights(g1)
    rho = W.random_rho(g1, 3)
    phi1, *_ = O.potential(g1, 10, rho, w)
    phi2, *_ = O.potential(g2, 10, rho, w)
    assert np.abs(phi1 - phi2).max() < 1e-13 * np.abs(phi1).max()


def test_swap_symmetry():
    g = W.yinyang(8, W.uniform_edges(6), 10)
    w = O.overlap_weights(g)
    rho = W.random_rho(g, 4)
    phi, *_ = O.potential(g, 10, rho, w)
    phis, *_ = O.potential(g, 10, rho[::-1].copy(), w)
    assert np.abs(phis - phi[::-1]).max() < 1e-13 * np.abs(phi).max()


def test_rotated_single_patch_gives_same_potential():
    """Eq. ylm_transform: a full polar grid whose frame is rotated by arbitrary
    Euler angles, with the density rotated with it, gives the same values."""
    g0 = W.polar(8, 16, W.uniform_edges(4), 8)
    e = (0.7, 1.1, -0.4)
    g1 = W.polar(8, 16, W.uniform_edges(4), 8, euler=e)
    rho = W.random_rho(g0, 5)
    phi0, *_ = O.potential(g0, 8, rho)
    phi1, *_ = O.potential(g1, 8, rho)
    assert np.abs(phi0 - phi1).max() < 1e-13 * np.abs(phi0).max()


def test_ellipsoid_potential_converges_to_closed_form():
    """Sec. 5.1: the discretised potential approaches Chandrasekhar's solution;
    the error shrinks with resolution and is largest near the surface."""
    errs = []
    for nt, nr in ((8, 16), (16, 32)):
        g = W.yinyang(nt, W.uniform_edges(nr), 12)
        rho = W.cell_average(g, W.Ellipsoid(), sub=4)
        w = O.overlap_weights(g)
        phi, *_ = O.potential(g, 12, rho, w)
        i = np.arange(g.n_r - 4, g.n_r)  # shells well outside the body
        th = g.theta0 + (np.arange(g.n_theta) + 1) * g.dtheta
        ph = g.phi0 + (np.arange(g.n_phi) + 1) * g.dphi
        T, P = np.meshgrid(th, ph, indexing="ij")
        v = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)]).reshape(3, -1)
        e = W.Ellipsoid()
        err = 0.0
        for n in i:
            x = g.r_edges[n + 1] * v
            import torch
            X, Y, Z = e.to_body(torch.tensor(x[0]), torch.tensor(x[1]), torch.tensor(x[2]), "torch")
            ref = np.array([O.ellipsoid_phi(e.a, e.b, e.c, 1.0, 1.0, a, b, c)
                            for a, b, c in zip(X.numpy(), Y.numpy(), Z.numpy())])
            err = max(err, np.abs(phi[0, n].reshape(-1) - ref).max() / np.abs(ref).max())
        errs.append(err)
    assert errs[1] < errs[0] and errs[1] < 2e-2, errs


def test_per_patch_overlap_weights_scale_each_patch_own_rows():
    """U is w_jk times the cell integral of the patch's own harmonics
    (Eqs. U_C/U_S): weights given per patch scale only that patch's rows;
    equal per-patch weights reproduce the shared-weight tables exactly."""
    g = W.config1()
    rng = np.random.Generator(np.random.PCG64(3))
    w = rng.uniform(0.2, 1.0, size=(2, g.n_ang))
    U1, Q1 = O.tables(g, 6, None)
    Uw, Qw = O.tables(g, 6, w)
    assert np.array_equal(Qw, Q1)
    for p in range(2):
        assert np.abs(Uw[p] - w[p][:, None] * U1[p]).max() < 1e-15 * np.abs(U1).max()
    Us, _ = O.tables(g, 6, w[0])
    Ue, _ = O.tables(g, 6, np.stack([w[0], w[0]]))
    assert np.array_equal(Us, Ue)


# --- convergence of the Yin-Yang discretisation (Sec. 4.2, Sec. 5) --------------

def _global_harmonic(l, m, kind, R):
    """s_lm P_l^m(cos theta) {cos, sin}(m phi) in global angles, for a density
    given in the Yin frame (x_global = R x_Yin); P_l^m from scipy, with the
    Condon-Shortley phase."""
    s = math.sqrt(math.factorial(l - m) / math.factorial(l + m))

    def f(x, y, z, xp):
        import torch
        X = R[0, 0] * x + R[0, 1] * y + R[0, 2] * z
        Y = R[1, 0] * x + R[1, 1] * y + R[1, 2] * z
        Z = R[2, 0] * x + R[2, 1] * y + R[2, 2] * z
        ct = (Z / torch.sqrt(X * X + Y * Y + Z * Z)).numpy()
        ph = torch.atan2(Y, X).numpy()
        return torch.from_numpy(s * lpmv(m, l, ct) * (np.cos(m * ph) if kind == "c" else np.sin(m * ph)))
    return f


def test_yinyang_weights_converge_to_orthogonality():
    """Moments of a cell-averaged real harmonic on the Yin-Yang grid tend to
    4 pi/(2l+1) in its own column and zero elsewhere (orthogonality of the
    Y_lm, Eqs. A_lm_mult/B_lm_mult with the overlap weights); the error falls
    about four-fold per halving of the cell size."""
    L = 5
    cases = [(0, 0, "c"), (1, 0, "c"), (2, 1, "c"), (3, 2, "s"), (4, 3, "c"), (5, 1, "s")]
    errs = []
    for k in (8, 16):
        g = W.yinyang(k, W.uniform_edges(1), L)
        R = O.rotation(*g.euler[0])
        U, _ = O.tables(g, L, O.overlap_weights(g), want_Q=False)
        err = 0.0
        for l, m, kind in cases:
            B = O.moments(g, L, U, W.cell_average(g, _global_harmonic(l, m, kind, R), sub=4))[0]
            ref = np.zeros_like(B)
            ref[l * l if m == 0 else l * l + 2 * m - (kind == "c")] = 4 * math.pi / (2 * l + 1)
            err = max(err, np.abs(B - ref).max())
        errs.append(err)
    assert errs[0] < 0.15 and errs[1] < 0.04 and errs[0] / errs[1] > 3.0, errs


def test_one_patch_and_yinyang_agree_for_smooth_density():
    """The same smooth density on a one-patch polar grid and on the Yin-Yang
    grid at the same cell size gives radial sums M that agree to O(Delta^2)."""
    L = 8
    blobs = W.Blobs(np.array([[0.3, -0.2, 0.25], [-0.35, 0.1, -0.3]]), np.array([0.25, 0.3]), np.array([1.0, 0.7]))
    edges = W.uniform_edges(6)
    diffs = []
    for k in (8, 16):
        yy = W.yinyang(k, edges, L)
        po = W.polar(2 * k, 4 * k, edges, L, frame=O.rotation(*yy.euler[0]).T)
        M = []
        for g, w in ((yy, O.overlap_weights(yy)), (po, None)):
            U, _ = O.tables(g, L, w, want_Q=False)
            M.append(O.radial(g, L, O.moments(g, L, U, W.cell_average(g, blobs, sub=4))))
        diffs.append(np.abs(M[0] - M[1]).max() / np.abs(M[1]).max())
    assert diffs[0] < 1e-3 and diffs[1] < 2.5e-4 and diffs[0] / diffs[1] > 3.0, diffs


# --- evaluation at the angular cell centres ---------------------------------------

def test_centre_evaluation_matches_brute_force():
    """Phi at the cells' angular centres (outer shell radius) from the oracle's
    tables agrees with the addition-theorem brute force at the same points."""
    g = W.yinyang(4, W.geometric_edges(6, 1.5), 8)
    g.eval_point = "centre"
    w = O.overlap_weights(g)
    rho = W.random_rho(g, 9)
    phi, *_ = O.potential(g, 8, rho, w)
    pts = [(p, i, c) for p in range(2) for i in (0, 3, 5) for c in (0, 9, 47)]
    p, i, c = map(np.array, zip(*pts))
    bf = O.brute_phi(g, 8, w, rho, p, i, c, nq=12)
    got = phi.reshape(2, g.n_r, -1)[p, i, c]
    assert np.abs(got - bf).max() <= 1e-13 * np.abs(bf).max()
    gv = W.yinyang(4, W.geometric_edges(6, 1.5), 8)
    phv, *_ = O.potential(gv, 8, rho, w)
    assert np.abs(phv - phi).max() > 1e-6 * np.abs(phi).max()  # a different point set


def test_centre_evaluation_of_homogeneous_sphere():
    g = W.yinyang(8, W.uniform_edges(10), 0)
    g.eval_point = "centre"
    w = O.overlap_weights(g)
    R = g.r_edges[6]
    phi, *_ = O.potential(g, 0, _sphere_rho(g, 6), w)
    r = g.r_edges[1:]
    exact = np.where(r >= R, -4 * math.pi / 3 * R ** 3 / r, -2 * math.pi * (R * R - r * r / 3))
    assert np.abs(phi.reshape(2, g.n_r, -1) - exact[None, :, None]).max() < 1e-13


def test_uniform_density_on_yinyang_has_only_small_spurious_multipoles():
    """A uniform shell on the Yin-Yang grid: the monopole is exactly 4 pi; the
    dipole vanishes to rounding, since the grid with its overlap weights is
    symmetric under y -> -y, z -> -z and the Yin<->Yang map (which sends x to
    -x); degrees 2..6 carry spurious terms from the cell-constant weights of
    the cells the overlap boundary cuts, falling about four-fold per halving
    of the cell size."""
    errs = []
    for k in (8, 16):
        g = W.yinyang(k, W.uniform_edges(1), 6)
        U, _ = O.tables(g, 6, O.overlap_weights(g), want_Q=False)
        B = O.moments(g, 6, U, np.ones(g.shape))[0]
        assert abs(B[0] - 4 * math.pi) < 1e-13
        assert np.abs(B[1:4]).max() < 1e-14
        errs.append(np.abs(B[4:]).max())
    assert errs[0] < 2e-2 and errs[0] / errs[1] > 3.0, errs
