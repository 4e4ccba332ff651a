"""Plain FP64 CPU oracle of the multipole gravity solver (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package; the
product library never does.  The C code (``oracle.c``) is single-threaded
and shares no source with the GPU path.  ``tables_parallel`` only splits the
same single-threaded table routine over cell ranges in worker processes, so
that large grids finish in tests; each cell is still computed by the plain
routine.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ProcessPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain C99, IEEE arithmetic)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _OrcGrid(C.Structure):
    _fields_ = [
        ("n_patches", C.c_int), ("n_r", C.c_int), ("n_theta", C.c_int), ("n_phi", C.c_int),
        ("r_edges", C.POINTER(C.c_double)),
        ("theta0", C.c_double), ("phi0", C.c_double), ("dtheta", C.c_double), ("dphi", C.c_double),
        ("euler", C.POINTER(C.c_double)),
        ("G", C.c_double),
        ("w_stride", C.c_int),
        ("eval_centre", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        gp = C.POINTER(_OrcGrid)
        L.orc_rotation.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_legendre.argtypes = [C.c_int, C.c_double, dp]
        L.orc_gauss_legendre.argtypes = [C.c_int, dp, dp]
        L.orc_overlap_weights.argtypes = [gp, dp]
        L.orc_tables_range.argtypes = [gp, C.c_int, dp, C.c_int, C.c_int, dp, dp]
        L.orc_moments.argtypes = [gp, C.c_int, dp, dp, C.c_int, ip, dp]
        L.orc_radial_factor.argtypes = [dp, C.c_int, C.c_int, C.c_int]
        L.orc_radial_factor.restype = C.c_double
        L.orc_radial.argtypes = [gp, C.c_int, dp, C.c_int, ip, dp]
        L.orc_expand.argtypes = [gp, C.c_int, dp, dp, C.c_int, ip, dp]
        L.orc_phi_points.argtypes = [gp, C.c_int, dp, C.c_int, ip, ip, ip, dp]
        L.orc_brute_phi.argtypes = [gp, C.c_int, dp, dp, C.c_int, C.c_int, ip, ip, ip, dp]
        L.orc_ellipsoid_phi.argtypes = [C.c_double] * 8
        L.orc_ellipsoid_phi.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


class _G:
    """Keeps the ctypes grid struct and the arrays it points to alive."""

    def __init__(self, grid):
        self.r = _f64(grid.r_edges)
        self.e = _f64(np.asarray(grid.euler).reshape(-1))
        s = _OrcGrid()
        s.n_patches, s.n_r, s.n_theta, s.n_phi = grid.n_patches, grid.n_r, grid.n_theta, grid.n_phi
        s.r_edges, s.euler = _dp(self.r), _dp(self.e)
        s.theta0, s.phi0, s.dtheta, s.dphi = grid.theta0, grid.phi0, grid.dtheta, grid.dphi
        s.G = grid.G
        s.eval_centre = int(getattr(grid, "eval_point", "vertex") == "centre")
        self.s = s

    def set_w_stride(self, w, n_ang):
        """Weights given per patch ([n_patches, n_ang]) or one set for all."""
        if w is not None and w.size not in (n_ang, self.s.n_patches * n_ang):
            raise ValueError("overlap weights must have n_ang or n_patches*n_ang entries")
        self.s.w_stride = n_ang if (w is not None and w.size != n_ang) else 0

    @property
    def ref(self):
        return C.byref(self.s)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def n_lm(lmax):
    return (lmax + 1) ** 2


def rotation(alpha, beta, gamma):
    R = np.zeros(9)
    lib().orc_rotation(alpha, beta, gamma, _dp(R))
    return R.reshape(3, 3)


def legendre(lmax, x):
    out = np.zeros((lmax + 1) * (lmax + 2) // 2)
    _check(lib().orc_legendre(lmax, float(x), _dp(out)), "legendre")
    return out


def gauss_legendre(n):
    x, w = np.zeros(n), np.zeros(n)
    _check(lib().orc_gauss_legendre(n, _dp(x), _dp(w)), "gauss_legendre")
    return x, w


def radial_factor(r_edges, n, i, l):
    r = _f64(r_edges)
    return lib().orc_radial_factor(_dp(r), n, i, l)


def overlap_weights(grid):
    g = _G(grid)
    w = np.zeros(grid.n_theta * grid.n_phi)
    _check(lib().orc_overlap_weights(g.ref, _dp(w)), "overlap_weights")
    return w


def tables(grid, lmax, w=None, cells=None, want_U=True, want_Q=True):
    """U, Q of shape [n_patches, n_ang, n_lm] (rows outside `cells` zero)."""
    g = _G(grid)
    n_ang = grid.n_theta * grid.n_phi
    U = np.zeros((grid.n_patches, n_ang, n_lm(lmax))) if want_U else None
    Q = np.zeros((grid.n_patches, n_ang, n_lm(lmax))) if want_Q else None
    c0, c1 = (0, n_ang) if cells is None else cells
    wv = None if w is None else _f64(w)
    g.set_w_stride(wv, n_ang)
    _check(lib().orc_tables_range(g.ref, lmax, _dp(wv), c0, c1, _dp(U), _dp(Q)), "tables")
    return U, Q


def _tables_worker(args):
    grid, lmax, w, c0, c1, want_U, want_Q = args
    U, Q = tables(grid, lmax, w, (c0, c1), want_U, want_Q)
    return c0, c1, (U[:, c0:c1] if U is not None else None), (Q[:, c0:c1] if Q is not None else None)


def tables_parallel(grid, lmax, w=None, workers=8, want_U=True, want_Q=True):
    """Same as tables(), cell ranges computed in worker processes."""
    n_ang = grid.n_theta * grid.n_phi
    U = np.zeros((grid.n_patches, n_ang, n_lm(lmax))) if want_U else None
    Q = np.zeros((grid.n_patches, n_ang, n_lm(lmax))) if want_Q else None
    chunk = max(1, (n_ang + 4 * workers - 1) // (4 * workers))
    jobs = [(grid, lmax, w, c, min(n_ang, c + chunk), want_U, want_Q) for c in range(0, n_ang, chunk)]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for c0, c1, u, q in ex.map(_tables_worker, jobs):
            if U is not None:
                U[:, c0:c1] = u
            if Q is not None:
                Q[:, c0:c1] = q
    return U, Q


def moments(grid, lmax, U, rho, shells=None, B=None):
    g = _G(grid)
    U = _f64(U)
    rho = _f64(rho)
    if B is None:
        B = np.zeros((grid.n_r, n_lm(lmax)))
    sh = _i32(shells)
    _check(lib().orc_moments(g.ref, lmax, _dp(U), _dp(rho), 0 if sh is None else len(sh), _ip(sh), _dp(B)),
           "moments")
    return B


def radial(grid, lmax, B, shells=None):
    g = _G(grid)
    B = _f64(B)
    M = np.zeros((grid.n_r, n_lm(lmax)))
    sh = _i32(shells)
    _check(lib().orc_radial(g.ref, lmax, _dp(B), 0 if sh is None else len(sh), _ip(sh), _dp(M)), "radial")
    return M


def expand(grid, lmax, Q, M, shells=None):
    g = _G(grid)
    Q, M = _f64(Q), _f64(M)
    phi = np.zeros((grid.n_patches, grid.n_r, grid.n_theta * grid.n_phi))
    sh = _i32(shells)
    _check(lib().orc_expand(g.ref, lmax, _dp(Q), _dp(M), 0 if sh is None else len(sh), _ip(sh), _dp(phi)),
           "expand")
    return phi.reshape(grid.n_patches, grid.n_r, grid.n_theta, grid.n_phi)


def phi_points(grid, lmax, M, p, i, c):
    g = _G(grid)
    M = _f64(M)
    p, i, c = _i32(p), _i32(i), _i32(c)
    out = np.zeros(len(p))
    _check(lib().orc_phi_points(g.ref, lmax, _dp(M), len(p), _ip(p), _ip(i), _ip(c), _dp(out)), "phi_points")
    return out


def brute_phi(grid, lmax, w, rho, p, i, c, nq=12):
    g = _G(grid)
    rho = _f64(rho)
    wv = None if w is None else _f64(w)
    g.set_w_stride(wv, grid.n_theta * grid.n_phi)
    p, i, c = _i32(p), _i32(i), _i32(c)
    out = np.zeros(len(p))
    _check(lib().orc_brute_phi(g.ref, lmax, _dp(wv), _dp(rho), nq, len(p), _ip(p), _ip(i), _ip(c), _dp(out)),
           "brute_phi")
    return out


def ellipsoid_phi(a, b, c, rho0, G, X, Y, Z):
    return lib().orc_ellipsoid_phi(a, b, c, rho0, G, X, Y, Z)


def potential(grid, lmax, rho, w=None, parallel=0):
    """Whole discretised solve: tables, moments, radial sums, expansion.
    Returns (phi, B, M, U, Q)."""
    if parallel:
        U, Q = tables_parallel(grid, lmax, w, workers=parallel)
    else:
        U, Q = tables(grid, lmax, w)
    B = moments(grid, lmax, U, rho)
    M = radial(grid, lmax, B)
    phi = expand(grid, lmax, Q, M)
    return phi, B, M, U, Q
