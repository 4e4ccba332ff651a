"""Seeded synthetic grids and densities shared by the tests, the smoke check
and the benchmark.

This module only builds inputs: grid descriptions and cell-averaged density
arrays.  It holds none of the solver's arithmetic (no harmonics, weights,
rotations of harmonics or radial sums); positions of cell sub-samples are
mapped into one common Cartesian frame with a per-patch 3x3 matrix that the
caller provides (for the Yin-Yang grid: the identity for Yin and the
Yin<->Yang matrix of Eq. caryytransform for Yang).

Density layout: ``rho[n_patches][n_r][n_theta][n_phi]`` (phi fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PI = math.pi

# Eq. caryytransform: (xi,eta,zeta)_Yin = P (xi,eta,zeta)_Yang.
YY_SWAP = np.array([[-1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
# Euler angles of the Yin and Yang frames (Sec. 4.1).
EULER_YIN = (PI / 2, PI / 4, 3 * PI / 2)
EULER_YANG = (PI / 2, PI / 4, PI / 2)
# The common polar axis S of the two patches, in Yin (or Yang) coordinates.
AXIS_S = np.array([0.0, 1.0, 1.0]) / math.sqrt(2.0)


@dataclass
class Grid:
    n_patches: int
    n_r: int
    n_theta: int
    n_phi: int
    r_edges: np.ndarray
    theta0: float
    phi0: float
    dtheta: float
    dphi: float
    euler: np.ndarray  # [n_patches, 3]
    G: float = 1.0
    lmax: int = 0
    # matrices mapping each patch's local Cartesian frame to the density frame
    frames: list = field(default_factory=list)
    name: str = ""
    # where Phi is evaluated in each cell, on the shell's outer radius:
    # "vertex" (the upper vertex, Eq. gravpotmult) or "centre" (angular centre)
    eval_point: str = "vertex"

    @property
    def n_ang(self):
        return self.n_theta * self.n_phi

    @property
    def n_lm(self):
        return (self.lmax + 1) ** 2

    @property
    def n_cells(self):
        return self.n_patches * self.n_r * self.n_ang

    @property
    def shape(self):
        return (self.n_patches, self.n_r, self.n_theta, self.n_phi)


def yinyang(n_theta, r_edges, lmax, G=1.0, name="", buffer_cells=0):
    """Yin-Yang grid of Sec. 4.1 at spacing pi/(2 n_theta); each patch spans
    [pi/4, 3pi/4] x [-3pi/4, 3pi/4] (plus `buffer_cells` cells each side)."""
    d = (PI / 2) / n_theta
    b = buffer_cells
    r_edges = np.asarray(r_edges, dtype=np.float64)
    return Grid(2, len(r_edges) - 1, n_theta + 2 * b, 3 * n_theta + 2 * b, r_edges,
                PI / 4 - b * d, -3 * PI / 4 - b * d, d, d,
                np.array([EULER_YIN, EULER_YANG], dtype=np.float64), G, lmax,
                [np.eye(3), YY_SWAP.copy()], name)


def polar(n_theta, n_phi, r_edges, lmax, G=1.0, euler=(0.0, 0.0, 0.0), frame=None, name=""):
    """One patch covering the whole sphere (the grid of Sec. 2.2)."""
    r_edges = np.asarray(r_edges, dtype=np.float64)
    return Grid(1, len(r_edges) - 1, n_theta, n_phi, r_edges, 0.0, -PI, PI / n_theta, 2 * PI / n_phi,
                np.array([euler], dtype=np.float64), G, lmax,
                [np.eye(3) if frame is None else np.asarray(frame, dtype=np.float64)], name)


def patches(euler, n_theta, n_phi, theta0, phi0, dtheta, dphi, r_edges, lmax, G=1.0, name=""):
    """A general set of geometrically identical patches (Sec. 3), one row of
    Euler angles per patch.  No density frames are attached: such grids take
    plain seeded cell values (random_rho)."""
    euler = np.asarray(euler, dtype=np.float64).reshape(-1, 3)
    r_edges = np.asarray(r_edges, dtype=np.float64)
    return Grid(len(euler), len(r_edges) - 1, n_theta, n_phi, r_edges, theta0, phi0, dtheta, dphi, euler, G, lmax,
                [], name)


def uniform_edges(n_r, r_max=1.0):
    return np.linspace(0.0, r_max, n_r + 1)


def geometric_edges(n_r, q):
    """r_0 = 0, r_i = q^(i - n_r): ratio-q spacing normalised to R_max = 1."""
    e = np.zeros(n_r + 1)
    e[1:] = q ** (np.arange(1, n_r + 1) - n_r)
    return e


def log_edges(n_r, decades):
    """r_0 = 0, r_i = 10^(-decades (n_r - i)/(n_r - 1))."""
    e = np.zeros(n_r + 1)
    e[1:] = 10.0 ** (-decades * (n_r - np.arange(1, n_r + 1)) / (n_r - 1))
    return e


# ---------------------------------------------------------------------------
# densities, evaluated in the density frame (Yin frame for Yin-Yang grids)

@dataclass
class Ellipsoid:
    a: float = 0.5
    b: float = 0.4
    c: float = 0.3
    rho0: float = 1.0
    tilt: float = PI / 8          # about zeta_Yin (Sec. 5.1)
    spin: float = 0.0             # extra rotation of the body about AXIS_S

    def to_body(self, x, y, z, xp):
        if self.spin != 0.0:
            # rotate the evaluation point by -spin about AXIS_S (Rodrigues)
            k = AXIS_S
            c, s = math.cos(-self.spin), math.sin(-self.spin)
            kd = k[0] * x + k[1] * y + k[2] * z
            cx = k[1] * z - k[2] * y
            cy = k[2] * x - k[0] * z
            cz = k[0] * y - k[1] * x
            x, y, z = (x * c + cx * s + k[0] * kd * (1 - c),
                       y * c + cy * s + k[1] * kd * (1 - c),
                       z * c + cz * s + k[2] * kd * (1 - c))
        ct, st = math.cos(self.tilt), math.sin(self.tilt)
        X = x * ct - y * st
        Y = x * st + y * ct
        return X, Y, z

    def __call__(self, x, y, z, xp):
        X, Y, Z = self.to_body(x, y, z, xp)
        inside = (X / self.a) ** 2 + (Y / self.b) ** 2 + (Z / self.c) ** 2 <= 1.0
        return inside.to(x.dtype) * self.rho0 if xp == "torch" else inside.astype(x.dtype) * self.rho0


@dataclass
class Blobs:
    centres: np.ndarray  # [n,3]
    sigma: np.ndarray
    amp: np.ndarray

    def __call__(self, x, y, z, xp):
        if xp == "torch":
            # all blobs at once, in groups that bound the temporary size
            import torch
            c = torch.tensor(np.asarray(self.centres), dtype=x.dtype, device=x.device)
            inv = torch.tensor(-0.5 / np.asarray(self.sigma) ** 2, dtype=x.dtype, device=x.device)
            amp = torch.tensor(np.asarray(self.amp), dtype=x.dtype, device=x.device)
            xs, ys, zs = x.reshape(-1, 1), y.reshape(-1, 1), z.reshape(-1, 1)
            out = torch.zeros(xs.shape[0], dtype=x.dtype, device=x.device)
            step = 16
            for b0 in range(0, c.shape[0], step):
                b1 = min(c.shape[0], b0 + step)
                d2 = (xs - c[b0:b1, 0]) ** 2 + (ys - c[b0:b1, 1]) ** 2 + (zs - c[b0:b1, 2]) ** 2
                out += (amp[b0:b1] * torch.exp(d2 * inv[b0:b1])).sum(dim=1)
            return out.reshape(x.shape)
        out = 0.0 * x
        for (cx, cy, cz), s, a in zip(self.centres, self.sigma, self.amp):
            d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
            out = out + a * np.exp(-d2 / (2 * s * s))
        return out


def random_directions(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_blobs(rng, n, r_lo=0.1, r_hi=0.8, s_lo=0.02, s_hi=0.1, a_lo=0.1, a_hi=2.0, r_shift=0.0):
    d = random_directions(rng, n)
    r = rng.uniform(r_lo, r_hi, size=n) + r_shift
    return Blobs(d * r[:, None], rng.uniform(s_lo, s_hi, size=n), rng.uniform(a_lo, a_hi, size=n))


class Sum:
    def __init__(self, *parts):
        self.parts = parts

    def __call__(self, x, y, z, xp):
        out = None
        for p in self.parts:
            v = p(x, y, z, xp)
            out = v if out is None else out + v
        return out


def cell_average(grid: Grid, density, sub=4, device="cpu", shells_per_chunk=None, as_tensor=False,
                 out_dtype=None):
    """Volume-weighted (r^2 sin theta) midpoint average of `density` over each
    cell with sub^3 sub-samples, computed with torch on `device`.  Returns a
    float64 numpy array of grid.shape, or (as_tensor) a tensor on `device`
    of out_dtype (default float64)."""
    import torch

    dev = torch.device(device)
    f64 = torch.float64
    if as_tensor:
        out = torch.empty(grid.shape, dtype=out_dtype or f64, device=dev)
    else:
        out = np.zeros(grid.shape, dtype=np.float64)
    s = (torch.arange(sub, dtype=f64, device=dev) + 0.5) / sub
    th = grid.theta0 + (torch.arange(grid.n_theta, dtype=f64, device=dev)[:, None] + s[None, :]) * grid.dtheta
    ph = grid.phi0 + (torch.arange(grid.n_phi, dtype=f64, device=dev)[:, None] + s[None, :]) * grid.dphi
    # [nt, sub] and [np, sub] -> directions [nt, sub, np, sub]
    st, ct = torch.sin(th), torch.cos(th)
    sp, cp = torch.sin(ph), torch.cos(ph)
    ux = st[:, :, None, None] * cp[None, None, :, :]
    uy = st[:, :, None, None] * sp[None, None, :, :]
    uz = ct[:, :, None, None].expand_as(ux)
    wang = st[:, :, None, None].expand_as(ux)
    if shells_per_chunk is None:
        per_shell = grid.n_ang * sub ** 3
        budget = 8e6 if dev.type == "cuda" else 4e6
        shells_per_chunk = max(1, int(budget // per_shell))
    r_edges = torch.tensor(grid.r_edges, dtype=f64, device=dev)
    for g in range(grid.n_patches):
        F = torch.tensor(grid.frames[g], dtype=f64, device=dev)
        vx = F[0, 0] * ux + F[0, 1] * uy + F[0, 2] * uz
        vy = F[1, 0] * ux + F[1, 1] * uy + F[1, 2] * uz
        vz = F[2, 0] * ux + F[2, 1] * uy + F[2, 2] * uz
        for i0 in range(0, grid.n_r, shells_per_chunk):
            i1 = min(grid.n_r, i0 + shells_per_chunk)
            lo, hi = r_edges[i0:i1], r_edges[i0 + 1:i1 + 1]
            r = lo[:, None] + (hi - lo)[:, None] * s[None, :]          # [ns, sub]
            wr = r * r
            R = r[:, :, None, None, None, None]
            x = R * vx[None, None]
            y = R * vy[None, None]
            z = R * vz[None, None]
            val = density(x, y, z, "torch")
            wt = wr[:, :, None, None, None, None] * wang[None, None]
            num = (val * wt).sum(dim=(1, 3, 5))
            den = wt.sum(dim=(1, 3, 5))
            if as_tensor:
                out[g, i0:i1] = (num / den).to(out.dtype)
            else:
                out[g, i0:i1] = (num / den).cpu().numpy()
    return out


# ---------------------------------------------------------------------------
# the five workloads

def config1():
    """Yin-Yang at pi/32 (16x48 per patch), 32 uniform shells on (0,1],
    lmax 8, homogeneous ellipsoid (0.5,0.4,0.3), 4^3 sub-samples."""
    return yinyang(16, uniform_edges(32), 8, name="c1")


def density1():
    return Ellipsoid()


def config2():
    """Yin-Yang at pi/128 (64x192), 400 shells with ratio 1.02 normalised to
    R_max = 1 (r_0 = 0), lmax 25."""
    return yinyang(64, geometric_edges(400, 1.02), 25, name="c2")


def density2(seed=1002):
    rng = np.random.Generator(np.random.PCG64(seed))
    return Sum(Ellipsoid(), random_blobs(rng, 16))


def config3():
    """Config 1's grid at lmax 40 (split-BF16 precision case)."""
    return yinyang(16, uniform_edges(32), 40, name="c3")


def density3(seed=1003):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = Ellipsoid()
    mass = 4.0 / 3.0 * PI * e.a * e.b * e.c * e.rho0
    sigma = 0.01
    amp = mass / ((2 * PI) ** 1.5 * sigma ** 3)
    d = random_directions(rng, 1)[0]
    return Sum(e, Blobs(np.array([0.6 * d]), np.array([sigma]), np.array([amp])))


def config5():
    """Yin-Yang at pi/256 (128x384), 1200 log-spaced shells over three
    decades (r_0 = 0), lmax 48."""
    return yinyang(128, log_edges(1200, 3.0), 48, name="c5")


def density5(t, seed=1005):
    """Snapshot t of the evolving field: ellipsoid spun by 0.05 t rad about
    the common polar axis plus 64 blobs drifting outward by 0.01 t."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return Sum(Ellipsoid(spin=0.05 * t), random_blobs(rng, 64, r_shift=0.01 * t))


def config4_fields(n=64, base_seed=4000):
    """The 64 uneven fields of the batching workload: (grid, density)."""
    out = []
    for f in range(n):
        rng = np.random.Generator(np.random.PCG64(base_seed + f))
        n_r = int(rng.integers(100, 801))
        n_theta = int(rng.choice([32, 64, 128]))      # Delta = pi/64, pi/128, pi/256
        lmax = int(rng.integers(12, 33))
        ax = rng.uniform(0.2, 0.7, size=3)
        nb = int(rng.integers(4, 33))
        grid = yinyang(n_theta, uniform_edges(n_r), lmax, name=f"c4f{f}")
        dens = Sum(Ellipsoid(a=ax[0], b=ax[1], c=ax[2]), random_blobs(rng, nb))
        out.append((grid, dens))
    return out


def random_rho(grid: Grid, seed, positive=True):
    """Plain seeded random cell values (for parity tests that need no
    physical structure)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.uniform(0.0, 1.0, size=grid.shape) if positive else rng.normal(size=grid.shape)
    return v
