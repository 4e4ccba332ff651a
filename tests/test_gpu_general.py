"""The general multi-patch path (no parity fold): any number of patches at
any Euler angles, with tables of every patch and the patch sum of Eq. B_CS
inside the contraction (Sec. 3, Sec. 4.3).  Parity against the oracle in
FP64 and split-BF16, per-patch overlap weights, and mixing with folded plans
in one batch."""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "split_bf16": 1e-6, "split_bf16_tiered": 1e-6}


def euler_of(R):
    """Euler angles (alpha, beta, gamma) of a rotation x = R xi in the
    convention of Eq. rottransmatrix (sin beta != 0)."""
    R = np.asarray(R).reshape(9)
    beta = np.arccos(np.clip(R[8], -1.0, 1.0))
    return np.arctan2(R[7], R[6]), beta, np.arctan2(R[5], -R[2])


def yy_rotated():
    """The Yin-Yang grid turned as a whole by a fixed rotation: the two
    frames no longer differ by pi about z, so the fold does not apply, but
    the closed-form overlap weights (which depend on the relative frames
    only) still do."""
    g = W.yinyang(8, W.geometric_edges(14, 1.2), 9, name="yy_rot")
    X = O.rotation(0.7, 1.1, -0.4)
    eul = [euler_of(X @ O.rotation(*e)) for e in g.euler]
    g = W.patches(eul, g.n_theta, g.n_phi, g.theta0, g.phi0, g.dtheta, g.dphi, g.r_edges, g.lmax, name="yy_rot")
    return g, O.overlap_weights(W.yinyang(8, W.geometric_edges(14, 1.2), 9)), None


def three_patches():
    """Three patches at seeded Euler angles with their own overlap weights;
    108 cells per patch, so every patch block of K ends in padding."""
    rng = np.random.Generator(np.random.PCG64(2024))
    eul = rng.uniform(0.2, 2.9, size=(3, 3))
    d = (np.pi / 2) / 6
    g = W.patches(eul, 6, 18, np.pi / 4, -3 * np.pi / 4, d, d, W.uniform_edges(11), 8, name="three")
    w = rng.uniform(0.3, 1.0, size=(3, g.n_ang))
    return g, w, w


def two_free():
    """Two patches at unrelated Euler angles, one set of weights, 300 cells
    per patch (three angular tiles)."""
    rng = np.random.Generator(np.random.PCG64(77))
    d = (np.pi / 2) / 10
    g = W.patches([[0.3, 1.2, 2.0], [2.2, 0.5, -1.0]], 10, 30, np.pi / 4, -3 * np.pi / 4, d, d,
                  W.geometric_edges(19, 1.15), 12, name="two_free")
    w = rng.uniform(0.5, 1.0, size=g.n_ang)
    return g, w, w


def yy_rotated_high_degree():
    """The turned Yin-Yang grid at lmax 30: the tiered split form takes
    three products on the degrees above its six-product tier."""
    base = W.yinyang(16, W.geometric_edges(6, 1.3), 30)
    X = O.rotation(-0.3, 2.0, 0.8)
    eul = [euler_of(X @ O.rotation(*e)) for e in base.euler]
    g = W.patches(eul, base.n_theta, base.n_phi, base.theta0, base.phi0, base.dtheta, base.dphi, base.r_edges,
                  base.lmax, name="yy_rot_hi")
    return g, O.overlap_weights(base), None


def polar_turned():
    g = W.polar(8, 16, W.uniform_edges(9), 7, euler=(0.4, 0.9, -1.3), name="polar_turned")
    return g, None, None


CASES = {"yy_rot": yy_rotated, "three": three_patches, "two_free": two_free, "polar_turned": polar_turned,
         "yy_rot_hi": yy_rotated_high_degree}


@functools.lru_cache(maxsize=8)
def case(key):
    g, w_oracle, w_plan = CASES[key]()
    rho = W.random_rho(g, 4321)
    phi, B, M, U, Q = O.potential(g, g.lmax, rho, w_oracle)
    return g, w_plan, rho, phi, B


@pytest.mark.parametrize("precision", ["fp64", "split_bf16", "split_bf16_tiered"])
@pytest.mark.parametrize("key", list(CASES))
def test_general_path_matches_oracle(key, precision):
    import torch
    import paper_1903_08475_amd as mpg
    g, w, rho, phi_ref, _ = case(key)
    plan = mpg.Plan(g, precision=precision, overlap_w=w)
    out = plan.potential(torch.tensor(rho, device="cuda")).cpu().numpy()
    err = rel_err(out, phi_ref)
    print(f"{key} {precision}: vs oracle {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("key", ["three", "yy_rot"])
def test_general_moments_and_tables(key):
    import torch
    import paper_1903_08475_amd as mpg
    g, w, rho, _, B_ref = case(key)
    plan = mpg.Plan(g, overlap_w=w)
    B, _ = plan.moments(torch.tensor(rho, device="cuda"))
    assert rel_err(B.cpu().numpy()[0], B_ref) < 1e-12
    U, Q, wg = (t.cpu().numpy() for t in plan.tables())
    w_ref = np.broadcast_to(CASES[key]()[1], wg.shape)
    assert np.abs(wg - w_ref).max() < 1e-13
    Uo, Qo = O.tables(g, g.lmax, CASES[key]()[1])
    assert rel_err(U, Uo) < 1e-13 and rel_err(Q, Qo) < 1e-13


def test_identical_per_patch_weights_keep_the_fold():
    """Per-patch weights that are equal on Yin and Yang leave the plan on
    the folded path: the result is the shared-weight result bit for bit."""
    import torch
    import paper_1903_08475_amd as mpg
    g = W.config1()
    w = O.overlap_weights(g)
    rho = torch.tensor(W.random_rho(g, 11), device="cuda")
    a = mpg.Plan(g, overlap_w=w).potential(rho)
    b = mpg.Plan(g, overlap_w=np.stack([w, w])).potential(rho)
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "split_bf16", "split_bf16_tiered"])
def test_batch_mixes_general_and_folded_plans(precision):
    import torch
    import paper_1903_08475_amd as mpg
    items = [case("three"), case("two_free")]
    gs = [it[0] for it in items] + [W.config1()]
    ws = [it[1] for it in items] + [None]
    rhos_np = [it[2] for it in items] + [W.random_rho(gs[-1], 5)]
    plans = [mpg.Plan(g, precision=precision, overlap_w=w) for g, w in zip(gs, ws)]
    rhos = [torch.tensor(r, device="cuda") for r in rhos_np]
    outs = [torch.full_like(r, float("nan")) for r in rhos]
    for _ in range(2):
        mpg.potential_batch(plans, rhos, outs)
        singles = [p.potential(r) for p, r in zip(plans, rhos)]
        torch.cuda.synchronize()
        for o, s_ in zip(outs, singles):
            assert rel_err(o.cpu().numpy(), s_.cpu().numpy()) < TOL[precision]
    for it, o in zip(items, outs):
        assert rel_err(o.cpu().numpy(), it[3]) < TOL[precision]
