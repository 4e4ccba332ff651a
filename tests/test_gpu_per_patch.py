"""The per-patch comparison method (moments of every patch in its own
frame, radial sums per patch, potentials of the patches added; Sec. 1 and
Sec. 4.3): the same discretised potential as the paper's method up to
rounding, checked against the oracle in FP64 and split-BF16, and its
per-patch moments against the oracle's moments on a patch in its own
frame."""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import rel_err
from test_gpu_general import yy_rotated, yy_rotated_high_degree

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "split_bf16": 1e-6, "split_bf16_tiered": 1e-6}


def three_shared():
    rng = np.random.Generator(np.random.PCG64(99))
    eul = rng.uniform(0.2, 2.9, size=(3, 3))
    d = (np.pi / 2) / 6
    g = W.patches(eul, 6, 18, np.pi / 4, -3 * np.pi / 4, d, d, W.uniform_edges(10), 7, name="three_shared")
    w = rng.uniform(0.4, 1.0, size=g.n_ang)
    return g, w, w


def yinyang_c1():
    g = W.config1()
    return g, O.overlap_weights(g), None


def ragged():
    g = W.yinyang(6, W.geometric_edges(37, 1.08), 11, name="ragged")
    return g, O.overlap_weights(g), None


def polar():
    g = W.polar(10, 20, W.uniform_edges(13), 9, name="polar")
    return g, None, None


CASES = {"c1": yinyang_c1, "ragged": ragged, "polar": polar, "yy_rot": yy_rotated, "three_shared": three_shared,
         "yy_rot_hi": yy_rotated_high_degree}


@functools.lru_cache(maxsize=8)
def case(key):
    g, w_oracle, w_plan = CASES[key]()
    rho = W.random_rho(g, 2468)
    phi, *_ = O.potential(g, g.lmax, rho, w_oracle)
    return g, w_oracle, w_plan, rho, phi


@pytest.mark.parametrize("precision", ["fp64", "split_bf16", "split_bf16_tiered"])
@pytest.mark.parametrize("key", list(CASES))
def test_per_patch_method_matches_oracle(key, precision):
    import torch
    import paper_1903_08475_amd as mpg
    g, _, w, rho, phi_ref = case(key)
    plan = mpg.Plan(g, precision=precision, overlap_w=w, method="per_patch")
    out = plan.potential(torch.tensor(rho, device="cuda")).cpu().numpy()
    err = rel_err(out, phi_ref)
    print(f"{key} {precision} per-patch: vs oracle {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("key", ["c1", "three_shared"])
def test_per_patch_moments_are_each_patch_in_its_own_frame(key):
    """E_g of every patch equals the oracle's moments of that patch's cells
    on a single patch with the identity frame and the same weights."""
    import torch
    import paper_1903_08475_amd as mpg
    g, w_oracle, w, rho, _ = case(key)
    plan = mpg.Plan(g, overlap_w=w, method="per_patch")
    B, _ = plan.moments(torch.tensor(rho, device="cuda"))
    B = B.cpu().numpy()[0]
    loc = W.patches([[0.0, 0.0, 0.0]], g.n_theta, g.n_phi, g.theta0, g.phi0, g.dtheta, g.dphi, g.r_edges, g.lmax)
    U, _ = O.tables(loc, g.lmax, w_oracle, want_Q=False)
    for p in range(g.n_patches):
        E = O.moments(loc, g.lmax, U, rho[p:p + 1])
        assert rel_err(B[p], E) < 1e-12, p


def test_per_patch_and_global_methods_agree_on_device():
    import torch
    import paper_1903_08475_amd as mpg
    g = W.config1()
    rho = torch.tensor(W.random_rho(g, 8), device="cuda").repeat(3, 1, 1, 1, 1).contiguous()
    rho[1] *= 0.5
    a = mpg.Plan(g, max_fields=3).potential(rho)
    b = mpg.Plan(g, max_fields=3, method="per_patch").potential(rho)
    assert rel_err(b.cpu().numpy(), a.cpu().numpy()) < 1e-13


def test_per_patch_method_limits():
    import torch
    import paper_1903_08475_amd as mpg
    g, w, _ = CASES["three_shared"]()
    with pytest.raises(mpg.MpgError):
        mpg.Plan(g, overlap_w=np.stack([w, w, 0.5 * w]), method="per_patch")
    p = mpg.Plan(g, overlap_w=np.stack([w, w, w]), method="per_patch")
    r = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(mpg.MpgError):
        mpg.potential_batch([p], [r], [r.clone()])
