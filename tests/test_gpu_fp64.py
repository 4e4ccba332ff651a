"""Parity of the FP64 GPU path with the CPU oracle (bar: 1e-12 max-norm
relative for FP64), element by element on seeded inputs."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import GRIDS, cell_areas, oracle_tables, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def torch_mods():
    import torch
    import paper_1903_08475_amd as mpg
    return torch, mpg


@pytest.mark.parametrize("key", ["c1", "ragged", "polar", "tiny", "medium"])
def test_tables_match_oracle(key):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    plan = mpg.Plan(g)
    Ug, Qg, wg = (t.cpu().numpy() for t in plan.tables())
    assert rel_err(Ug, U) < 1e-13, rel_err(Ug, U)
    assert rel_err(Qg, Q) < 1e-13, rel_err(Qg, Q)
    if w is not None:
        A = cell_areas(g)
        # covered area per cell, absolute
        assert np.abs((1 - wg) * A - (1 - w) * A).max() < 2e-16 * 8, np.abs((wg - w) * A).max()
    else:
        assert np.all(wg == 1.0)


def _rho(g, seed, kind="random"):
    if kind == "ellipsoid":
        return W.cell_average(g, W.Ellipsoid(), sub=2)
    return W.random_rho(g, seed)


@pytest.mark.parametrize("key", ["c1", "ragged", "polar", "tiny", "medium"])
def test_moments_match_oracle(key):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    rho = _rho(g, 11)
    B = O.moments(g, g.lmax, U, rho)
    M = O.radial(g, g.lmax, B)
    plan = mpg.Plan(g)
    Bg, Mg = plan.moments(torch.tensor(rho, device="cuda"))
    Bg, Mg = Bg[0].cpu().numpy(), Mg[0].cpu().numpy()
    assert rel_err(Bg, B) < TOL64, rel_err(Bg, B)
    assert rel_err(Mg, M) < TOL64, rel_err(Mg, M)


@pytest.mark.parametrize("key", ["c1", "ragged", "polar", "tiny", "medium"])
def test_potential_matches_oracle(key):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    rho = _rho(g, 12, "ellipsoid" if key == "c1" else "random")
    B = O.moments(g, g.lmax, U, rho)
    M = O.radial(g, g.lmax, B)
    phi = O.expand(g, g.lmax, Q, M)
    plan = mpg.Plan(g)
    out = plan.potential(torch.tensor(rho, device="cuda")).cpu().numpy()
    assert out.shape == phi.shape
    assert rel_err(out, phi) < TOL64, rel_err(out, phi)


@pytest.mark.parametrize("key", ["c1", "ragged", "polar", "tiny", "medium"])
@pytest.mark.parametrize("method", ["global", "per_patch"])
def test_moment_tile_sides_agree(key, method):
    """The FP64 moment contraction's two tile sides (128 and 64) give the
    same moments and potential bit for bit (every output takes the same
    products in the same order), with one K split and with two; the 64-tile
    result also matches the oracle."""
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    if method == "per_patch" and g.n_patches < 2:
        pytest.skip("one patch: the per-patch method is the global one")
    t = torch.tensor(_rho(g, 13), device="cuda")
    plan = mpg.Plan(g, method=method)
    for splitk in (1, 2):
        plan.set_tuning(splitk=splitk, gemm1_rows=1)
        B1, M1 = (x.cpu().numpy() for x in plan.moments(t))
        p1 = plan.potential(t).cpu().numpy()
        plan.set_tuning(gemm1_rows=2)
        B2, M2 = (x.cpu().numpy() for x in plan.moments(t))
        p2 = plan.potential(t).cpu().numpy()
        print(f"{key} {method} split {splitk}: 64 vs 128 tiles, max abs diff B {np.abs(B2 - B1).max():.3e}")
        assert np.array_equal(B1, B2) and np.array_equal(M1, M2) and np.array_equal(p1, p2)
    if method == "global":
        B = O.moments(g, g.lmax, U, t.cpu().numpy())
        assert rel_err(B2[0], B) < TOL64


def test_batched_fields_match_single_solves():
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("ragged")
    rhos = np.stack([W.random_rho(g, 100 + f) for f in range(3)])
    plan = mpg.Plan(g, max_fields=3)
    out = plan.potential(torch.tensor(rhos, device="cuda")).cpu().numpy()
    for f in range(3):
        M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rhos[f]))
        phi = O.expand(g, g.lmax, Q, M)
        assert rel_err(out[f], phi) < TOL64


def test_float32_input_and_output():
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("c1")
    rho32 = W.random_rho(g, 13).astype(np.float32)
    M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rho32.astype(np.float64)))
    phi = O.expand(g, g.lmax, Q, M)
    plan = mpg.Plan(g)
    t = torch.tensor(rho32, device="cuda")
    out64 = plan.potential(t, out_dtype=torch.float64).cpu().numpy()
    assert rel_err(out64, phi) < TOL64
    out32 = plan.potential(t).cpu().numpy()
    assert out32.dtype == np.float32
    assert rel_err(out32, phi) < 2e-7


def test_zero_density_gives_zero_potential():
    torch, mpg = torch_mods()
    g = W.config1()
    plan = mpg.Plan(g)
    out = plan.potential(torch.zeros(g.shape, dtype=torch.float64, device="cuda"))
    assert float(out.abs().max()) == 0.0


def test_linearity_and_swap_symmetry_on_device():
    torch, mpg = torch_mods()
    g = W.config1()
    plan = mpg.Plan(g)
    a = torch.tensor(W.random_rho(g, 1), device="cuda")
    b = torch.tensor(W.random_rho(g, 2), device="cuda")
    pa, pb = plan.potential(a), plan.potential(b)
    pab = plan.potential(2.0 * a - 0.5 * b)
    assert float((pab - (2.0 * pa - 0.5 * pb)).abs().max() / pab.abs().max()) < 1e-13
    ps = plan.potential(a.flip(0).contiguous())
    assert float((ps - pa.flip(0)).abs().max() / pa.abs().max()) < 1e-13


def test_bad_calls_raise():
    torch, mpg = torch_mods()
    g = W.config1()
    plan = mpg.Plan(g, max_fields=1)
    rho = torch.zeros((2,) + g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(mpg.MpgError):
        plan.potential(rho)  # two fields > max_fields
    with pytest.raises(ValueError):
        plan.potential(torch.zeros(7, dtype=torch.float64, device="cuda"))
    plan.close()  # a destroyed plan is refused, not used
    with pytest.raises(mpg.MpgError) as err:
        plan.potential(rho[:1])
    assert err.value.code == mpg.MPG_EINVAL


def test_plan_whose_work_space_does_not_fit_fails_cleanly():
    """A plan whose FP64 work space exceeds the GPU's memory (4096 fields of
    2000 shells at lmax 48: about 160 GB per work array) is refused with
    MPG_ENOMEM, frees what it had allocated, and later plans solve correctly."""
    torch, mpg = torch_mods()
    big = W.yinyang(4, W.uniform_edges(2000), 48)
    with pytest.raises(mpg.MpgError) as err:
        mpg.Plan(big, max_fields=4096)
    assert err.value.code == mpg.MPG_ENOMEM
    assert "work space" in str(err.value)
    g, w, U, Q = oracle_tables("ragged")
    rho = W.random_rho(g, 41)
    phi = O.expand(g, g.lmax, Q, O.radial(g, g.lmax, O.moments(g, g.lmax, U, rho)))
    out = mpg.Plan(g).potential(torch.tensor(rho, device="cuda")).cpu().numpy()
    assert rel_err(out, phi) < TOL64
