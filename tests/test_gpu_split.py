"""Parity of the split-BF16 GPU path (six-product three-piece bf16 MFMA
contractions, FP32 accumulation, FP64 scans) with the CPU oracle and with
the FP64 GPU path.  Bar: 1e-6 max-norm relative error of Phi."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import oracle_tables, rel_err

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-6


def torch_mods():
    import torch
    import paper_1903_08475_amd as mpg
    return torch, mpg


def density(key, g):
    if key == "c3":
        return W.cell_average(g, W.density3(), sub=4)
    if key == "c1":
        return W.cell_average(g, W.density1(), sub=4)
    return W.random_rho(g, 21)


@pytest.mark.parametrize("key", ["c3", "c1", "ragged", "polar", "medium", "tiny"])
def test_split_potential_matches_oracle_and_fp64_path(key):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    rho = density(key, g)
    M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rho))
    phi = O.expand(g, g.lmax, Q, M)
    t = torch.tensor(rho, device="cuda")
    out = mpg.Plan(g, precision="split_bf16").potential(t).cpu().numpy()
    ref64 = mpg.Plan(g, precision="fp64").potential(t).cpu().numpy()
    e_orc, e_64 = rel_err(out, phi), rel_err(out, ref64)
    print(f"{key}: split-BF16 vs oracle {e_orc:.3e}, vs FP64 GPU {e_64:.3e}")
    assert e_orc < TOL_SPLIT and e_64 < TOL_SPLIT


def test_split_moments_match_oracle():
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("c3")
    rho = density("c3", g)
    B = O.moments(g, g.lmax, U, rho)
    M = O.radial(g, g.lmax, B)
    Bg, Mg = mpg.Plan(g, precision="split_bf16").moments(torch.tensor(rho, device="cuda"))
    assert rel_err(Bg[0].cpu().numpy(), B) < TOL_SPLIT
    assert rel_err(Mg[0].cpu().numpy(), M) < TOL_SPLIT


def test_split_float32_fields_batched():
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("ragged")
    rhos = np.stack([W.random_rho(g, 300 + f) for f in range(3)]).astype(np.float32)
    plan = mpg.Plan(g, precision="split_bf16", max_fields=3)
    out = plan.potential(torch.tensor(rhos, device="cuda"), out_dtype=torch.float64).cpu().numpy()
    for f in range(3):
        M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rhos[f].astype(np.float64)))
        phi = O.expand(g, g.lmax, Q, M)
        assert rel_err(out[f], phi) < TOL_SPLIT


def test_split_zero_density():
    torch, mpg = torch_mods()
    g = W.config1()
    out = mpg.Plan(g, precision="split_bf16").potential(torch.zeros(g.shape, dtype=torch.float32, device="cuda"))
    assert float(out.abs().max()) == 0.0


def test_stage_timing_counts_launches():
    torch, mpg = torch_mods()
    g = W.config1()
    plan = mpg.Plan(g, precision="split_bf16")
    plan.timing(True)
    rho = torch.ones(g.shape, dtype=torch.float64, device="cuda")
    for _ in range(3):
        plan.potential(rho)
    st = plan.stage_times()
    assert all(st[k][1] == 3 for k in st) and all(st[k][0] > 0 for k in st)
    assert all(v[1] == 0 for v in plan.stage_times().values())
