"""Parity of the split-BF16 GPU path (three-piece bf16 MFMA contractions
with six products, or three above the low-degree tier; FP32 accumulation,
FP64 scans) with the CPU oracle and with the FP64 GPU path.  Bar: 1e-6
max-norm relative error of Phi, and of the moments B and M that
mpg_moments returns in both split forms (formed with six products on every
column)."""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import oracle_tables, rel_err

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-6
TOL_MOMENTS = {"split_bf16": 1e-6, "split_bf16_tiered": 1e-6}
SPLITS = ["split_bf16", "split_bf16_tiered"]


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


@pytest.mark.parametrize("precision", SPLITS)
@pytest.mark.parametrize("key", ["c3", "c1", "ragged", "polar", "medium", "tiny"])
def test_split_potential_matches_oracle_and_fp64_path(key, precision):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    rho = density(key, g)
    M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rho))
    phi = O.expand(g, g.lmax, Q, M)
    t = torch.tensor(rho, device="cuda")
    out = mpg.Plan(g, precision=precision).potential(t).cpu().numpy()
    ref64 = mpg.Plan(g, precision="fp64").potential(t).cpu().numpy()
    e_orc, e_64 = rel_err(out, phi), rel_err(out, ref64)
    print(f"{key} {precision}: vs oracle {e_orc:.3e}, vs FP64 GPU {e_64:.3e}")
    assert e_orc < TOL_SPLIT and e_64 < TOL_SPLIT


@pytest.mark.parametrize("precision", SPLITS)
def test_split_moments_match_oracle(precision):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("c3")
    rho = density("c3", g)
    B = O.moments(g, g.lmax, U, rho)
    M = O.radial(g, g.lmax, B)
    Bg, Mg = mpg.Plan(g, precision=precision).moments(torch.tensor(rho, device="cuda"))
    eb, em = rel_err(Bg[0].cpu().numpy(), B), rel_err(Mg[0].cpu().numpy(), M)
    print(f"{precision}: B vs oracle {eb:.3e}, M vs oracle {em:.3e}")
    assert eb < TOL_MOMENTS[precision] and em < TOL_MOMENTS[precision]


def test_tiered_moments_equal_the_six_product_form():
    """mpg_moments forms the tiered plan's moments with six products on every
    column, so they equal the six-product form's bit for bit; its potential
    (three products above the tier) differs from the six-product form's."""
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("c3")
    t = torch.tensor(density("c3", g), device="cuda")
    six, tiered = mpg.Plan(g, precision="split_bf16"), mpg.Plan(g, precision="split_bf16_tiered")
    B6, M6 = six.moments(t)
    BT, MT = tiered.moments(t)
    assert torch.equal(B6, BT) and torch.equal(M6, MT)
    p6, pT = six.potential(t), tiered.potential(t)
    assert not torch.equal(p6, pT)
    assert rel_err(pT.cpu().numpy(), p6.cpu().numpy()) < TOL_SPLIT


@pytest.mark.parametrize("precision", SPLITS)
def test_split_float32_fields_batched(precision):
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("ragged")
    rhos = np.stack([W.random_rho(g, 300 + f) for f in range(3)]).astype(np.float32)
    plan = mpg.Plan(g, precision=precision, max_fields=3)
    out = plan.potential(torch.tensor(rhos, device="cuda"), out_dtype=torch.float64).cpu().numpy()
    for f in range(3):
        M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rhos[f].astype(np.float64)))
        phi = O.expand(g, g.lmax, Q, M)
        assert rel_err(out[f], phi) < TOL_SPLIT


@functools.lru_cache(maxsize=1)
def largest_degree_case():
    g = W.yinyang(16, W.geometric_edges(5, 1.3), 64, name="lmax64")
    rho = W.random_rho(g, 64)
    phi, *_ = O.potential(g, g.lmax, rho, O.overlap_weights(g))
    return g, rho, phi


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("split_bf16_tiered", TOL_SPLIT)])
def test_largest_degree(precision, tol):
    """lmax 64, the largest the plan accepts (4225 moments, ragged column
    blocks), on config 1's angular grid with a few shells."""
    torch, mpg = torch_mods()
    g, rho, phi = largest_degree_case()
    out = mpg.Plan(g, precision=precision).potential(torch.tensor(rho, device="cuda")).cpu().numpy()
    err = rel_err(out, phi)
    print(f"lmax 64 {precision}: vs oracle {err:.3e}")
    assert err < tol


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


@pytest.mark.parametrize("key,method", [("c1", "global"), ("ragged", "global"), ("polar", "global"),
                                        ("medium", "global"), ("tiny", "global"), ("ragged", "per_patch")])
def test_expansion_block_shapes_agree(key, method):
    """The expansion's two block shapes (128 x 256 and 256 x 128) give the
    same potential; the shape set back gives the first result again."""
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    t = torch.tensor(density(key, g).astype(np.float32), device="cuda")
    plan = mpg.Plan(g, precision="split_bf16_tiered", method=method)
    wide = plan.potential(t).cpu().numpy()
    plan.set_tuning(gemm2_rows=2)
    tall = plan.potential(t).cpu().numpy()
    plan.set_tuning(gemm2_rows=1)
    again = plan.potential(t).cpu().numpy()
    print(f"{key} {method}: 256x128 vs 128x256 blocks, max abs diff {np.abs(tall - wide).max():.3e}")
    assert np.array_equal(wide, again)
    assert rel_err(tall, wide) <= 1e-12


@pytest.mark.parametrize("key,method", [("c1", "global"), ("ragged", "global"), ("polar", "global"),
                                        ("medium", "global"), ("tiny", "global"), ("ragged", "per_patch")])
@pytest.mark.parametrize("precision", ["split_bf16_tiered", "split_bf16"])
def test_moment_block_shapes_agree(key, method, precision):
    """The moment contraction's two block shapes (128 x 256 and 256 x 128)
    give the same moments and potential bit for bit (every output takes the
    same products in the same order), with one K split and with three (or
    two, as far as the plan's K allows)."""
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables(key)
    t = torch.tensor(density(key, g).astype(np.float32), device="cuda")
    plan = mpg.Plan(g, precision=precision, method=method)
    done_split = False
    for splitk in (1, 3, 2):
        try:
            plan.set_tuning(splitk=splitk, gemm1_rows=1)
        except mpg.MpgError:
            continue  # more splits than the plan's work space holds (small K)
        if splitk == 2 and done_split:
            break
        done_split = splitk > 1
        B1, M1 = (x.cpu().numpy() for x in plan.moments(t))
        wide = plan.potential(t).cpu().numpy()
        plan.set_tuning(gemm1_rows=2)
        B2, M2 = (x.cpu().numpy() for x in plan.moments(t))
        tall = plan.potential(t).cpu().numpy()
        print(f"{key} {method} {precision} split {splitk}: moment blocks 256x128 vs 128x256, "
              f"max abs diff B {np.abs(B2 - B1).max():.3e}, Phi {np.abs(tall - wide).max():.3e}")
        assert np.array_equal(B1, B2) and np.array_equal(M1, M2)
        assert np.array_equal(wide, tall)


def test_set_tuning_rejects_out_of_range_values():
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("tiny")
    plan = mpg.Plan(g, precision="split_bf16")
    for kw in ({"gemm1_rows": 3}, {"gemm2_rows": 3}, {"chunks": 17}, {"splitk": 10 ** 6}):
        with pytest.raises(mpg.MpgError):
            plan.set_tuning(**kw)


@pytest.mark.parametrize("precision", ["fp64", "split_bf16", "split_bf16_tiered"])
def test_solves_are_bitwise_reproducible(precision):
    """Every reduction runs in a fixed order (K splits summed in order in the
    scan, no atomics in the arithmetic), so repeated solves, with other work
    in between and with a K split of 2, give the same bits."""
    torch, mpg = torch_mods()
    g, w, U, Q = oracle_tables("medium")
    t = torch.tensor(density("medium", g), device="cuda")
    if precision != "fp64":
        t = t.float()
    plan = mpg.Plan(g, precision=precision)
    other = mpg.Plan(*oracle_tables("ragged")[:1], precision=precision)
    first = plan.potential(t).cpu().numpy()
    for splitk in (0, 2):
        if splitk:
            plan.set_tuning(splitk=splitk)
            first = plan.potential(t).cpu().numpy()
        for _ in range(2):
            other.potential(torch.rand(other.shape, device="cuda", dtype=t.dtype))
            assert np.array_equal(plan.potential(t).cpu().numpy(), first)
