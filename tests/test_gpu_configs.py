"""The two workloads that are parity cases rather than benchmark lines, at
their full sizes: the FP64 GPU workload (Yin-Yang pi/128, 400 shells of
ratio 1.02, lmax 25, ellipsoid + 16 blobs, float64 density) and the 64-field
uneven batch.  Outputs are checked at vertices the oracle computes one by
one; its moments cover every shell, since every radius needs them all."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = {"fp64": 1e-12, "split_bf16": 1e-6, "split_bf16_tiered": 1e-6}


def sample_points(g, seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.integers(0, g.n_patches, n)
    i = np.concatenate([[0, g.n_r - 1], rng.integers(0, g.n_r, n - 2)])
    c = rng.integers(0, g.n_theta * g.n_phi, n)
    return p, i, c


def oracle_at(g, rho, p, i, c):
    """The oracle's potential at vertices (p, i, c) of a full density."""
    w = O.overlap_weights(g) if g.n_patches == 2 else None
    U, _ = O.tables_parallel(g, g.lmax, w, workers=16, want_Q=False)
    B = O.moments(g, g.lmax, U, rho)
    M = O.radial(g, g.lmax, B, shells=sorted(set(i.tolist())))
    return O.phi_points(g, g.lmax, M, p, i, c)


def test_fp64_workload_at_sampled_vertices():
    import torch
    import paper_1903_08475_amd as mpg
    g = W.config2()
    rho = W.cell_average(g, W.density2(), sub=4, device="cuda")
    p, i, c = sample_points(g, 2002, 64)
    ref = oracle_at(g, rho, p, i, c)
    t = torch.tensor(rho, device="cuda")
    for precision in ("fp64", "split_bf16_tiered"):
        out = mpg.Plan(g, precision=precision).potential(t).cpu().numpy().reshape(g.n_patches, g.n_r, -1)
        err = rel_err(out[p, i, c], ref)
        print(f"c2 {precision}: max rel err at sampled vertices {err:.3e}")
        assert err < TOL[precision]


def test_batching_workload_against_single_solves_and_oracle():
    """All 64 fields in one batched call per precision: every field equals its
    single-plan solve, and three fields (the smallest) match the oracle at
    sampled vertices."""
    import torch
    import paper_1903_08475_amd as mpg
    fields = W.config4_fields()
    rhos = [W.cell_average(g, d, sub=2, device="cuda", as_tensor=True) for g, d in fields]
    work = [g.n_cells * g.n_lm for g, _ in fields]
    small = sorted(range(len(fields)), key=lambda k: work[k])[:3]
    refs = {}
    for k in small:
        g = fields[k][0]
        p, i, c = sample_points(g, 4100 + k, 32)
        refs[k] = (p, i, c, oracle_at(g, rhos[k].cpu().numpy(), p, i, c))
    for precision, dt in (("split_bf16_tiered", torch.float32), ("fp64", torch.float64)):
        plans = [mpg.Plan(g, precision=precision) for g, _ in fields]
        r = [x.to(dt) for x in rhos]
        out = [torch.full_like(x, float("nan")) for x in r]
        mpg.potential_batch(plans, r, out)
        worst = 0.0
        for k, (pl, x, o) in enumerate(zip(plans, r, out)):
            single = pl.potential(x)
            e = rel_err(o.cpu().numpy(), single.cpu().numpy())
            worst = max(worst, e)
            assert e < TOL[precision], (k, e)
        for k, (p, i, c, ref) in refs.items():
            g = fields[k][0]
            got = out[k].cpu().numpy().reshape(g.n_patches, g.n_r, -1)[p, i, c]
            e = rel_err(got, ref)
            print(f"c4 field {k} {precision}: vs oracle {e:.3e}")
            assert e < TOL[precision]
        print(f"c4 {precision}: batch vs single solves, worst {worst:.3e}")
        del plans, out
        torch.cuda.empty_cache()
