"""Phi evaluated at the cells' angular centres (on the outer radius of each
shell) instead of their upper vertices: the GPU paths against the oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import GRIDS, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "split_bf16": 1e-6, "split_bf16_tiered": 1e-6}


@pytest.mark.parametrize("method", ["global", "per_patch"])
@pytest.mark.parametrize("precision", ["fp64", "split_bf16_tiered"])
@pytest.mark.parametrize("key", ["c1", "ragged", "polar"])
def test_centre_evaluation_matches_oracle(key, precision, method):
    import torch
    import paper_1903_08475_amd as mpg
    g = GRIDS[key]()
    g.eval_point = "centre"
    w = O.overlap_weights(g) if g.n_patches == 2 else None
    U, Q = O.tables(g, g.lmax, w)
    rho = W.random_rho(g, 61)
    if precision != "fp64":
        rho = rho.astype(np.float32).astype(np.float64)
    phi = O.expand(g, g.lmax, Q, O.radial(g, g.lmax, O.moments(g, g.lmax, U, rho)))
    t = torch.tensor(rho, device="cuda")
    if precision != "fp64":
        t = t.float()
    out = mpg.Plan(g, precision=precision, method=method).potential(t).cpu().numpy()
    err = rel_err(out, phi)
    gv = GRIDS[key]()
    vert = mpg.Plan(gv, precision=precision, method=method).potential(t).cpu().numpy()
    print(f"{key} {precision} {method}: centre vs oracle {err:.3e}; vertex differs by {rel_err(vert, phi):.3e}")
    assert err < TOL[precision]
    assert rel_err(vert, phi) > 100 * TOL[precision]  # the two point sets differ
