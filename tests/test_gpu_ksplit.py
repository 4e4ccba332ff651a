"""Coverage of the K splits of the moment contraction and of the row range
of mpg_moments, against the oracle: grids and K splits where the chunk
rule once left trailing angular cells out (Eq. B_CS sums over every
cell), and more (field, shell) rows than one grid dimension holds."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import rel_err

pytestmark = pytest.mark.gpu


def test_fp64_yinyang_pi256_default_split():
    """Yin-Yang at pi/256, lmax 12, 385 uniform shells (a grid of the batching
    workload's range): the default K split of the FP64 plan is 37, where 16
    cells used to drop out.  B and M against the oracle over every shell."""
    import torch
    import paper_1903_08475_amd as mpg
    g = W.yinyang(128, W.uniform_edges(385), 12, name="pi256_l12")
    w = O.overlap_weights(g)
    U, _ = O.tables_parallel(g, g.lmax, w, workers=16, want_Q=False)
    rho = W.random_rho(g, 385)
    B = O.moments(g, g.lmax, U, rho)
    M = O.radial(g, g.lmax, B)
    t = torch.tensor(rho, device="cuda")
    for precision, tol in (("fp64", 1e-12), ("split_bf16_tiered", 1e-6)):
        Bg, Mg = mpg.Plan(g, precision=precision).moments(t)
        eb, em = rel_err(Bg[0].cpu().numpy(), B), rel_err(Mg[0].cpu().numpy(), M)
        print(f"pi/256 lmax 12 {precision}: B {eb:.3e}, M {em:.3e}")
        assert eb < tol and em < tol


@pytest.mark.parametrize("precision,splits,tol", [("split_bf16", (53, 79), 1e-6), ("fp64", (29, 53, 79), 1e-12)])
def test_polar_5120_cells_odd_splits(precision, splits, tol):
    """A one-patch grid of 32 x 160 cells (5120, a multiple of 128): K
    splits 53 and 79 of the split form's 32-cell slabs (and 29, 53, 79 of
    the FP64 form's 16-cell slabs), each of which the old chunk rule left
    short of the last cells, cover every cell."""
    import torch
    import paper_1903_08475_amd as mpg
    g = W.polar(32, 160, W.uniform_edges(3), 4, name="polar5120")
    U, _ = O.tables(g, g.lmax, None, want_Q=False)
    rho = W.random_rho(g, 5120)
    B = O.moments(g, g.lmax, U, rho)
    t = torch.tensor(rho, device="cuda")
    plan = mpg.Plan(g, precision=precision)
    for s in splits:
        plan.set_tuning(splitk=s)
        Bg, _ = plan.moments(t)
        e = rel_err(Bg[0].cpu().numpy(), B)
        print(f"polar 5120 {precision} K split {s}: B {e:.3e}")
        assert e < tol


def test_moments_beyond_65535_rows():
    """64 fields of 1100 shells (70400 rows) on a coarse Yin-Yang grid: the
    moments of the first and the last field match the oracle."""
    import torch
    import paper_1903_08475_amd as mpg
    g = W.yinyang(4, W.uniform_edges(1100), 3, name="rows70k")
    n = 64
    w = O.overlap_weights(g)
    U, _ = O.tables(g, g.lmax, w, want_Q=False)
    rhos = np.stack([W.random_rho(g, 9000 + f) for f in (0, n - 1)])
    t = torch.empty((n,) + g.shape, dtype=torch.float64, device="cuda")
    t.uniform_(0.0, 1.0)
    t[0] = torch.tensor(rhos[0], device="cuda")
    t[n - 1] = torch.tensor(rhos[1], device="cuda")
    Bg, Mg = mpg.Plan(g, precision="fp64", max_fields=n).moments(t)
    for k, f in enumerate((0, n - 1)):
        B = O.moments(g, g.lmax, U, rhos[k])
        M = O.radial(g, g.lmax, B)
        eb, em = rel_err(Bg[f].cpu().numpy(), B), rel_err(Mg[f].cpu().numpy(), M)
        print(f"field {f} of {n} (rows {f * g.n_r}..{(f + 1) * g.n_r - 1}): B {eb:.3e}, M {em:.3e}")
        assert eb < 1e-12 and em < 1e-12
