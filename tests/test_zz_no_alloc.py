"""mpg_potential_static (the solve without allocation: a static device work
space instead of the plan's) against mpg_potential through the C ABI, on
two calls in a row, the second with a smaller input, and across plans whose
work arrays lay out the shared static array differently."""
import numpy as np
import pytest

import workloads as W
from gpu_util import rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "split_bf16": 1e-6, "split_bf16_tiered": 1e-6}


def fields(g, seeds, dtype):
    import torch
    return torch.tensor(np.stack([W.random_rho(g, s) for s in seeds]), device="cuda").to(dtype)


@pytest.mark.parametrize("precision", ["fp64", "split_bf16_tiered", "split_bf16"])
def test_static_equals_potential_two_calls(precision):
    import torch
    import paper_1903_08475_amd as mpg
    dt = torch.float64 if precision == "fp64" else torch.float32
    g = W.yinyang(6, W.geometric_edges(37, 1.08), 11, name="ragged")
    plan = mpg.Plan(g, precision=precision, max_fields=3)
    for k, rho in enumerate((fields(g, (11, 12, 13), dt), fields(g, (14,), dt))):
        ref = plan.potential(rho)
        out = torch.full_like(rho, float("nan"))
        plan.potential_static(rho, out)
        torch.cuda.synchronize()
        e = rel_err(out.cpu().numpy(), ref.cpu().numpy())
        same = bool(torch.equal(out, ref))
        print(f"{precision} call {k} ({rho.shape[0]} fields): static vs plan work space {e:.3e}, identical {same}")
        assert e <= TOL[precision]


def test_static_across_plans_and_sizes():
    """A large call of one plan leaves the static array full of its data; a
    smaller plan (other layout), then the first plan again with fewer fields,
    each match mpg_potential."""
    import torch
    import paper_1903_08475_amd as mpg
    big = W.yinyang(16, W.uniform_edges(64), 20, name="big")
    small = W.polar(10, 20, W.uniform_edges(13), 9, name="polar")
    pb = mpg.Plan(big, precision="split_bf16_tiered", max_fields=4)
    ps = mpg.Plan(small, precision="split_bf16_tiered", max_fields=2)
    for plan, g, seeds in ((pb, big, (1, 2, 3, 4)), (ps, small, (5, 6)), (pb, big, (7,)), (ps, small, (8,))):
        rho = fields(g, seeds, torch.float32)
        ref = plan.potential(rho)
        out = torch.full_like(rho, float("nan"))
        plan.potential_static(rho, out)
        torch.cuda.synchronize()
        e = rel_err(out.cpu().numpy(), ref.cpu().numpy())
        print(f"{g.name} {len(seeds)} fields: static vs plan work space {e:.3e}")
        assert e <= 1e-6


def test_static_refuses_a_call_beyond_its_work_space():
    """The FP64 workload's grid (pi/128, 400 shells, lmax 25) fits the static
    work space in FP64; its split form (bf16 pieces of the input) does not
    and is refused with the size it needs, leaving the output untouched."""
    import torch
    import paper_1903_08475_amd as mpg
    g = W.config2()
    rho = fields(g, (21,), torch.float64)
    p64 = mpg.Plan(g, precision="fp64")
    ref = p64.potential(rho)
    out = torch.zeros_like(rho)
    p64.potential_static(rho, out)
    torch.cuda.synchronize()
    assert rel_err(out.cpu().numpy(), ref.cpu().numpy()) <= 1e-12
    ps = mpg.Plan(g, precision="split_bf16_tiered")
    r32 = rho.float()
    out32 = torch.zeros_like(r32)
    with pytest.raises(mpg.MpgError, match="MiB static work space"):
        ps.potential_static(r32, out32)
    assert float(out32.abs().max()) == 0.0
    # the plan still solves through its own work space afterwards
    assert rel_err(ps.potential(r32).cpu().numpy(), ref.cpu().numpy()) <= 1e-6
