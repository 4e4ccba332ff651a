"""Batched solve of uneven fields (persistent work-queue kernels replayed
from a hipGraph) against single-plan solves and the oracle, and the
autotuner's choices against parity."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import oracle_tables, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "split_bf16": 1e-6, "split_bf16_tiered": 1e-6}


def fields():
    return [
        W.yinyang(6, W.geometric_edges(37, 1.08), 11, name="b0"),
        W.yinyang(8, W.uniform_edges(20), 16, name="b1"),
        W.polar(10, 20, W.uniform_edges(13), 9, name="b2"),
        W.yinyang(16, W.uniform_edges(150), 23, name="b3"),
        W.yinyang(4, W.uniform_edges(5), 3, name="b4"),
        W.yinyang(12, W.geometric_edges(70, 1.05), 30, name="b5"),
    ]


def oracle_phi(g, rho):
    w = O.overlap_weights(g) if g.n_patches == 2 else None
    phi, *_ = O.potential(g, g.lmax, rho, w)
    return phi


@pytest.mark.parametrize("precision", ["fp64", "split_bf16", "split_bf16_tiered"])
def test_batch_matches_oracle_over_replays(precision):
    import torch
    import paper_1903_08475_amd as mpg
    gs = fields()
    plans = [mpg.Plan(g, precision=precision) for g in gs]
    for rep in range(3):
        rhos_np = [W.random_rho(g, 5000 + 10 * rep + k) for k, g in enumerate(gs)]
        rhos = [torch.tensor(r, device="cuda") for r in rhos_np]
        phis = [torch.full_like(r, float("nan")) for r in rhos]
        mpg.potential_batch(plans, rhos, phis)
        # eager work on the same stream between replays
        singles = [p.potential(r) for p, r in zip(plans, rhos)]
        torch.cuda.synchronize()
        for k, g in enumerate(gs):
            got = phis[k].cpu().numpy()
            assert np.isfinite(got).all()
            ref = oracle_phi(g, rhos_np[k])
            assert rel_err(got, ref) < TOL[precision], (rep, g.name, rel_err(got, ref))
            assert rel_err(got, singles[k].cpu().numpy()) < TOL[precision]


def test_batch_float32_and_reuse_of_graph():
    import torch
    import paper_1903_08475_amd as mpg
    gs = fields()[:3]
    plans = [mpg.Plan(g, precision="split_bf16") for g in gs]
    rhos = [torch.tensor(W.random_rho(g, 7000 + k).astype(np.float32), device="cuda") for k, g in enumerate(gs)]
    a = [torch.empty_like(r) for r in rhos]
    b = [torch.empty_like(r) for r in rhos]
    mpg.potential_batch(plans, rhos, a)
    mpg.potential_batch(plans, rhos, b)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    for k, g in enumerate(gs):
        ref = oracle_phi(g, rhos[k].double().cpu().numpy())
        assert rel_err(a[k].cpu().numpy(), ref) < 1e-6


@pytest.mark.parametrize("precision", ["split_bf16_tiered", "fp64"])
def test_batch_field_completion_times(precision):
    """Per-field completion times inside one batched solve: positive, no
    later than the batch's end seen by events on its stream, and the last
    one close to it; unknown plan lists are rejected."""
    import torch
    import paper_1903_08475_amd as mpg
    gs = fields()
    plans = [mpg.Plan(g, precision=precision) for g in gs]
    dt = torch.float64 if precision == "fp64" else torch.float32
    rhos = [torch.tensor(W.random_rho(g, 8100 + k), dtype=dt, device="cuda") for k, g in enumerate(gs)]
    outs = [torch.empty_like(r) for r in rhos]
    for _ in range(3):  # builds the graph, then warm replays
        mpg.potential_batch(plans, rhos, outs)
    stream = plans[0].stream
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    mpg.potential_batch(plans, rhos, outs)
    b.record(stream)
    ms = mpg.batch_field_times(plans, dt)
    total = a.elapsed_time(b)
    print(f"{precision}: field completion ms {np.round(ms, 3).tolist()}, batch {total:.3f} ms")
    assert (ms > 0).all() and ms.max() <= total * 1.05 + 0.05
    # the events also cover the argument upload and the graph launch, which
    # dominate a batch this small (0.1-0.2 ms of a 0.25 ms call)
    assert ms.max() >= 0.3 * total
    with pytest.raises(mpg.MpgError):
        mpg.batch_field_times(plans[:2], dt)


def test_batch_rejects_duplicate_plans_and_mixed_precision():
    import torch
    import paper_1903_08475_amd as mpg
    g = W.config1()
    p = mpg.Plan(g)
    q = mpg.Plan(g, precision="split_bf16")
    r = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(mpg.MpgError):
        mpg.potential_batch([p, p], [r, r], [r.clone(), r.clone()])
    with pytest.raises(mpg.MpgError):
        mpg.potential_batch([p, q], [r, r], [r.clone(), r.clone()])


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_autotune_keeps_parity(precision):
    import torch
    import paper_1903_08475_amd as mpg
    g, w, U, Q = oracle_tables("medium")
    rho = W.random_rho(g, 31)
    t = torch.tensor(rho, device="cuda")
    plan = mpg.Plan(g, precision=precision)
    sk, ch, g1, rows = plan.autotune(t)
    assert sk >= 1 and ch in (4, 8, 12, 16) and g1 in (1, 2) and rows in (1, 2)
    M = O.radial(g, g.lmax, O.moments(g, g.lmax, U, rho))
    phi = O.expand(g, g.lmax, Q, M)
    out = plan.potential(t).cpu().numpy()
    print(f"{precision}: autotuned splitk {sk}, scan chunks {ch}, moment rows {g1}, expansion rows {rows}, "
          f"err {rel_err(out, phi):.3e}")
    assert rel_err(out, phi) < TOL[precision]


def test_autotune_cache_file(tmp_path):
    """Choices stored in a cache file are applied to a new plan of the same
    grid without timing, and the solve equals the first plan's bit for bit."""
    import json
    import torch
    import paper_1903_08475_amd as mpg
    g, w, U, Q = oracle_tables("medium")
    t = torch.tensor(W.random_rho(g, 33), device="cuda").float()
    cache = str(tmp_path / "tuning.json")
    p1 = mpg.Plan(g, precision="split_bf16_tiered")
    first = p1.autotune(t, cache=cache)
    table = json.load(open(cache))
    assert table == {p1.tuning_key(1, "float32"): list(first)}
    p2 = mpg.Plan(g, precision="split_bf16_tiered")
    assert p2.autotune(t, cache=cache) == first
    assert np.array_equal(p1.potential(t).cpu().numpy(), p2.potential(t).cpu().numpy())


@pytest.mark.parametrize("precision", ["split_bf16_tiered", "split_bf16"])
def test_batch_matches_single_solves_over_replays(precision):
    """The fused batch kernel runs the single-plan kernels' tiles per item
    (its K splits may differ): every field matches a single solve of its
    plan to the split tolerance, over replays with new inputs."""
    import torch
    import paper_1903_08475_amd as mpg
    gs = fields()
    plans = [mpg.Plan(g, precision=precision) for g in gs]
    singles = [mpg.Plan(g, precision=precision) for g in gs]
    for rep in range(2):
        rhos = [torch.tensor(W.random_rho(g, 7000 + 10 * rep + k), dtype=torch.float32, device="cuda")
                for k, g in enumerate(gs)]
        outs = [torch.full_like(r, float("nan")) for r in rhos]
        mpg.potential_batch(plans, rhos, outs)
        for k, (s, r, o) in enumerate(zip(singles, rhos, outs)):
            ref = s.potential(r)
            e = rel_err(o.cpu().numpy(), ref.cpu().numpy())
            print(f"{precision} rep {rep} field {k}: batch vs single {e:.3e}")
            assert e < TOL[precision]


# per field of fields(): scan chunks, moment and expansion block shapes
CHOICES = [(4, 2, 1), (8, 1, 2), (12, 2, 2), (16, 1, 1), (3, 2, 1), (1, 1, 2)]


@pytest.mark.parametrize("precision", ["split_bf16_tiered", "split_bf16", "fp64"])
def test_batch_takes_each_plans_choices(precision):
    """Each field of a batch runs with its own plan's scan chunks and block
    shapes (set here, different for every field); batch_choices reports
    them with the batch's K split, and a single solve with exactly those
    choices gives the batched field bit for bit, over two replays."""
    import torch
    import paper_1903_08475_amd as mpg
    gs = fields()
    dt = torch.float64 if precision == "fp64" else torch.float32
    plans = [mpg.Plan(g, precision=precision) for g in gs]
    for p, (ch, g1, g2) in zip(plans, CHOICES):
        p.set_tuning(chunks=ch, gemm1_rows=g1, gemm2_rows=g2)
    choices = mpg.batch_choices(plans, dt)
    for g, (sk, ch, g1, g2), (ch0, g10, g20) in zip(gs, choices, CHOICES):
        assert sk >= 1 and ch == min(ch0, g.n_r)
        assert (g1, g2) == ((g10, 1) if precision == "fp64" else (g10, g20))
    singles = [mpg.Plan(g, precision=precision) for g in gs]
    for s, c in zip(singles, choices):
        s.set_tuning(*c)
    print(f"{precision}: batch choices {choices}")
    for rep in range(2):
        rhos = [torch.tensor(W.random_rho(g, 7300 + 10 * rep + k), dtype=dt, device="cuda")
                for k, g in enumerate(gs)]
        outs = [torch.full_like(r, float("nan")) for r in rhos]
        mpg.potential_batch(plans, rhos, outs)
        for k, (s, r, o) in enumerate(zip(singles, rhos, outs)):
            ref = s.potential(r)
            diff = (o - ref).abs().max().item()
            assert torch.equal(o, ref), (rep, k, diff)


def test_batch_wait_give_up_path_exits(monkeypatch):
    """A batch built with a wait limit of one poll: the persistent kernel
    still exits (blocks whose producers are not done give up and every block
    drains); the give-up, if one happened, is reported, and a batch built
    afterwards with the default limit solves correctly."""
    import torch
    import paper_1903_08475_amd as mpg
    gs = fields()
    rhos = [torch.tensor(W.random_rho(g, 7100 + k), dtype=torch.float32, device="cuda") for k, g in enumerate(gs)]
    monkeypatch.setenv("MPG_BATCH_SPIN_LIMIT", "1")
    plans = [mpg.Plan(g, precision="split_bf16_tiered") for g in gs]
    outs = [torch.zeros_like(r) for r in rhos]
    mpg.potential_batch(plans, rhos, outs)
    torch.cuda.synchronize()
    try:
        mpg.batch_field_times(plans, torch.float32)
        gave_up = False
    except mpg.MpgError as err:
        assert "gave up" in str(err)
        gave_up = True
    print(f"wait limit 1: a wait gave up: {gave_up}")
    monkeypatch.delenv("MPG_BATCH_SPIN_LIMIT")
    plans2 = [mpg.Plan(g, precision="split_bf16_tiered") for g in gs]
    outs2 = [torch.full_like(r, float("nan")) for r in rhos]
    mpg.potential_batch(plans2, rhos, outs2)
    mpg.batch_field_times(plans2, torch.float32)
    for p, r, o in zip(plans2, rhos, outs2):
        assert rel_err(o.cpu().numpy(), p.potential(r).cpu().numpy()) < 1e-6
