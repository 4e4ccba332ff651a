"""Host-side logic of bench.py (no GPU): the count of bf16 products per
algorithmic product of the split forms, and the guard that keeps HBM
traffic figures taken on other kernel sources out of the benchmark line."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def count_products(lmax, tier, wave=64, slab=32):
    """Brute force over the real columns of each m-parity block: a moment
    column takes six products when its 64-column wave tile (moments) or its
    32-moment K slab (expansion) reaches a degree <= tier.  The expansion
    walks its slabs from the highest degree down and the leading
    (three-product) slabs come in even numbers, so one more slab at the
    tier's edge may take six."""
    res = {}
    for stage in ("moments", "expansion"):
        six = tot = 0
        for par in (0, 1):
            degs = [l for l in range(lmax + 1) for m in range(l + 1) if m % 2 == par
                    for _ in range(1 if m == 0 else 2)]
            n = len(degs)
            if stage == "moments":
                six_cols = {c for c in range(n) if any(d <= tier for d in degs[(c // wave) * wave:(c // wave + 1) * wave])}
            else:
                n_sl = -(-n // slab)
                tier_sl = {c // slab for c in range(n) if degs[c] <= tier}
                n3 = n_sl - len(tier_sl)
                n3 = n3 if n3 == n_sl else n3 - n3 % 2
                six_cols = {c for c in range(n) if c // slab < n_sl - n3}
            six += len(six_cols)
            tot += n
        res[stage] = (6 * six + 3 * (tot - six)) / tot
    return res


def test_products_per_term_matches_brute_force_count():
    for lmax in (8, 15, 16, 25, 48, 64):
        got = bench.products_per_term(lmax, "split_bf16_tiered")
        ref = count_products(lmax, 15)
        for stage in ("moments", "expansion"):
            assert abs(got[stage] - ref[stage]) < 1e-12, (lmax, stage, got, ref)
    assert bench.products_per_term(48, "split_bf16") == {"moments": 6.0, "expansion": 6.0}
    assert bench.products_per_term(15, "split_bf16_tiered") == {"moments": 6.0, "expansion": 6.0}
    assert abs(bench.products_per_term(48, "split_bf16_tiered")["moments"] - 3.32) < 0.01


def test_traffic_is_used_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = "split_bf16_tiered:moments"
    assert bench.traffic_record("moments", "split_bf16_tiered") in (None, rec[key]["bytes_per_launch"])
    fake = tmp_path / "profiles"
    fake.mkdir()
    rec[key]["source_hash"] = "0" * 16
    (fake / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda source="gemm_bf16.hip": "1" * 16)
    assert bench.traffic_record("moments", "split_bf16_tiered") is None
    # a record stamped with the current hash of its own kernel file is used
    rec[key]["source_hash"] = "1" * 16
    (fake / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_record("moments", "split_bf16_tiered") == rec[key]["bytes_per_launch"]


def test_separable_flops_count():
    """Products of the separable phi transforms on the large workload: rows
    x (2 lmax + 1) columns x 192 mirror pairs (moments) or 193 points
    (expansion: 191 mirror pairs, phi = 0 and the last vertex)."""
    import workloads as W
    g = W.config5()
    f = bench.separable_flops(g, 8)
    rows = 8 * 2 * 1200 * 128
    assert f["phi_moments"] == 2.0 * rows * 192 * 97
    assert f["phi_expansion"] == 2.0 * rows * 193 * 97
