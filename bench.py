"""Benchmark of one solve step on one MI355X.

A step is one pass of the whole hot path (moment contraction, radial scans,
expansion) over one batch of 8 snapshots of the large workload: Yin-Yang grid
at pi/256 (128x384 cells per patch), 1200 log-spaced shells, lmax 48,
float32 densities, split-BF16 contractions in the tiered form (three bf16
products per product, six on the moments of degree <= 15).  Inputs are
resident in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line (see the fields below).  The six-product split form and
the FP64 path are timed on the same workload for comparison (with the
max-norm relative difference of each split form to the FP64 result), and the
CPU oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid cells·(l,m) terms/s per solve, split-BF16 vs FP64 at ≤1e-6 rel err"
PEAK_BF16 = 2.5e15     # dense bf16 MFMA, FLOP/s
PEAK_FP64 = 78.6e12    # FP64 MFMA, FLOP/s
PEAK_HBM = 8.0e12      # HBM3E, bytes/s
HBM_PEAK = 8.0e12      # B/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash(source="gemm_bf16.hip"):
    """Hash of the sources a path's contractions are compiled from (their
    file and every header of the library's sources): gemm_bf16.hip for the
    split contractions, sep_f64.hip for the separable method's."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_08475_amd", "csrc")
    names = [source] + sorted(n for n in os.listdir(csrc) if n.endswith(".h"))
    for name in names:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(stage, precision):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    key = f"{precision}:{stage}"
    r = rec.get(key)
    source = "sep_f64.hip" if precision.startswith("separable") else "gemm_bf16.hip"
    if not r or r.get("source_hash") != kernel_source_hash(source):
        return None
    return r.get("bytes_per_launch")


TIER_LMAX = {"moments": 15, "expansion": 15}  # MPG_TIER_LMAX


def products_per_term(lmax, precision, blk=64, slab=32):
    """bf16 MFMA products per algorithmic product, averaged over the moment
    columns of the folded contractions (even and odd m blocks): six for the
    six-product form; for the tiered form six on the columns of a moment
    contraction wave tile of 64 columns (or an expansion K slab of 32) that
    reaches into the low-degree tier, else three."""
    if precision != "split_bf16_tiered":
        return {"moments": 6.0, "expansion": 6.0}
    res = {}
    for stage, gran in (("moments", blk), ("expansion", slab)):
        cols = {0: 0, 1: 0}
        tier = {0: 0, 1: 0}
        for l in range(lmax + 1):
            for m in range(l + 1):
                c = 1 if m == 0 else 2
                cols[m % 2] += c
                if l <= TIER_LMAX[stage]:
                    tier[m % 2] += c
        tot = prod = 0.0
        for par in (0, 1):
            n, t = cols[par], tier[par]
            t6 = min(n, -(-t // slab) * slab)  # tier columns rounded up to K slabs
            if stage == "moments":
                t6 = min(n, -(-t6 // gran) * gran)
            else:
                n_sl = -(-n // slab)
                n3 = max(n_sl - t6 // slab, 0)
                n3 = n3 if n3 == n_sl else n3 & ~1
                t6 = min(n, (n_sl - n3) * slab)
            tot += n
            prod += 6 * t6 + 3 * (n - t6)
        res[stage] = prod / tot
    return res


def make_inputs(grid, n_snap, device):
    import torch
    import workloads as W
    rho = torch.empty((n_snap,) + grid.shape, dtype=torch.float32, device=device)
    for t in range(n_snap):
        rho[t] = W.cell_average(grid, W.density5(t), sub=2, device=device, as_tensor=True,
                                out_dtype=torch.float32)
        log(f"[bench] snapshot {t} generated")
    return rho


def time_path(plan, rho, phi, steps, warmup):
    """Mean ms/step over the timed region, per-step percentiles, wall time and
    per-stage device times.  Every event is recorded on the plan's stream."""
    import torch
    for _ in range(warmup):
        plan.potential(rho, out=phi)
    torch.cuda.synchronize()
    plan.timing(True)
    plan.stage_times(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(plan.stream)
    for k in range(steps):
        plan.potential(rho, out=phi)
        ev[k + 1].record(plan.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = plan.stage_times(reset=True)
    plan.timing(False)
    per_step = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    pct = {"p10": float(np.percentile(per_step, 10)), "median": float(np.median(per_step)),
           "p90": float(np.percentile(per_step, 90))}
    return ev[0].elapsed_time(ev[steps]) / steps, wall, stages, pct


def cpu_baseline(lmax):
    """The oracle, as it stands, on a bounded sample of the same workload:
    the large workload's lmax and radial spacing law on a coarser angular
    grid (pi/128, 64x192 per patch) and 144 shells.  Timed: moments, radial
    sums and expansion, single-threaded (its table build, run on a process
    pool beforehand, is excluded, as on the GPU)."""
    import oracle as O
    import workloads as W
    g = W.yinyang(64, W.log_edges(144, 3.0), lmax)
    rho = W.random_rho(g, 5005)
    w = O.overlap_weights(g)
    U, Q = O.tables_parallel(g, lmax, w, workers=max(1, min(16, os.cpu_count() or 1)))
    t0 = time.perf_counter()
    B = O.moments(g, lmax, U, rho)
    M = O.radial(g, lmax, B)
    O.expand(g, lmax, Q, M)
    dt = time.perf_counter() - t0
    terms = g.n_cells * g.n_lm
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {
        "value": terms / dt,
        "unit": "terms/s",
        "cores": 1,
        "cpu": cpu,
        "kind": "oracle",
        "sample": (f"lmax {lmax}, Yin-Yang pi/128 (2x64x192 cells), 144 log-spaced shells, "
                   f"{terms:.3e} terms; moments + radial sums + expansion in {dt:.1f} s, "
                   f"single thread ({os.cpu_count()} host cores)"),
    }


def fp64_workload(dev, steps):
    """The FP64 workload (Yin-Yang pi/128, 400 shells of ratio 1.02, lmax 25,
    ellipsoid + 16 blobs, float64 density): ms per solve on the FP64 path
    (plan autotuned), throughput, and the FP64 MFMA fraction of its moment
    contraction (2 flops per folded term against 78.6 TFLOP/s)."""
    import torch
    import paper_1903_08475_amd as mpg
    import workloads as W
    g = W.config2()
    rho = W.cell_average(g, W.density2(), sub=4, device=dev, as_tensor=True)
    phi = torch.empty_like(rho)
    plan = mpg.Plan(g, precision="fp64")
    tuned = plan.autotune(rho)
    ms, _, st, pct = time_path(plan, rho, phi, steps, 2)
    per = {k: v[0] / max(1, v[1]) for k, v in st.items()}
    flops = 2.0 * g.n_r * g.n_ang * g.n_lm
    out = {"workload": "Yin-Yang pi/128 (2x64x192 cells), 400 shells of ratio 1.02, lmax 25, float64",
           "precision": "fp64", "ms_per_solve": ms, "ms_percentiles": pct,
           "value": g.n_cells * g.n_lm / (ms * 1e-3), "unit": "terms/s", "stage_ms": per,
           "moments_fp64_mfma_frac": flops / (per["moments"] * 1e-3) / PEAK_FP64,
           "expansion_fp64_mfma_frac": flops / (per["expansion"] * 1e-3) / PEAK_FP64,
           "autotuned": {"gemm1_splitk": tuned[0], "scan_chunks": tuned[1],
                         "moment_tiles": "128x128" if tuned[2] == 1 else "64x64"}}
    log(f"[bench] FP64 workload: {ms:.3f} ms per solve")
    return out


def separable_flops(grid, n_fields):
    """Algorithmic FP64 flops of one launch of each phi transform of the
    separable method: 2 per product, rows (field, patch, shell, theta row)
    x phi columns (2 lmax + 1) x cells walked by the moments' (half of a
    row's under the mirror fold) or points computed by the expansion's (one
    per mirror pair, plus the unpaired ones)."""
    rows = n_fields * grid.n_patches * grid.n_r * grid.n_theta
    n = grid.n_phi
    mir = n % 2 == 0 and abs(grid.phi0 + 0.5 * n * grid.dphi) <= 1e-12
    cells = n // 2 if mir else n
    centre = getattr(grid, "eval_point", "vertex") == "centre"
    points = (n // 2 if centre else n // 2 + 1) if mir else n
    cols = 2 * grid.lmax + 1
    return {"phi_moments": 2.0 * rows * cells * cols, "phi_expansion": 2.0 * rows * points * cols}


def separable_bytes(grid, n_fields, split=False):
    """Algorithmic HBM bytes of one launch of each phi transform: the FP32
    field once (4 bytes per cell) and the phi transforms once (2 lmax + 1
    columns per row; FP64, or in the split form FP32 past the order-0
    column)."""
    rows = n_fields * grid.n_patches * grid.n_r * grid.n_theta
    field = 4.0 * rows * grid.n_phi
    transforms = rows * (8.0 + (4.0 if split else 8.0) * 2 * grid.lmax)
    return {"phi_moments": field + transforms, "phi_expansion": field + transforms}


SEP_STAGES = {"input_split": "phi_moments", "moments": "theta_and_rotations", "radial_scan": "radial_scan",
              "expansion": "phi_expansion"}
SEP_KERNELS = {"phi_moments": "k_sep_phi1 (moments' phi transform, FP64 MFMA)",
               "phi_expansion": "k_sep_phi2 (expansion's phi transform, FP64 MFMA)"}
SEP_KERNELS_SPLIT = {"phi_moments": "k_sep_phi1s (moments' phi transform, split-BF16 MFMA)",
                     "phi_expansion": "k_sep_phi2s (expansion's phi transform, split-BF16 MFMA)"}


def separable_workload(grid, rho, steps, warmup, ref=None, precision="fp64"):
    """The separable method (FP64, or its split form: the phi transforms in
    six bf16 piece products with FP32 accumulation) on the large workload:
    ms per solve, per-stage times (the theta contractions and rotations
    launch twice per solve), the roofline of its dominant kernel (the
    costlier phi transform) and its difference from a reference potential
    when given."""
    import torch
    import paper_1903_08475_amd as mpg
    n = rho.shape[0]
    plan = mpg.Plan(grid, precision=precision, max_fields=n, method="separable")
    phi = torch.empty_like(rho)
    ms, _, st, pct = time_path(plan, rho, phi, steps, warmup)
    per = {SEP_STAGES[k]: v[0] / max(1, v[1]) for k, v in st.items()}
    per_solve = {SEP_STAGES[k]: v[0] / steps for k, v in st.items()}
    flops = separable_flops(grid, n)
    dom = max(("phi_moments", "phi_expansion"), key=lambda k: per[k])
    achieved = flops[dom] / (per[dom] * 1e-3)
    out = {"precision": precision, "ms_per_step": ms, "ms_per_step_percentiles": pct,
           "value": grid.n_cells * grid.n_lm * n / (ms * 1e-3), "unit": "terms/s",
           "stage_ms_per_solve": per_solve}
    key = "separable" if precision == "fp64" else "separable_split"
    if precision == "fp64":
        out["phi_fp64_mfma_frac"] = {k: flops[k] / (per[k] * 1e-3) / PEAK_FP64 for k in flops}
        out["roofline"] = {"bound": "mfma", "kernel": SEP_KERNELS[dom], "achieved": achieved / 1e12,
                           "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
                           "traffic": traffic_record(dom, key), "avg_launch_ms": per[dom],
                           "algorithmic_flops_per_launch": flops[dom]}
    else:
        # six bf16 MFMA products per product leave the split transforms bound
        # by HBM: algorithmic bytes are the FP32 field (read by the moments',
        # written by the expansion's) and the phi transforms between them
        byts = separable_bytes(grid, n, split=True)
        ach = byts[dom] / (per[dom] * 1e-3)
        out["phi_bf16_mfma_frac"] = {k: 6 * flops[k] / (per[k] * 1e-3) / PEAK_BF16 for k in flops}
        out["phi_hbm_frac"] = {k: byts[k] / (per[k] * 1e-3) / PEAK_HBM for k in byts}
        out["roofline"] = {"bound": "hbm", "kernel": SEP_KERNELS_SPLIT[dom], "achieved": ach / 1e9,
                           "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                           "traffic": traffic_record(dom, key), "avg_launch_ms": per[dom],
                           "algorithmic_bytes_per_launch": byts[dom],
                           "algorithmic_flops_per_launch": flops[dom]}
    if ref is not None:
        out64 = torch.empty_like(ref)
        plan.potential(rho, out=out64)
        torch.cuda.synchronize()
        out["vs_dense_fp64_max_rel_err"] = float((out64 - ref).abs().max() / ref.abs().max())
        del out64
    log(f"[bench] separable method: {ms:.3f} ms/step; per solve {per_solve}")
    del plan, phi
    return out


def precision_workload(dev):
    """The precision workload (Yin-Yang pi/32, 32 shells, lmax 40; ellipsoid +
    a point-like Gaussian mass): max-norm relative error of Phi against the
    oracle for both split forms and the FP64 path, and split vs FP64."""
    import torch
    import oracle as O
    import paper_1903_08475_amd as mpg
    import workloads as W
    g = W.config3()
    rho = W.cell_average(g, W.density3(), sub=4)
    phi_ref, *_ = O.potential(g, g.lmax, rho, O.overlap_weights(g))
    t = torch.tensor(rho, device=dev)
    res = {"workload": "Yin-Yang pi/32 (2x16x48 cells), 32 shells, lmax 40, ellipsoid + Gaussian mass"}
    phis = {}
    for prec in ("fp64", "split_bf16_tiered", "split_bf16"):
        phis[prec] = mpg.Plan(g, precision=prec).potential(t).cpu().numpy()
        res[f"{prec}_vs_oracle_max_rel_err"] = float(np.abs(phis[prec] - phi_ref).max() / np.abs(phi_ref).max())
    for prec in ("split_bf16_tiered", "split_bf16"):
        res[f"{prec}_vs_fp64_max_rel_err"] = float(np.abs(phis[prec] - phis["fp64"]).max()
                                                   / np.abs(phis["fp64"]).max())
    log(f"[bench] precision workload: tiered vs oracle {res['split_bf16_tiered_vs_oracle_max_rel_err']:.3e}")
    return res


def batch_workload(dev, reps, autotune=True, precisions=("split_bf16_tiered", "split_bf16", "fp64")):
    """The batching workload: 64 seeded fields of uneven sizes (shells
    U{100..800}, Delta in {pi/64, pi/128, pi/256}, lmax U{12..32}; ellipsoid
    with random semi-axes plus 4-32 blobs), solved in one batched call (one
    persistent launch per stage, replayed from a captured hipGraph), in the
    split-BF16 forms on the float32-rounded densities and in FP64.  Reports
    the batch makespan, its throughput, the per-field completion times
    inside one batched call (p50/p99, device wall clock), and per-field
    single-solve latencies (p50/p99) beside them."""
    import torch
    import paper_1903_08475_amd as mpg
    import workloads as W
    fields = W.config4_fields()
    rho64 = []
    for k, (g, d) in enumerate(fields):
        rho64.append(W.cell_average(g, d, sub=2, device=dev, as_tensor=True))
        if k % 16 == 15:
            log(f"[bench] batch: {k + 1} fields generated")
    terms = sum(g.n_cells * g.n_lm for g, _ in fields)
    res = {"fields": len(fields), "terms_per_batch": terms, "plans_autotuned": autotune,
           "cells_per_batch": sum(g.n_cells for g, _ in fields)}
    phis = {}
    for prec in precisions:
        dtype = torch.float64 if prec == "fp64" else torch.float32
        plans = [mpg.Plan(g, precision=prec) for g, _ in fields]
        rhos = [r.to(dtype) for r in rho64]
        out = [torch.empty_like(r) for r in rhos]
        if autotune:  # each field's plan on its own input (the batch takes its shapes and scan chunks)
            for p, r in zip(plans, rhos):
                p.autotune(r)
            log(f"[bench] batch {prec}: {len(plans)} plans autotuned")
        ch = mpg.batch_choices(plans, dtype)
        res.setdefault("choices", {})[prec] = {
            "gemm1_256x128": sum(c[2] == 2 for c in ch), "gemm2_256x128": sum(c[3] == 2 for c in ch),
            "scan_chunks": {str(k): sum(c[1] == k for c in ch) for k in sorted({c[1] for c in ch})}}
        mpg.potential_batch(plans, rhos, out)  # builds and captures the graph
        torch.cuda.synchronize()
        stream = plans[0].stream
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            mpg.potential_batch(plans, rhos, out)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        # completion time of every field inside the last batched call (device wall clock)
        done = mpg.batch_field_times(plans, dtype)
        lat = []
        for p, r, o in zip(plans, rhos, out):
            p.potential(r, out=o)  # warm
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(p.stream)
            p.potential(r, out=o)
            e1.record(p.stream)
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1))
        lat = np.array(lat)
        res[prec] = {"batch_ms": ms, "value": terms / (ms * 1e-3), "unit": "terms/s",
                     "field_done_in_batch_ms_p50": float(np.percentile(done, 50)),
                     "field_done_in_batch_ms_p99": float(np.percentile(done, 99)),
                     "single_field_ms_p50": float(np.percentile(lat, 50)),
                     "single_field_ms_p99": float(np.percentile(lat, 99)),
                     "sum_single_field_ms": float(lat.sum())}
        log(f"[bench] batch {prec}: {ms:.2f} ms per batch, singles p50 {res[prec]['single_field_ms_p50']:.3f} "
            f"p99 {res[prec]['single_field_ms_p99']:.3f} ms")
        mpg.potential_batch(plans, rhos, out)
        torch.cuda.synchronize()
        phis[prec] = out
        del plans
    for prec in precisions:
        if prec == "fp64" or "fp64" not in phis:
            continue
        err = 0.0
        for x, y in zip(phis[prec], phis["fp64"]):
            err = max(err, float((x.double() - y).abs().max() / y.abs().max()))
        res[prec]["vs_fp64_max_rel_err"] = err
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--snapshots", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--precision", default="split_bf16_tiered", choices=["split_bf16_tiered", "split_bf16"],
                    help="split form of the timed step (the other one is timed beside it)")
    ap.add_argument("--no-other-split", action="store_true", help="skip timing the other split form")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plans' default K split and scan schedule instead of autotuning them")
    ap.add_argument("--tuning", default=None,
                    help="SPLITK,CHUNKS,GEMM1_ROWS,GEMM2_ROWS (or SPLITK,CHUNKS,GEMM2_ROWS with 128x256 moment "
                         "blocks): apply these choices to the timed plan instead of autotuning it (e.g. to "
                         "profile the configuration an autotuned run chose, without its timing launches)")
    ap.add_argument("--no-compare", action="store_true", help="skip the per-patch comparison method")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-field uneven batch (one batched call per precision)")
    ap.add_argument("--batch-all", action="store_true",
                    help="time the batch in the six-product split form too")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the FP64 workload and the precision workload")
    ap.add_argument("--no-separable", action="store_true", help="skip the separable method")
    ap.add_argument("--sep-precision", default="fp64", choices=["fp64", "split_bf16"],
                    help="precision of --only separable")
    ap.add_argument("--only", choices=["fp64", "precision", "batch", "separable"], default=None,
                    help="run only this workload (no headline line; e.g. to profile its kernels) and print its "
                         "JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the solver has no multi-GPU path)", file=sys.stderr)
        return 2
    if args.only:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        if args.only == "fp64":
            res = fp64_workload(dev, 10)
        elif args.only == "separable":
            import workloads as W
            grid = W.config5()
            res = separable_workload(grid, make_inputs(grid, args.snapshots, dev), args.steps, args.warmup,
                                     precision=args.sep_precision)
        elif args.only == "precision":
            res = precision_workload(dev)
        else:
            precs = ("split_bf16_tiered", "split_bf16", "fp64") if args.batch_all else ("split_bf16_tiered", "fp64")
            res = batch_workload(dev, args.batch_reps, autotune=not args.no_autotune, precisions=precs)
        print(json.dumps({args.only: res}), flush=True)
        return 0

    import workloads as W
    cpu = None
    if not args.no_cpu_baseline:
        # first, before the GPU is initialised (the table build forks workers)
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(W.config5().lmax)
        log(f"[bench] CPU oracle: {cpu['value']:.3e} terms/s")

    import torch
    import paper_1903_08475_amd as mpg

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    grid = W.config5()
    n = args.snapshots
    rho = make_inputs(grid, n, dev)
    phi = torch.empty_like(rho)
    terms_per_step = grid.n_cells * grid.n_lm * n
    rows, n_ang, n_lm = n * grid.n_r, grid.n_ang, grid.n_lm
    alg_flops = 2.0 * rows * n_ang * n_lm  # per contraction launch (folded)

    prec = args.precision
    other = "split_bf16" if prec == "split_bf16_tiered" else "split_bf16_tiered"
    log(f"[bench] building {prec} plan")
    plan = mpg.Plan(grid, precision=prec, max_fields=n)
    tuned = None
    def shape(r):
        return "128x256" if r == 1 else "256x128"
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        sk, ch, g1, g2 = vals if len(vals) == 4 else (vals[0], vals[1], 1, vals[2])
        plan.set_tuning(sk, ch, g1, g2)
        tuned = {"gemm1_splitk": sk, "scan_chunks": ch, "moment_block": shape(g1), "expansion_block": shape(g2),
                 "given": True}
        log(f"[bench] tuning given: {tuned}")
    elif not args.no_autotune:
        sk, ch, g1, g2 = plan.autotune(rho)
        tuned = {"gemm1_splitk": sk, "scan_chunks": ch, "moment_block": shape(g1), "expansion_block": shape(g2)}
        log(f"[bench] autotuned: {tuned}")
    ms, wall, stages, pct = time_path(plan, rho, phi, args.steps, args.warmup)
    log(f"[bench] {prec}: {ms:.3f} ms/step ({pct}); stages {stages}")
    prods = products_per_term(grid.lmax, prec)
    desc = {"split_bf16": "six MFMA products per product",
            "split_bf16_tiered": (f"three MFMA products per product (h*h + h*m + m*h), six on the moments of "
                                  f"degree <= {TIER_LMAX['moments']} ({prods['moments']:.2f} per product on "
                                  f"average)")}

    out = {
        "metric": METRIC,
        "value": terms_per_step / (ms * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_percentiles": pct,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": ("large: Yin-Yang pi/256 (2x128x384 cells), 1200 log-spaced shells over 3 decades, "
                         "lmax 48, batch of 8 float32 snapshots (ellipsoid spun 0.05 rad/step + 64 drifting "
                         "blobs)"),
            "global_batch": n,
            "n_cells_per_snapshot": grid.n_cells,
            "n_lm": n_lm,
            "terms_per_step": terms_per_step,
            "precision": (f"{prec}: three bf16 pieces per operand, {desc[prec]}, FP32 accumulate, "
                          "FP64 flush, FP64 tables and scans"),
            "parallelism": "single GPU",
            "autotuned": tuned,
        },
    }

    # dominant kernel and its roofline
    per = {k: (v[0] / max(1, v[1])) for k, v in stages.items()}
    dom = max(("moments", "expansion"), key=lambda k: per[k])
    achieved = alg_flops / (per[dom] * 1e-3)
    out["roofline"] = {
        "bound": "mfma",
        "kernel": "k_gemm1 (split-BF16 moment contraction)" if dom == "moments" else
                  "k_gemm2 (split-BF16 expansion)",
        "achieved": achieved / 1e12,
        "peak": PEAK_BF16 / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_BF16,
        "traffic": traffic_record(dom, prec),
        "executed_mfma_frac": prods[dom] * achieved / PEAK_BF16,
        "products_per_term": prods[dom],
        "avg_launch_ms": per[dom],
        "stage_ms": {k: per[k] for k in per},
    }

    sep = sep_split = None
    phi_other = None
    if not args.no_other_split:
        log(f"[bench] {other} on the same workload")
        po = mpg.Plan(grid, precision=other, max_fields=n)
        if not args.no_autotune:
            po.autotune(rho)
        phi_other = torch.empty_like(rho)
        ms_o, _, st_o, _ = time_path(po, rho, phi_other, args.steps, 1)
        out["other_split_form"] = {
            "precision": other,
            "value": terms_per_step / (ms_o * 1e-3),
            "ms_per_step": ms_o,
            "stage_ms": {k: v[0] / max(1, v[1]) for k, v in st_o.items()},
            "products_per_term": products_per_term(grid.lmax, other),
        }
        log(f"[bench] {other}: {ms_o:.3f} ms/step")
        del po

    if not args.no_fp64:
        log("[bench] FP64 path on the same workload")
        ref = torch.empty_like(rho, dtype=torch.float64)
        plan64 = mpg.Plan(grid, precision="fp64", max_fields=n)
        if not args.no_autotune:
            plan64.autotune(rho)
        ms64, _, st64, _ = time_path(plan64, rho, ref, args.fp64_steps, 1)
        plan.potential(rho, out=phi)
        torch.cuda.synchronize()
        err = float((phi.to(torch.float64) - ref).abs().max() / ref.abs().max())
        out["fp64_path"] = {
            "value": terms_per_step / (ms64 * 1e-3),
            "ms_per_step": ms64,
            "stage_ms": {k: v[0] / max(1, v[1]) for k, v in st64.items()},
            "fp64_mfma_frac": alg_flops / (st64["moments"][0] / max(1, st64["moments"][1]) * 1e-3) / PEAK_FP64,
        }
        out["split_vs_fp64_max_rel_err"] = err
        out["speedup_vs_fp64"] = ms64 / ms
        if phi_other is not None:
            out["other_split_form"]["vs_fp64_max_rel_err"] = float(
                (phi_other.to(torch.float64) - ref).abs().max() / ref.abs().max())
        del plan64
        if not args.no_separable:
            log("[bench] separable method on the same workload (FP64 and split-BF16)")
            sep = separable_workload(grid, rho, args.steps, args.warmup, ref)
            sep_split = separable_workload(grid, rho, args.steps, args.warmup, ref, precision="split_bf16")
        del ref

    if not args.no_compare:
        # the comparison method of the paper: every patch's moments in its own
        # frame, potentials of the patches added (same result up to rounding)
        log(f"[bench] per-patch comparison method ({prec})")
        pp = mpg.Plan(grid, precision=prec, max_fields=n, method="per_patch")
        if not args.no_autotune:
            pp.autotune(rho)
        phi_pp = torch.empty_like(rho)
        ms_pp, _, st_pp, _ = time_path(pp, rho, phi_pp, args.fp64_steps, 1)
        plan.potential(rho, out=phi)
        torch.cuda.synchronize()
        out["per_patch_method"] = {
            "value": terms_per_step / (ms_pp * 1e-3),
            "ms_per_step": ms_pp,
            "stage_ms": {k: v[0] / max(1, v[1]) for k, v in st_pp.items()},
            "max_rel_diff_vs_paper_method": float((phi_pp.double() - phi.double()).abs().max()
                                                  / phi.double().abs().max()),
            "paper_method_speedup": ms_pp / ms,
        }
        log(f"[bench] per-patch method: {ms_pp:.2f} ms/step ({ms_pp / ms:.2f}x the paper's method)")
        del pp, phi_pp

    if not args.no_workloads or not args.no_batch:
        del rho, phi
        torch.cuda.empty_cache()
    if not args.no_workloads:
        log("[bench] FP64 workload")
        out["fp64_workload"] = fp64_workload(dev, 10)
        log("[bench] precision workload")
        out["precision_workload"] = precision_workload(dev)
    if not args.no_batch:
        log("[bench] 64-field batch")
        torch.cuda.empty_cache()
        precs = ("split_bf16_tiered", "split_bf16", "fp64") if args.batch_all else ("split_bf16_tiered", "fp64")
        out["batch"] = batch_workload(dev, args.batch_reps, autotune=not args.no_autotune, precisions=precs)

    if args.no_fp64 and not args.no_separable:
        log("[bench] separable method on the same workload (FP64 and split-BF16)")
        sep = separable_workload(grid, rho, args.steps, args.warmup)
        sep_split = separable_workload(grid, rho, args.steps, args.warmup, precision="split_bf16")
    if sep is not None:
        # the headline: the fastest separable form within the metric's bar
        # (split-BF16 within 1e-6 of FP64; FP64 within 1e-12 of the oracle);
        # the dense split-BF16 path's line moves under its own key
        head = sep
        split_ok = sep_split is not None and sep_split.get("vs_dense_fp64_max_rel_err", 0.0) <= 1e-6
        if split_ok and sep_split["ms_per_step"] < sep["ms_per_step"]:
            head = sep_split
        dense = {k: out.pop(k) for k in ("value", "ms_per_step", "ms_per_step_percentiles", "roofline")}
        dense.update(dtype="bf16", precision=out["config"]["precision"], autotuned=out["config"].pop("autotuned"))
        for k in ("split_vs_fp64_max_rel_err", "speedup_vs_fp64"):
            if k in out:
                dense[k] = out.pop(k)
        out["dense_split_bf16"] = dense
        split_head = head is sep_split
        out.update(value=head["value"], ms_per_step=head["ms_per_step"],
                   ms_per_step_percentiles=head["ms_per_step_percentiles"], dtype="bf16" if split_head else "f64",
                   roofline=head["roofline"])
        out["config"]["precision"] = (
            ("separable method, split-BF16: per-patch phi transforms (mirror cells folded) as six bf16 piece "
             "products per product on MFMA with FP32 accumulation (at most 192 terms), theta contractions per "
             "order and rotations per degree on FP64 MFMA; FP64 tables and scans") if split_head else
            ("separable method in FP64: per-patch phi transforms (mirror cells folded), theta contractions per "
             "order and rotations per degree on FP64 MFMA; FP64 tables and scans"))
        if split_head:
            out["split_vs_fp64_max_rel_err"] = sep_split["vs_dense_fp64_max_rel_err"]
        out["separable_method"] = sep
        if sep_split is not None:
            out["separable_split_bf16"] = sep_split
        if "fp64_path" in out:
            out["speedup_vs_dense_fp64"] = out["fp64_path"]["ms_per_step"] / head["ms_per_step"]
            out["speedup_vs_dense_split_bf16"] = dense["ms_per_step"] / head["ms_per_step"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
