"""Queue order of the fused batch kernel (host logic, CPU): the library's
list scheduler (csrc/batch_order.h, compiled with g++) on the work items of
the 64-field batching workload.  Every item must come after every item of
its field's previous stage (a block only ever waits for items that running
blocks have taken, so the kernel cannot deadlock), and a replay of the queue
with perturbed item costs must keep the blocks busy."""
import os
import subprocess
import tempfile

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1903_08475_amd", "csrc")
WORKERS = 256

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "batch_order.h"
int main() {
    int n, workers;
    if (std::scanf("%d %d", &n, &workers) != 2) return 1;
    std::vector<mpg::FieldShape> s(n);
    for (auto &x : s)
        if (std::scanf("%d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d", &x.split_units, &x.rows1, &x.units_e,
                       &x.units_o, &x.six_e, &x.six_o, &x.kang, &x.splitk_min, &x.splitk_max, &x.scan_blocks,
                       &x.n_r, &x.chunks, &x.rows2, &x.cols2, &x.k2_three, &x.k2_six) != 16) return 1;
    for (const auto &it : mpg::fused_items(s, workers))
        std::printf("%d %d %d %d %d %.6f %d\n", it.f, it.st, it.a, it.b, it.c,
                    mpg::fused_cost(s[it.f], mpg::fused_splitk(s[it.f]), it.st, it.a, it.b) * (it.st == 3 ? it.c : 1),
                    mpg::fused_splitk(s[it.f]));
    return 0;
}
"""


def cdiv(a, b):
    return -(-a // b)


def shape(g, lmax, splitk_max=32, tier=15, chunks=16, g1=1, g2=1):
    """The fused kernel's work units of one Yin-Yang field (column layout:
    even-m and odd-m blocks padded to 32; tiles of 128, K slabs of 32;
    blocks of 128 x 256 (g1, g2 = 1) or 256 x 128 (2))."""
    kang = cdiv(g.n_theta * g.n_phi, 128) * 128
    ne = sum(1 if m == 0 else 2 for l in range(lmax + 1) for m in range(0, l + 1, 2))
    no = (lmax + 1) ** 2 - ne
    te = sum(1 if m == 0 else 2 for l in range(min(lmax, tier) + 1) for m in range(0, l + 1, 2))
    to = (min(lmax, tier) + 1) ** 2 - te
    ne_p, no_p = cdiv(ne, 32) * 32, cdiv(no, 32) * 32
    six_e, six_o = min(cdiv(te, 32) * 32, ne_p), min(cdiv(to, 32) * 32, no_p)
    nb = 2 if g1 == 1 else 1  # column tiles per moment block
    pe, po = cdiv(cdiv(ne_p, 128), nb), cdiv(cdiv(no_p, 128), nb)

    def three(nsl, six_sl):
        n3 = max(nsl - six_sl, 0)
        return n3 if n3 == nsl else n3 & ~1
    e3, o3 = three(ne_p // 32, six_e // 32), three(no_p // 32, six_o // 32)
    rt = cdiv(g.n_r, 128)
    at = kang // 128
    return [rt * cdiv(kang // 32, 4), rt if g1 == 1 else cdiv(rt, 2), pe, po, min(cdiv(six_e, 128 * nb), pe),
            min(cdiv(six_o, 128 * nb), po), kang, 1, splitk_max, cdiv(ne_p + no_p, 64), g.n_r, min(chunks, g.n_r),
            rt if g2 == 1 else cdiv(rt, 2), cdiv(at, 2) if g2 == 1 else at, e3 + o3,
            (ne_p // 32 - e3) + (no_p // 32 - o3)]


def schedule(shapes):
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "drv.cpp"), os.path.join(d, "drv")
        with open(src, "w") as f:
            f.write(DRIVER)
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True)
        inp = f"{len(shapes)} {WORKERS}\n" + "\n".join(" ".join(map(str, s)) for s in shapes) + "\n"
        out = subprocess.run([exe], input=inp, stdout=subprocess.PIPE, text=True, check=True).stdout
    return [tuple(float(v) if k == 5 else int(v) for k, v in enumerate(l.split())) for l in out.splitlines()]


def replay(queue, n_fields, rng, spread):
    """Blocks take items in queue order; an item starts once its field's
    previous stage has finished.  Costs are perturbed by U(1-spread, 1+spread)."""
    free = np.zeros(WORKERS)
    fin = {}
    left = {}
    for f, st, *_ in queue:
        left[(f, st)] = left.get((f, st), 0) + 1
    wait = busy = 0.0
    for f, st, a, b, c, cost, _ in queue:
        w = int(np.argmin(free))
        dep = 0.0
        if st > 0 and (f, st - 1) in left:
            assert left[(f, st - 1)] == 0, "an item precedes a producer"
            dep = fin[(f, st - 1)]
        start = max(free[w], dep)
        wait += start - free[w]
        t = cost * rng.uniform(1 - spread, 1 + spread)
        busy += t
        free[w] = start + t
        fin[(f, st)] = max(fin.get((f, st), 0.0), free[w])
        left[(f, st)] -= 1
    done = np.array([max(v for (g, s), v in fin.items() if g == f) for f in range(n_fields)])
    return free.max(), wait, busy, done


def check_queue(shapes, queue):
    """Every item exactly once, and every item after its producers."""
    expect = set()
    for f, s in enumerate(shapes):
        su, rt1, pe, po, _, _, _, _, _, sb, _, _, rt2, ap, _, _ = s
        sk = next(q[6] for q in queue if q[0] == f)
        expect |= {(f, 0, u) for u in range(0, su, 16)}
        expect |= {(f, 1, c, m, z) for z in range(sk) for m in range(rt1) for c in range(pe + po)}
        expect |= {(f, 2, x) for x in range(sb)}
        expect |= {(f, 3, m, a, min(2, ap - a)) for a in range(0, ap, 2) for m in range(rt2)}
    got = [(f, 0, a) if st == 0 else (f, 1, a, b, c) if st == 1 else (f, 2, a) if st == 2 else (f, 3, a, b, c)
           for f, st, a, b, c, _, _ in queue]
    assert len(got) == len(set(got)) == len(expect) and set(got) == expect
    # producers first
    seen = {}
    for f, st, *_ in queue:
        seen[(f, st)] = seen.get((f, st), 0) + 1
    count = dict(seen)
    seen.clear()
    for f, st, *_ in queue:
        if st > 0:
            assert seen.get((f, st - 1), 0) == count[(f, st - 1)]
        seen[(f, st)] = seen.get((f, st), 0) + 1


def test_batch_queue_order_of_the_64_field_workload():
    fields = W.config4_fields()
    shapes = [shape(g, g.lmax) for g, _ in fields]
    queue = schedule(shapes)
    check_queue(shapes, queue)
    # replays: exact and perturbed costs
    total = sum(q[5] for q in queue)
    rng = np.random.Generator(np.random.PCG64(7))
    for spread in (0.0, 0.3, 0.6):
        span, wait, busy, done = replay(queue, len(fields), rng, spread)
        lower = busy / WORKERS
        print(f"spread {spread}: makespan {span:.0f} (lower bound {lower:.0f}, ratio {span / lower:.3f}), "
              f"waits {wait / (busy + wait):.3%} of block time, field done p50 {np.median(done) / span:.2f} "
              f"p99 {np.percentile(done, 99) / span:.2f} of the makespan")
        assert span <= 1.12 * lower
        assert np.median(done) <= 0.6 * span
    assert total > 0


def test_batch_queue_with_each_fields_own_shapes():
    """Fields whose plans chose other block shapes and scan chunks: the
    queue still holds every item once, producers first, and replays keep
    the blocks busy."""
    fields = W.config4_fields()
    rng = np.random.Generator(np.random.PCG64(11))
    shapes = [shape(g, g.lmax, chunks=int(rng.choice([4, 8, 12, 16])), g1=int(rng.integers(1, 3)),
                    g2=int(rng.integers(1, 3))) for g, _ in fields]
    queue = schedule(shapes)
    check_queue(shapes, queue)
    span, wait, busy, done = replay(queue, len(fields), rng, 0.3)
    print(f"mixed shapes: makespan / lower bound {span / (busy / WORKERS):.3f}, "
          f"field done p50 {np.median(done) / span:.2f} of the makespan")
    assert span <= 1.12 * busy / WORKERS
    assert np.median(done) <= 0.6 * span
