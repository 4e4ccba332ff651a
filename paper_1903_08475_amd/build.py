"""Build the HIP library libmpg.so for gfx950 in-tree.

    python -m paper_1903_08475_amd.build
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libmpg.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions (v_pk_*_f32) stay off: some of their forms have
    # returned wrong results on this target without any error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    # private arrays stay in registers (or visibly in scratch), never in LDS
    "-mllvm", "-disable-promote-alloca-to-lds",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def build(verbose=True, jobs=None):
    """Compile every source to an object file (in parallel), then link the
    shared library; the result replaces libmpg.so atomically."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = jobs or max(1, min(len(sources()), os.cpu_count() or 1, 8))
    with tempfile.TemporaryDirectory(prefix="mpg_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in sources()]
        cmds = [[hipcc, *flags, *inc, "-c", src, "-o", obj] for src, obj in zip(sources(), objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(jobs) as pool:
            outs = list(pool.map(_run, cmds))
        tmp = SO + ".tmp%d" % os.getpid()
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        outs.append(_run(link))
    text = "\n".join(o for o in outs if o.strip())
    if text and verbose:
        print(text)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build()
    sys.exit(0)
