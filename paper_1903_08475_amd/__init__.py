"""MI355X multipole gravity solver for multi-patch spherical grids.

Thin ctypes binding of the C ABI in ``include/mpg.h`` (built as
``libmpg.so``).  Every step of a solve runs in the library's HIP kernels;
this module only marshals arguments.  PyTorch supplies device memory and
the current HIP stream.  There is no CPU fallback: importing the binding
without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpg.so")

MPG_OK, MPG_EINVAL, MPG_ENOMEM, MPG_EDEVICE, MPG_EUNSUPPORTED = 0, -1, -2, -3, -4
MPG_FP64, MPG_SPLIT_BF16, MPG_SPLIT_BF16_TIERED = 0, 1, 2
MPG_F64, MPG_F32 = 0, 1

PRECISIONS = {"fp64": MPG_FP64, "split_bf16": MPG_SPLIT_BF16, "split_bf16_tiered": MPG_SPLIT_BF16_TIERED}
# "global": the paper's method; "per_patch": the comparison method (moments
# of every patch in its own frame, potentials of the patches added);
# "separable": the paper's method with each angular contraction factored
# into a phi transform and a theta contraction per order m (FP64; one patch
# or the Yin/Yang fold, patch 0 in the common frame)
METHODS = {"global": 0, "per_patch": 1, "separable": 2}
# where Phi is evaluated in each cell (on the shell's outer radius)
EVAL_POINTS = {"vertex": 0, "centre": 1}

# Every symbol the C ABI exports (kept equal to include/mpg.h by a test).
EXPORTS = ("mpg_plan", "mpg_plan_method", "mpg_moments", "mpg_potential", "mpg_potential_static",
           "mpg_potential_batch",
           "mpg_batch_field_times", "mpg_batch_choices", "mpg_autotune", "mpg_set_tuning", "mpg_tables",
           "mpg_plan_info",
           "mpg_timing", "mpg_stage_times", "mpg_sync", "mpg_destroy", "mpg_last_error")
STAGES = ("input_split", "moments", "radial_scan", "expansion")


class MpgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mpg error {code}: {msg}")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [
        ("n_patches", C.c_int), ("n_r", C.c_int), ("n_theta", C.c_int), ("n_phi", C.c_int),
        ("r_edges", C.POINTER(C.c_double)),
        ("theta0", C.c_double), ("phi0", C.c_double), ("dtheta", C.c_double), ("dphi", C.c_double),
        ("euler", C.POINTER(C.c_double)),
        ("overlap_w", C.POINTER(C.c_double)),
        ("G", C.c_double),
        ("w_per_patch", C.c_int),
        ("eval_point", C.c_int),
    ]


_lib = None


def lib():
    """Load libmpg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1903_08475_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.mpg_plan.argtypes = [C.POINTER(_Grid), C.c_int, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.mpg_plan_method.argtypes = [C.POINTER(_Grid), C.c_int, C.c_int, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.mpg_moments.argtypes = [vp, C.c_int, vp, C.c_int, vp, vp]
        L.mpg_potential.argtypes = [vp, C.c_int, vp, C.c_int, vp, C.c_int]
        L.mpg_potential_static.argtypes = [vp, C.c_int, vp, C.c_int, vp, C.c_int]
        L.mpg_potential_batch.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.c_int]
        L.mpg_batch_field_times.argtypes = [C.c_int, C.POINTER(vp), C.c_int, dp]
        ip = C.POINTER(C.c_int)
        L.mpg_batch_choices.argtypes = [C.c_int, C.POINTER(vp), C.c_int, ip, ip, ip, ip]
        L.mpg_autotune.argtypes = [vp, C.c_int, vp, C.c_int, ip, ip, ip, ip]
        L.mpg_set_tuning.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
        L.mpg_tables.argtypes = [vp, vp, vp, vp]
        L.mpg_plan_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_longlong)]
        L.mpg_timing.argtypes = [vp, C.c_int]
        L.mpg_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.c_int]
        L.mpg_sync.argtypes = [vp]
        L.mpg_destroy.argtypes = [vp]
        L.mpg_destroy.restype = None
        L.mpg_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != MPG_OK:
        raise MpgError(rc, lib().mpg_last_error().decode())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return MPG_F64
    if t.dtype == torch.float32:
        return MPG_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Plan:
    """A solver plan for one grid and lmax (tables built once on the device).

    grid: any object with n_patches, n_r, n_theta, n_phi, r_edges, theta0,
    phi0, dtheta, dphi, euler, G and optionally eval_point ("vertex", the
    default, or "centre") (e.g. ``workloads.Grid``).
    """

    def __init__(self, grid, lmax=None, precision="fp64", max_fields=1, stream=None, overlap_w=None,
                 method="global"):
        import torch
        self.lmax = grid.lmax if lmax is None else lmax
        self.grid = grid
        self.precision = precision
        self.max_fields = max_fields
        self.method = method
        self.shape = (grid.n_patches, grid.n_r, grid.n_theta, grid.n_phi)
        self.n_lm = (self.lmax + 1) ** 2
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._r = np.ascontiguousarray(grid.r_edges, dtype=np.float64)
        self._e = np.ascontiguousarray(np.asarray(grid.euler).reshape(-1), dtype=np.float64)
        n_ang = grid.n_theta * grid.n_phi
        self._w = None if overlap_w is None else np.ascontiguousarray(overlap_w, dtype=np.float64)
        if self._w is not None and self._w.size not in (n_ang, grid.n_patches * n_ang):
            raise ValueError("overlap_w must hold n_theta*n_phi or n_patches*n_theta*n_phi weights")
        g = _Grid()
        g.n_patches, g.n_r, g.n_theta, g.n_phi = grid.n_patches, grid.n_r, grid.n_theta, grid.n_phi
        g.r_edges = self._r.ctypes.data_as(C.POINTER(C.c_double))
        g.theta0, g.phi0, g.dtheta, g.dphi = grid.theta0, grid.phi0, grid.dtheta, grid.dphi
        g.euler = self._e.ctypes.data_as(C.POINTER(C.c_double))
        g.overlap_w = None if self._w is None else self._w.ctypes.data_as(C.POINTER(C.c_double))
        g.G = grid.G
        g.w_per_patch = int(self._w is not None and self._w.size != n_ang)
        ev = getattr(grid, "eval_point", "vertex")
        if ev not in EVAL_POINTS:
            raise ValueError(f"eval_point must be one of {sorted(EVAL_POINTS)}")
        g.eval_point = EVAL_POINTS[ev]
        h = C.c_void_p()
        _check(lib().mpg_plan_method(C.byref(g), self.lmax, PRECISIONS[precision], max_fields, METHODS[method],
                                     _stream_handle(self.stream), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mpg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fields(self, rho):
        if not rho.is_cuda or not rho.is_contiguous():
            raise ValueError("rho must be a contiguous device tensor")
        per = int(np.prod(self.shape))
        if rho.numel() % per or rho.numel() == 0:
            raise ValueError(f"rho has {rho.numel()} elements, not a multiple of {per}")
        return rho.numel() // per

    def potential(self, rho, out=None, out_dtype=None):
        """Phi at every upper cell vertex, same layout as rho."""
        import torch
        n = self._fields(rho)
        if out is None:
            out = torch.empty(rho.shape, dtype=out_dtype or rho.dtype, device=rho.device)
        if not out.is_contiguous() or out.numel() != rho.numel():
            raise ValueError("out must be contiguous with rho's size")
        _check(lib().mpg_potential(self._h, n, C.c_void_p(rho.data_ptr()), _dtype_code(rho),
                                   C.c_void_p(out.data_ptr()), _dtype_code(out)))
        return out

    def potential_static(self, rho, out):
        """As potential(), through mpg_potential_static: nothing is allocated,
        so the caller passes the output tensor (same size as rho)."""
        n = self._fields(rho)
        if not out.is_cuda or not out.is_contiguous() or out.numel() != rho.numel():
            raise ValueError("out must be a contiguous device tensor of rho's size")
        _check(lib().mpg_potential_static(self._h, n, C.c_void_p(rho.data_ptr()), _dtype_code(rho),
                                          C.c_void_p(out.data_ptr()), _dtype_code(out)))
        return out

    def moments(self, rho):
        """(B, M) in the real moment index, float64 [n_fields, n_r, n_lm]
        ([n_fields, n_patches, n_r, n_lm] for the per-patch method)."""
        import torch
        n = self._fields(rho)
        lead = (n, self.shape[0]) if self.method == "per_patch" else (n,)
        B = torch.zeros(lead + (self.shape[1], self.n_lm), dtype=torch.float64, device=rho.device)
        M = torch.zeros_like(B)
        _check(lib().mpg_moments(self._h, n, C.c_void_p(rho.data_ptr()), _dtype_code(rho),
                                 C.c_void_p(B.data_ptr()), C.c_void_p(M.data_ptr())))
        return B, M

    def tuning_key(self, n_fields, dtype):
        """Key of this plan's tuning in a cache file: precision, method, grid
        size, lmax, the number of fields and the input dtype."""
        g = self.grid
        return (f"{self.precision}/{self.method}/patches{g.n_patches}/shells{g.n_r}/"
                f"cells{g.n_theta}x{g.n_phi}/lmax{self.lmax}/fields{n_fields}/max{self.max_fields}/{dtype}")

    def autotune(self, rho, cache=None):
        """Time the K split of the moment contraction, (split forms) its block
        shape, the scan schedule and (split forms) the expansion's block
        shape on this input and keep the fastest; returns (splitk, chunks,
        gemm1_rows, gemm2_rows).  With cache (a JSON file path), choices
        stored there for the same key are applied without timing, and new
        ones are added to it; choices applied from the cache set the moment
        shape of batched solves too (a tuning run keeps one of its own for
        them, see mpg_autotune)."""
        import json
        n = self._fields(rho)
        key = self.tuning_key(n, str(rho.dtype).replace("torch.", ""))
        table = {}
        if cache is not None and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table and len(table[key]) == 4:
                res = tuple(int(v) for v in table[key])
                try:
                    self.set_tuning(*res)
                    return res
                except MpgError:
                    pass  # not applicable to this plan (e.g. its work space): time afresh
        out = [C.c_int() for _ in range(4)]
        _check(lib().mpg_autotune(self._h, n, C.c_void_p(rho.data_ptr()), _dtype_code(rho),
                                  *(C.byref(v) for v in out)))
        res = tuple(v.value for v in out)
        if cache is not None:
            table[key] = list(res)
            tmp = f"{cache}.tmp{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return res

    def set_tuning(self, splitk=0, chunks=0, gemm1_rows=0, gemm2_rows=0):
        """Set the autotuner's choices (0 leaves one as it is)."""
        _check(lib().mpg_set_tuning(self._h, splitk, chunks, gemm1_rows, gemm2_rows))

    def tables(self):
        """(U, Q, w) as float64 device tensors [n_patches, n_ang, n_lm] (twice)
        and [n_patches, n_ang]."""
        import torch
        n_ang = self.shape[2] * self.shape[3]
        dev = torch.device("cuda", torch.cuda.current_device())
        U = torch.zeros((self.shape[0], n_ang, self.n_lm), dtype=torch.float64, device=dev)
        Q = torch.zeros_like(U)
        w = torch.zeros((self.shape[0], n_ang), dtype=torch.float64, device=dev)
        _check(lib().mpg_tables(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(Q.data_ptr()),
                                C.c_void_p(w.data_ptr())))
        self.sync()
        return U, Q, w

    def timing(self, enable=True):
        """Record HIP events around every stage of later compute calls."""
        _check(lib().mpg_timing(self._h, 1 if enable else 0))

    def stage_times(self, reset=True):
        """{stage: (total ms, launches)} since the last reset."""
        ms = (C.c_double * 4)()
        n = (C.c_longlong * 4)()
        _check(lib().mpg_stage_times(self._h, ms, n, 1 if reset else 0))
        return {STAGES[i]: (ms[i], n[i]) for i in range(4)}

    def sync(self):
        _check(lib().mpg_sync(self._h))


def potential_batch(plans, rhos, phis):
    """Solve independent fields with their own plans in one call: field k
    is one field of plans[k]'s grid (rhos[k] and phis[k] contiguous device
    tensors of that size and one shared dtype)."""
    n = len(plans)
    if n == 0:
        raise ValueError("no fields")
    if not (len(rhos) == len(phis) == n):
        raise ValueError("plans, rhos and phis differ in length")
    dt = _dtype_code(rhos[0])
    for k, (pl, r, p) in enumerate(zip(plans, rhos, phis)):
        if _dtype_code(r) != dt or _dtype_code(p) != dt:
            raise TypeError("all rho and phi must share one dtype")
        per = int(np.prod(pl.shape))
        for name, t in (("rho", r), ("phi", p)):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name}[{k}] must be a contiguous device tensor")
            if t.numel() != per:
                raise ValueError(f"{name}[{k}] has {t.numel()} elements; one field of its plan has {per}")
    H = (C.c_void_p * n)(*[p.handle for p in plans])
    R = (C.c_void_p * n)(*[r.data_ptr() for r in rhos])
    P = (C.c_void_p * n)(*[p.data_ptr() for p in phis])
    _check(lib().mpg_potential_batch(n, H, R, P, dt))
    return phis


def batch_choices(plans, dtype):
    """The choices each field takes in a batched solve of these plans in this
    element type (torch.float32 or torch.float64): a list of (splitk,
    chunks, gemm1_rows, gemm2_rows), one per field, in set_tuning's order."""
    import numpy as np
    import torch
    n = len(plans)
    dt = MPG_F64 if dtype == torch.float64 else MPG_F32
    H = (C.c_void_p * n)(*[p.handle for p in plans])
    out = [np.zeros(n, dtype=np.int32) for _ in range(4)]
    _check(lib().mpg_batch_choices(n, H, dt, *(a.ctypes.data_as(C.POINTER(C.c_int)) for a in out)))
    return [tuple(int(a[f]) for a in out) for f in range(n)]


def batch_field_times(plans, dtype):
    """Per-field completion times (ms from the start of the batched solve,
    device wall clock) of the last potential_batch call with these plans
    and element type (torch.float32 or torch.float64)."""
    import numpy as np
    import torch
    n = len(plans)
    dt = MPG_F64 if dtype == torch.float64 else MPG_F32
    H = (C.c_void_p * n)(*[p.handle for p in plans])
    ms = np.zeros(n, dtype=np.float64)
    _check(lib().mpg_batch_field_times(n, H, dt, ms.ctypes.data_as(C.POINTER(C.c_double))))
    return ms
