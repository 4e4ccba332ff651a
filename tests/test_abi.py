"""The C-ABI library loads and exports every symbol include/mpg.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1903_08475_amd as mpg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "mpg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared() == sorted(mpg.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mpg.LIB_PATH):
        pytest.fail("libmpg.so is not built (run `python -m paper_1903_08475_amd.build`)")
    L = ctypes.CDLL(mpg.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name


def test_last_error_is_empty_string_initially():
    L = mpg.lib()
    assert isinstance(L.mpg_last_error(), bytes)


def test_plan_rejects_bad_grids_on_host():
    """Argument validation happens before any device call."""
    import numpy as np
    import workloads as W
    L = mpg.lib()
    g = W.config1()
    r = np.ascontiguousarray(g.r_edges)
    e = np.ascontiguousarray(g.euler.reshape(-1))
    s = mpg._Grid()
    s.n_patches, s.n_r, s.n_theta, s.n_phi = 2, g.n_r, g.n_theta, g.n_phi
    s.r_edges = r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s.euler = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s.theta0, s.phi0, s.dtheta, s.dphi, s.G = g.theta0, g.phi0, g.dtheta, g.dphi, 1.0
    h = ctypes.c_void_p()
    assert L.mpg_plan(ctypes.byref(s), -1, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EINVAL
    assert L.mpg_plan(ctypes.byref(s), 8, 7, 1, None, ctypes.byref(h)) == mpg.MPG_EINVAL
    assert L.mpg_plan(ctypes.byref(s), 8, 0, 0, None, ctypes.byref(h)) == mpg.MPG_EINVAL
    s.eval_point = 2
    assert L.mpg_plan(ctypes.byref(s), 8, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EINVAL
    assert b"eval_point" in L.mpg_last_error()
    s.eval_point = mpg.EVAL_POINTS["centre"]
    assert L.mpg_plan(ctypes.byref(s), 65, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EINVAL  # lmax above 64
    assert L.mpg_plan_method(ctypes.byref(s), 8, 0, 1, 3, None, ctypes.byref(h)) == mpg.MPG_EINVAL  # method
    # the separable method takes FP64 or the six-product split form
    sep = mpg.METHODS["separable"]
    assert L.mpg_plan_method(ctypes.byref(s), 8, 2, 1, sep, None, ctypes.byref(h)) == mpg.MPG_EUNSUPPORTED
    assert b"MPG_SPLIT_BF16" in L.mpg_last_error()
    bad = r.copy()
    bad[5] = bad[4]
    s.r_edges = bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.mpg_plan(ctypes.byref(s), 8, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EINVAL
    assert b"increase" in L.mpg_last_error()
    s.r_edges = r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    e3 = np.concatenate([e, [0.1, 0.2, 0.3]])
    s.euler = e3.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s.n_patches = 3  # general path: more than two patches need overlap weights
    assert L.mpg_plan(ctypes.byref(s), 8, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EUNSUPPORTED
    assert b"overlap_w" in L.mpg_last_error()
    for n in (0, 17):
        s.n_patches = n
        assert L.mpg_plan(ctypes.byref(s), 8, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EINVAL
    s.n_patches = 2
    e2 = e.copy()
    e2[5] = 0.3  # Yang no longer Yin turned by pi about z, nor related by the Yin<->Yang map
    s.euler = e2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.mpg_plan(ctypes.byref(s), 8, 0, 1, None, ctypes.byref(h)) == mpg.MPG_EUNSUPPORTED
    assert b"overlap_w" in L.mpg_last_error()
    assert h.value is None
    assert L.mpg_moments(None, 1, None, 0, None, None) == mpg.MPG_EINVAL
    assert L.mpg_potential(None, 1, None, 0, None, 0) == mpg.MPG_EINVAL
    assert L.mpg_set_tuning(None, 1, 16, 1, 1) == mpg.MPG_EINVAL
    assert L.mpg_autotune(None, 1, None, 0, None, None, None, None) == mpg.MPG_EINVAL
    assert L.mpg_batch_choices(0, None, mpg.MPG_F32, None, None, None, None) == mpg.MPG_EINVAL


class _FakeTensor:
    """Stands in for a device tensor in the host-side argument checks."""

    def __init__(self, n, dtype):
        self.n, self.dtype, self.is_cuda = n, dtype, True

    def numel(self):
        return self.n

    def is_contiguous(self):
        return True

    def data_ptr(self):
        raise AssertionError("the library must not be called")


class _FakePlan:
    def __init__(self, shape):
        self.shape = shape

    @property
    def handle(self):
        raise AssertionError("the library must not be called")


def test_batch_refuses_wrong_size_fields_before_the_library():
    import torch
    plans = [_FakePlan((2, 4, 3, 5)), _FakePlan((1, 2, 2, 2))]
    good = [_FakeTensor(120, torch.float32), _FakeTensor(8, torch.float32)]
    short = [_FakeTensor(120, torch.float32), _FakeTensor(7, torch.float32)]
    two = [_FakeTensor(240, torch.float32), _FakeTensor(8, torch.float32)]
    with pytest.raises(ValueError, match="rho\\[1\\] has 7 elements"):
        mpg.potential_batch(plans, short, good)
    with pytest.raises(ValueError, match="phi\\[0\\] has 240 elements"):
        mpg.potential_batch(plans, good, two)
    with pytest.raises(TypeError):
        mpg.potential_batch(plans, good, [_FakeTensor(120, torch.float64), _FakeTensor(8, torch.float32)])
    with pytest.raises(ValueError):
        mpg.potential_batch(plans[:1], good, good)
