"""Helpers shared by the GPU tests: oracle results cached per process."""
import functools

import numpy as np

import oracle as O
import workloads as W


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def cell_areas(g):
    th = g.theta0 + np.arange(g.n_theta) * g.dtheta
    return np.repeat(g.dphi * (np.cos(th) - np.cos(th + g.dtheta)), g.n_phi)


@functools.lru_cache(maxsize=16)
def oracle_tables(key):
    g = GRIDS[key]()
    w = O.overlap_weights(g) if g.n_patches == 2 else None
    U, Q = O.tables_parallel(g, g.lmax, w, workers=8) if g.n_ang >= 2048 else O.tables(g, g.lmax, w)
    return g, w, U, Q


def small_ragged():
    # shells, angular cells and columns all leave ragged tiles
    return W.yinyang(6, W.geometric_edges(37, 1.08), 11, name="ragged")


def polar_small():
    return W.polar(10, 20, W.uniform_edges(13), 9, name="polar")


def tiny():
    return W.yinyang(1, W.uniform_edges(1), 0, name="tiny")


def medium():
    return W.yinyang(24, W.geometric_edges(150, 1.03), 20, name="medium")


GRIDS = {
    "c1": W.config1,
    "c3": W.config3,
    "ragged": small_ragged,
    "polar": polar_small,
    "tiny": tiny,
    "medium": medium,
}
