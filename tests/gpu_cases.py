"""Shared inputs and oracle results for the GPU parity tests (CPU side only)."""
import functools

import numpy as np

from oracle import fem, multigrid as mg, solve as osolve
from paper_2101_08453_amd import inputs


def make(name):
    if name == "c1":
        return inputs.c1()
    if name == "distorted":  # general isoparametric mesh, Gamma = bottom + x-low, anisotropic a
        return inputs.distorted_problem(9, 7, 5, seed=3, amp=0.2, a=(1.0, 1.5, 2.0),
                                        gamma=inputs.GAMMA_BOTTOM | inputs.GAMMA_XLO)
    if name == "ragged":  # odd counts everywhere, several tiles and a ragged tail, a3 = 3
        return inputs.hills_problem(37, 23, 7, 3, 11, a=(1.0, 1.0, 3.0), noise=0.3)
    if name == "box":  # uniform box, unit penalties
        return inputs.box_problem(16, 16, 8, hx=2.0, hy=2.0, hz=1.0, seed=4)
    if name == "tiles":  # larger than one element tile (15) and one column block (64) in x
        return inputs.fractal_problem(70, 33, 6, 60.0, 12)
    if name == "minimal":
        return inputs.box_problem(2, 2, 1, seed=1)
    raise KeyError(name)


CASES = ["c1", "distorted", "ragged", "box", "tiles"]


@functools.lru_cache(maxsize=None)
def problem(name):
    return make(name)


@functools.lru_cache(maxsize=None)
def system(name):
    return osolve.System.of(problem(name))


@functools.lru_cache(maxsize=None)
def hierarchy(name, coarse_max=1024, rule="operator", spacing="level"):
    p = problem(name)
    return mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, rule=rule, coarse_max=coarse_max,
                              spacing=spacing)


@functools.lru_cache(maxsize=None)
def solution(name):
    return osolve.solve(problem(name), rtol=1e-14)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def free_mask(p):
    return fem.free_mask(*p.dims, p.gamma)
