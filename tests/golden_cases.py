"""Readers of the text fixtures in tests/golden/ (closed forms and hand-derived
results, each cited in its file).  Input building only; no method arithmetic."""
import os
from fractions import Fraction

import numpy as np

from paper_2101_08453_amd import inputs

HERE = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                yield line


def cube_stencil():
    """{(di, dj, dk): K[n, n + offset] / h} of the uniform cube grid."""
    out = {}
    for line in _rows("q1_cube_stencil.txt"):
        di, dj, dk, v = line.split()
        out[(int(di), int(dj), int(dk))] = float(Fraction(v))
    return out


def coarsening_cases():
    """[(rule, spacing, a, gamma, coarse_max, (X, Y, Z), (coarsen_h, kept planes))]."""
    cases = []
    for line in _rows("coarsening_decisions.txt"):
        lhs, rhs = line.split("|")
        t = lhs.split()
        rule, _, spacing = t[0].partition(":")
        spacing = spacing or "level"
        a = [float(v) for v in t[1:4]]
        dx, nx, ny, gamma, cmax = float(t[4]), int(t[5]), int(t[6]), int(t[7]), int(t[8])
        if t[9] == "geom":
            thick = float(t[10]) * float(t[11]) ** np.arange(int(t[12]))
        else:
            thick = np.full(int(t[11]), float(t[10]))
        zeta = np.concatenate([[0.0], np.cumsum(thick)])
        grid = inputs.terrain_grid(np.zeros((ny + 1, nx + 1)), zeta, dx, dx)
        r = [int(v) for v in rhs.split()]
        cases.append((rule, spacing, a, gamma, cmax, grid, (bool(r[0]), r[1:])))
    return cases


def c5_gradient():
    """{"loss": L, "dL_da": [3], "directional": [20]} from c5_gradient.txt."""
    out = {"directional": []}
    for line in _rows("c5_gradient.txt"):
        t = line.split()
        if t[0] == "loss":
            out["loss"] = float(t[1])
        elif t[0] == "dL_da":
            out["dL_da"] = [float(v) for v in t[1:4]]
        elif t[0] == "dL_du0_dot_direction":
            out["directional"].append(float(t[2]))
    return out
