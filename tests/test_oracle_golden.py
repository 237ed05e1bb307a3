"""The oracle against the text fixtures of tests/golden/: the closed-form
interior stencil of the trilinear element on a cube grid, and coarsening
decisions derived by hand from the rule and thresholds of Sec. 3."""
import numpy as np
import pytest

from oracle import fem, multigrid as mg
from paper_2101_08453_amd import inputs
from tests import golden_cases as gold


@pytest.mark.parametrize("h", [1.0, 2.5, 30.0])
def test_cube_grid_stencil_equals_golden_closed_form(h):
    n = 4
    grid = inputs.terrain_grid(np.zeros((n + 1, n + 1)), h * np.arange(n + 1.0), h, h)
    K = fem.assemble_stiffness(*grid, (1.0, 1.0, 1.0))
    c = fem.node_index(2, 2, 2, n, n)
    want = gold.cube_stencil()
    assert len(want) == 27
    for (di, dj, dk), v in want.items():
        got = K[c, fem.node_index(2 + di, 2 + dj, 2 + dk, n, n)]
        assert abs(got - v * h) <= 1e-14 * h, (di, dj, dk)


@pytest.mark.parametrize("case", range(len(gold.coarsening_cases())))
def test_coarsening_decision_equals_golden(case):
    rule, spacing, a, gamma, cmax, (X, Y, Z), want = gold.coarsening_cases()[case]
    ch, keep = mg.decide(X, Y, Z, a, rule, gamma, cmax, spacing)
    assert (bool(ch), list(keep)) == want
