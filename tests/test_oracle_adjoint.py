"""Pins of the oracle's adjoint: the loss is exactly quadratic in u0, so
central differences along u0 are exact up to the solve tolerance (Q14);
along the penalties they are O(h^2)."""
import numpy as np

from oracle import adjoint
from paper_2101_08453_amd import inputs


def _problem():
    p = inputs.fractal_problem(12, 10, 5, 80.0, seed=21)
    mask = inputs.fire_mask(12, 10, seed=3) | True  # whole bottom layer keeps it well conditioned
    mask[:, :3] = False
    return p, mask


def test_u0_gradient_matches_central_differences():
    p, mask = _problem()
    L, g_u0, _ = adjoint.gradient(p, mask)
    dirs = inputs.random_directions(p.u0.shape, 4, seed=56)
    h = 1e-4
    for d in dirs:
        fd = (adjoint.loss_of(p, p.u0 + h * d, p.a, mask)
              - adjoint.loss_of(p, p.u0 - h * d, p.a, mask)) / (2 * h)
        an = float(np.sum(g_u0 * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * L)


def test_penalty_gradient_matches_central_differences():
    p, mask = _problem()
    p.a = np.array([1.0, 1.3, 2.0])
    _, _, g_a = adjoint.gradient(p, mask)
    h = 1e-4
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (adjoint.loss_of(p, p.u0, p.a + e, mask) - adjoint.loss_of(p, p.u0, p.a - e, mask)) / (2 * h)
        assert abs(fd - g_a[d]) <= 1e-6 * max(abs(g_a).max(), 1e-12)
