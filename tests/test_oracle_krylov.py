"""Pins of the oracle's symmetric V-cycle and multigrid-preconditioned CG
(an extension of the multigrid of Sec. 3): adjointness of the reverse sweep in
the energy inner product, symmetry and definiteness of the V-cycle operator,
the optimality of CG over the stationary iteration in the energy norm, and the
one-level case where the preconditioner is the exact inverse."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import multigrid as mg
from paper_2101_08453_amd import inputs


@pytest.fixture(scope="module")
def hier():
    p = inputs.hills_problem(12, 10, 6, 2, 71, a=(1.0, 1.0, 4.0), noise=0.2)
    return p, mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=40)


def _energy_error(K, x, xs):
    e = x - xs
    return float(np.sqrt(e @ (K @ e)))


def test_reverse_sweep_is_the_energy_adjoint_of_the_forward_sweep(hier):
    _, levels = hier
    M = mg.Multigrid(levels)
    K = levels[0].K
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, K.shape[0]))
    zero = np.zeros_like(x)
    Ef = lambda v: M.smooth(0, v, zero)
    Eb = lambda v: M.smooth(0, v, zero, reverse=True)
    lhs = Ef(x) @ (K @ y)
    rhs = x @ (K @ Eb(y))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the forward sweep alone is not self-adjoint: the pin can fail
    assert abs(lhs - x @ (K @ Ef(y))) > 1e-6 * abs(lhs)


def test_reverse_sweep_matches_full_vector_form(hier):
    _, levels = hier
    L = levels[0]
    M = mg.Multigrid(levels)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(L.mask.size) * L.mask
    f = rng.standard_normal(L.mask.size) * L.mask
    full = mg.gs_sweep_full(L.K_full, L.mask, L.dims, x, f, reverse=True)
    red = M.smooth(0, x[L.free], f[L.free], reverse=True)
    assert np.allclose(full[L.free], red, rtol=0, atol=1e-13 * np.abs(red).max())
    assert np.all(full[~L.mask] == 0.0)


@pytest.mark.parametrize("symmetric", [True, False])
def test_vcycle_operator_symmetry(hier, symmetric):
    _, levels = hier
    M = mg.Multigrid(levels, symmetric=symmetric)
    n = levels[0].K.shape[0]
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, n))
    ab, ba = a @ M.precondition(b), b @ M.precondition(a)
    if symmetric:
        assert abs(ab - ba) < 1e-12 * abs(ab)
        for s in range(4):
            v = np.random.default_rng(10 + s).standard_normal(n)
            assert v @ M.precondition(v) > 0.0
    else:
        assert abs(ab - ba) > 1e-6 * abs(ab)


def test_cg_energy_error_never_exceeds_the_stationary_iteration(hier):
    """The k-th CG iterate minimises the energy-norm error over the Krylov
    space that also holds the k-th iterate of x <- x + B (f - K x)."""
    p, levels = hier
    M = mg.Multigrid(levels, symmetric=True)
    K = levels[0].K
    f = np.random.default_rng(4).standard_normal(K.shape[0])
    xs = spla.spsolve(K.tocsc(), f)
    x = np.zeros_like(f)
    for k in range(1, 7):
        x = M.vcycle(x, f)
        xk, _ = M.pcg(f, steps=k)
        e_cg, e_st = _energy_error(K, xk, xs), _energy_error(K, x, xs)
        assert e_cg <= e_st * (1 + 1e-9), f"step {k}"
    assert e_cg < 0.5 * e_st


def test_cg_converges_to_the_direct_solution(hier):
    _, levels = hier
    M = mg.Multigrid(levels, symmetric=True)
    K = levels[0].K
    f = np.random.default_rng(5).standard_normal(K.shape[0])
    xs = spla.spsolve(K.tocsc(), f)
    x, hist = M.pcg(f, rtol=1e-12)
    assert np.abs(x - xs).max() < 1e-10 * np.abs(xs).max()
    assert np.linalg.norm(f - K @ x) <= 2e-12 * np.linalg.norm(f)
    assert len(hist) <= 12


def test_one_level_preconditioner_is_the_inverse():
    """With a single level the V-cycle is the direct solve, so CG ends in one step."""
    p = inputs.box_problem(4, 3, 2, seed=6)
    levels = mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=4096)
    assert len(levels) == 1
    M = mg.Multigrid(levels, symmetric=True)
    K = levels[0].K
    f = np.random.default_rng(7).standard_normal(K.shape[0])
    x, hist = M.pcg(f, steps=1)
    assert hist[0] < 1e-12
    assert np.abs(K @ x - f).max() < 1e-12 * np.abs(f).max()
