"""Pins of the oracle's vertical line smoother (block Gauss-Seidel over the
columns of each colour, every column solved exactly): the solution is a fixed
point, the error contracts in the energy norm, the reverse sweep is the energy
adjoint of the forward one, and where the only free nodes form one column a
single sweep is the direct solve while a point sweep is not."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import multigrid as mg
from paper_2101_08453_amd import inputs


def _level(p, coarse_max=60):
    return mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=coarse_max)


@pytest.fixture(scope="module")
def hills():
    p = inputs.hills_problem(10, 9, 6, 2, 81, a=(1.0, 1.0, 0.5), noise=0.2)
    return p, _level(p)


def _full(L, v):
    out = np.zeros(L.mask.size)
    out[L.free] = v
    return out


def test_exact_solution_is_a_fixed_point(hills):
    _, levels = hills
    L = levels[0]
    f = _full(L, np.random.default_rng(1).standard_normal(L.free.size))
    xs = _full(L, spla.spsolve(L.K.tocsc(), f[L.free]))
    for rev in (False, True):
        y = mg.line_sweep_full(L.K_full, L.mask, L.dims, xs, f, reverse=rev)
        assert np.abs(y - xs).max() < 1e-11 * np.abs(xs).max()


def test_error_contracts_in_the_energy_norm(hills):
    _, levels = hills
    L = levels[0]
    K = L.K
    rng = np.random.default_rng(2)
    for s in range(3):
        e = _full(L, rng.standard_normal(L.free.size))
        e1 = mg.line_sweep_full(L.K_full, L.mask, L.dims, e, np.zeros_like(e))
        n0 = e[L.free] @ (K @ e[L.free])
        n1 = e1[L.free] @ (K @ e1[L.free])
        assert n1 < n0


def test_reverse_line_sweep_is_the_energy_adjoint(hills):
    _, levels = hills
    L = levels[0]
    K = L.K
    rng = np.random.default_rng(3)
    x, y = (_full(L, v) for v in rng.standard_normal((2, L.free.size)))
    z = np.zeros_like(x)
    Ef = mg.line_sweep_full(L.K_full, L.mask, L.dims, x, z)[L.free]
    Eb = mg.line_sweep_full(L.K_full, L.mask, L.dims, y, z, reverse=True)[L.free]
    lhs = Ef @ (K @ y[L.free])
    rhs = x[L.free] @ (K @ Eb)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    Ef2 = mg.line_sweep_full(L.K_full, L.mask, L.dims, y, z)[L.free]
    assert abs(lhs - x[L.free] @ (K @ Ef2)) > 1e-6 * abs(lhs)


def test_a_single_free_column_is_solved_by_one_line_sweep():
    """2 x 2 elements with lambda = 0 on the sides and top leave one free
    column, so its block is the whole system."""
    p = inputs.hills_problem(2, 2, 9, 1, 82, a=(1.0, 1.0, 0.7))
    L = _level(p)[0]
    assert L.free.size == 9
    K = L.K
    f = _full(L, np.random.default_rng(4).standard_normal(L.free.size))
    xs = spla.spsolve(K.tocsc(), f[L.free])
    x0 = _full(L, np.random.default_rng(5).standard_normal(L.free.size))
    xl = mg.line_sweep_full(L.K_full, L.mask, L.dims, x0, f)
    xp = mg.gs_sweep_full(L.K_full, L.mask, L.dims, x0, f)
    assert np.abs(xl[L.free] - xs).max() < 1e-12 * np.abs(xs).max()
    assert np.abs(xp[L.free] - xs).max() > 1e-3 * np.abs(xs).max()


def test_symmetric_line_vcycle_is_symmetric_and_converges(hills):
    _, levels = hills
    M = mg.Multigrid(levels, symmetric=True, smoother="line")
    n = levels[0].K.shape[0]
    a, b = np.random.default_rng(5).standard_normal((2, n))
    ab, ba = a @ M.precondition(b), b @ M.precondition(a)
    assert abs(ab - ba) < 1e-12 * abs(ab)
    f = np.random.default_rng(6).standard_normal(n)
    x, hist = mg.Multigrid(levels, smoother="line").solve(f, rtol=1e-10)
    assert hist[-1] <= 1e-10 and len(hist) < 20
