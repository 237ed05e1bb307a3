"""Vertical line smoother (smoother = "line") through the C ABI against the
oracle: single forward and reverse sweeps, the V-cycle, converged solves in
both precisions and with CG, and its effect where the vertical coupling is
strong."""
import numpy as np
import pytest
import torch

from oracle import multigrid as mg
from paper_2101_08453_amd import inputs
from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mcw():
    from paper_2101_08453_amd import mcwind
    return mcwind


def _grid(name, **kw):
    print(f"[case] {name} {kw}", flush=True)
    return _mcw().grid_from_problem(gc.problem(name), **kw)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _level_vectors(L, seed):
    rng = np.random.default_rng(seed)
    m = L.mask.reshape(L.nz + 1, L.ny + 1, L.nx + 1)
    return rng.standard_normal(m.shape) * m, rng.standard_normal(m.shape) * m


@pytest.mark.parametrize("name", gc.CASES)
def test_line_sweeps_match_oracle(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60, smoother="line")
    levels = gc.hierarchy(name, coarse_max=60)
    for l in range(min(2, len(levels))):
        L = levels[l]
        for sweeps, rev in ((1, False), (-1, True)):
            x, f = _level_vectors(L, 30 + l)
            xg = _dev(x)
            g.smooth(l, xg, _dev(f), sweeps=sweeps)
            ref = mg.line_sweep_full(L.K_full, L.mask, L.dims, x.ravel(), f.ravel(), reverse=rev)
            assert gc.rel_err(xg.cpu().numpy().ravel(), ref) < 1e-12, (l, rev)


@pytest.mark.parametrize("name", ["c1", "distorted", "ragged"])
def test_line_vcycle_matches_oracle(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60, smoother="line")
    levels = gc.hierarchy(name, coarse_max=60)
    M = mg.Multigrid(levels, smoother="line")
    L = levels[0]
    x, f = _level_vectors(L, 31)
    xg = _dev(x)
    g.vcycle(xg, _dev(f))
    ref = M.vcycle(x.ravel()[L.free], f.ravel()[L.free])
    assert gc.rel_err(xg.cpu().numpy().ravel()[L.free], ref) < 1e-10


@pytest.mark.parametrize("krylov", [False, True])
@pytest.mark.parametrize("precision", ["fp32_refine", "fp64"])
@pytest.mark.parametrize("name", gc.CASES)
def test_line_solve_matches_oracle(name, precision, krylov):
    p = gc.problem(name)
    g, u0 = _grid(name, precision=precision, smoother="line", krylov=krylov, rtol=1e-12)
    lam, u, info = g.solve(u0)
    lam_ref, u_ref, _ = gc.solution(name)
    assert info["rel_residual"] <= 1e-12
    assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8
    assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8


def test_line_smoother_on_strong_vertical_coupling():
    """a = (1, 1, 1) over stretched layers from 5 m at dx = 30 m: the bottom
    layers couple vertically about 36 times more strongly than horizontally."""
    mcwind = _mcw()
    p = inputs.fractal_problem(256, 256, 15, 800.0 * 256 / 3000.0, 3)
    cyc = {}
    for sm in ("point", "line"):
        g, u0 = mcwind.grid_from_problem(p, precision="fp64", smoother=sm, rtol=1e-8)
        lam, _, info = g.solve(u0, want_u=False)
        cyc[sm] = (info["cycles"], info["rho"], lam)
        print(f"[line] {sm}: {info['cycles']} cycles, rate {info['rho']:.3f}", flush=True)
        g.close()
    assert cyc["line"][0] <= cyc["point"][0]
    d = float((cyc["line"][2] - cyc["point"][2]).abs().max() / cyc["point"][2].abs().max())
    assert d < 1e-6
