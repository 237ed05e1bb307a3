"""Multigrid-preconditioned conjugate gradients (krylov = 1) through the C ABI:
the reverse smoother sweep and the symmetric V-cycle against the oracle's,
CG iterates against the oracle's CG, converged solves against the FP64 oracle
in both precisions, and the reduction of V-cycles on an anisotropic grid."""
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
def test_reverse_sweep_matches_oracle(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60)
    levels = gc.hierarchy(name, coarse_max=60)
    for l in range(min(2, len(levels))):
        L = levels[l]
        x, f = _level_vectors(L, 20 + l)
        xg = _dev(x)
        g.smooth(l, xg, _dev(f), sweeps=-1)
        ref = mg.gs_sweep_full(L.K_full, L.mask, L.dims, x.ravel(), f.ravel(), reverse=True)
        assert gc.rel_err(xg.cpu().numpy().ravel(), ref) < 1e-12, f"level {l}"


@pytest.mark.parametrize("name", gc.CASES)
def test_symmetric_vcycle_matches_oracle(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60, krylov=True)
    levels = gc.hierarchy(name, coarse_max=60)
    M = mg.Multigrid(levels, symmetric=True)
    L = levels[0]
    x, f = _level_vectors(L, 21)
    xg = _dev(x)
    g.vcycle(xg, _dev(f))
    ref = M.vcycle(x.ravel()[L.free], f.ravel()[L.free])
    assert gc.rel_err(xg.cpu().numpy().ravel()[L.free], ref) < 1e-10
    # B = V-cycle from zero is symmetric on the GPU too
    a, b = _level_vectors(L, 22)
    Ba, Bb = torch.zeros_like(_dev(a)), torch.zeros_like(_dev(b))
    g.vcycle(Ba, _dev(b))
    g.vcycle(Bb, _dev(a))
    ab, ba = float((_dev(a) * Ba).sum()), float((_dev(b) * Bb).sum())
    assert abs(ab - ba) < 1e-11 * abs(ab)


@pytest.mark.parametrize("name", ["c1", "ragged", "tiles"])
def test_cg_iterates_match_oracle_cg(name):
    """k CG steps from zero (one inner solve, no restart) against the oracle's CG."""
    k = 4
    p = gc.problem(name)
    g, u0 = _grid(name, precision="fp64", coarse_direct_max=60, krylov=True,
                  inner_cycles=k, max_cycles=k, rtol=1e-15)
    levels = gc.hierarchy(name, coarse_max=60)
    M = mg.Multigrid(levels, symmetric=True)
    lam, _, info = g.solve(u0, want_u=False, check=False)
    assert info["cycles"] == k
    S = gc.system(name)
    xk, _ = M.pcg(S.f, steps=k)
    got = lam.cpu().numpy().ravel()[levels[0].free]
    assert gc.rel_err(got, xk) < 1e-9
    assert info["rel_residual"] > 1e-15  # not converged: this is the k-th iterate


@pytest.mark.parametrize("precision", ["fp32_refine", "fp64"])
@pytest.mark.parametrize("name", gc.CASES)
def test_cg_solve_matches_oracle(name, precision):
    p = gc.problem(name)
    g, u0 = _grid(name, precision=precision, krylov=True, rtol=1e-12)
    lam, u, info = g.solve(u0)
    lam_ref, u_ref, _ = gc.solution(name)
    assert info["rel_residual"] <= 1e-12
    assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8
    assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8
    assert info["rel_divergence"] < 1e-10


@pytest.mark.parametrize("use_graph", [True, False])
def test_cg_takes_fewer_cycles_on_stretched_anisotropic_grid(use_graph):
    """a3 = 10 over fractal terrain with stretched layers: the case where the
    V-cycle alone converges slowest."""
    mcwind = _mcw()
    p = inputs.fractal_problem(128, 128, 15, 800.0 * 128 / 3000.0, 3, a=(1.0, 1.0, 10.0))
    res = {}
    for krylov in (False, True):
        g, u0 = mcwind.grid_from_problem(p, krylov=krylov, use_graph=use_graph, rtol=1e-8)
        lam, _, info = g.solve(u0, want_u=False)
        res[krylov] = (lam, info)
        print(f"[cg] krylov={krylov} cycles {info['cycles']} rho {info['rho']:.3f}", flush=True)
        g.close()
    assert res[True][1]["rel_residual"] <= 1e-8
    assert res[True][1]["cycles"] < res[False][1]["cycles"]
    d = float((res[True][0] - res[False][0]).abs().max() / res[False][0].abs().max())
    assert d < 1e-6


def test_graph_replay_is_bitwise_equal_to_direct_launches():
    mcwind = _mcw()
    p = gc.problem("ragged")
    out = []
    for use_graph in (True, False):
        g, u0 = mcwind.grid_from_problem(p, krylov=True, use_graph=use_graph, inner_cycles=3,
                                         autotune=False)
        lam, _, info = g.solve(u0, want_u=False)
        out.append((lam, info["cycles"]))
        # a second solve on the same handle replays the captured step again
        lam2, _, _ = g.solve(u0, want_u=False)
        assert torch.equal(lam, lam2)
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])


def test_krylov_needs_a_symmetric_cycle_and_batched_cg_equals_single_solves():
    mcwind = _mcw()
    with pytest.raises(mcwind.MCWError, match="nu_pre == nu_post"):
        _grid("box", krylov=True, nu_pre=2, nu_post=1)
    probs = [gc.problem("ragged"), gc.problem("box")]
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(q, krylov=True) for q in probs])]
    lams, _, infos, status = mcwind.solve_batch(grids, u0s)
    assert status == "MCW_OK"
    for g, u0, lam in zip(grids, u0s, lams):
        lam1, _, _ = g.solve(u0.clone(), want_u=False)
        assert torch.equal(lam, lam1)
