"""Steps around the solve through the C ABI (mcw_interp_wind, mcw_surface_wind)
against the oracle: every element and column on the small cases (all branches
of the vertical rule, clamping at the coarse-grid edges, hint resets on
distorted columns), sampled elements on the 3000x3000x15 grid, argument
checks, and the whole coupled step (interpolate, solve, read out)."""
import numpy as np
import pytest
import torch

from oracle import coupling, solve as osolve
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


def _coarse(p, spacing, shift=0.0, seed=61):
    """Levels from above the lowest centre to below the highest one, so that the
    log law, the linear part and the top all occur."""
    Lx = p.X.max() - p.X.min()
    Ly = p.Y.max() - p.Y.min()
    _, zeta = coupling.heights_above_ground(p.X, p.Y, p.Z)
    first = 1.5 * zeta.min() / 0.9
    nl = max(2, int(np.log(zeta.max() / (1.1 * first)) / np.log(1.3)))
    cw = inputs.coarse_wind(Lx, Ly, spacing=spacing, nl=nl, seed=seed, first=first, ratio=1.3)
    cw["x0"] += shift * Lx  # part of the fine grid lies outside the columns: clamped
    return cw


def _dev_cw(cw):
    d = dict(cw)
    d["hagl"] = torch.from_numpy(cw["hagl"]).cuda()
    d["wind"] = torch.from_numpy(cw["wind"]).cuda()
    return d


@pytest.mark.parametrize("fine_coarse", [False, True])
@pytest.mark.parametrize("name", gc.CASES)
def test_interpolation_matches_oracle(name, fine_coarse):
    """fine_coarse: coarse columns every 10 m, so that the columns around a tile of
    64 x 4 element columns do not fit in the kernel's LDS and it reads them from
    global memory; otherwise they are staged."""
    p = gc.problem(name)
    print(f"[case] interp {name} fine_coarse {fine_coarse}", flush=True)
    g, _ = _mcw().grid_from_problem(p)
    spacing = 10.0 if fine_coarse else max(60.0, (p.X.max() - p.X.min()) / 5.0)
    cw = _coarse(p, spacing=spacing, shift=0.3)
    u0 = g.interp_wind(_dev_cw(cw)).cpu().numpy()
    ref = coupling.interp_wind(p.X, p.Y, p.Z, cw)
    _, zeta = coupling.heights_above_ground(p.X, p.Y, p.Z)
    # the case exercises the log law, the linear part and the top
    assert zeta.min() < cw["hagl"][0].min() and zeta.max() > cw["hagl"][-1].min()
    assert gc.rel_err(u0, ref) < 1e-12


@pytest.mark.parametrize("name", gc.CASES)
def test_surface_wind_matches_oracle(name):
    p = gc.problem(name)
    print(f"[case] surface {name}", flush=True)
    g, _ = _mcw().grid_from_problem(p)
    _, zeta = coupling.heights_above_ground(p.X, p.Y, p.Z)
    u = np.random.default_rng(5).standard_normal((3,) + zeta.shape)
    ud = torch.from_numpy(u).cuda()
    for H in (0.5 * zeta[0].min(), 0.05, float(np.median(zeta)), 2.0 * zeta.max()):
        out = g.surface_wind(ud, H, z0=0.1).cpu().numpy()
        ref = coupling.surface_wind(p.X, p.Y, p.Z, u, H, 0.1)
        assert gc.rel_err(out, ref) < 1e-12, H


def test_sampled_elements_on_the_3000x3000x15_grid():
    """The launch shape of the benchmark: 9.0 M element columns, 15 layers, a
    coarse wind every 600 m with 40 levels; 2000 sampled elements and columns."""
    mcwind = _mcw()
    p = inputs.c3()
    print("[case] 3000x3000x15 coupling, sampled", flush=True)
    dev = torch.device("cuda")
    g = mcwind.Grid(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev),
                    torch.from_numpy(p.Z).to(dev), p.a)
    cw = inputs.coarse_wind(90000.0, 90000.0, spacing=600.0, nl=40)
    u0 = g.interp_wind(_dev_cw(cw))
    uv = g.surface_wind(u0, 6.1, z0=0.1)
    rng = np.random.default_rng(7)
    nz, ny, nx = p.dims[2], p.dims[1], p.dims[0]
    ks, js, is_ = rng.integers(0, nz, 2000), rng.integers(0, ny, 2000), rng.integers(0, nx, 2000)
    got = u0[:, torch.from_numpy(ks), torch.from_numpy(js), torch.from_numpy(is_)].cpu().numpy()
    for s in range(2000):
        ref = coupling.interp_wind_element(p.X, p.Y, p.Z, cw, ks[s], js[s], is_[s])
        assert np.abs(got[:, s] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    u0h = u0[:, :, torch.from_numpy(js[:200]), torch.from_numpy(is_[:200])].cpu().numpy()
    gotuv = uv[:, torch.from_numpy(js[:200]), torch.from_numpy(is_[:200])].cpu().numpy()
    for s in range(200):
        ref = coupling.column_profile(
            np.array([coupling.element_centre(p.X, p.Y, p.Z, k, js[s], is_[s])[0][2] for k in range(nz)])
            - p.Z[0, js[s]:js[s] + 2, is_[s]:is_[s] + 2].mean(), u0h[:2, :, s], 6.1, 0.1)
        assert np.abs(gotuv[:, s] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_bad_coarse_wind_is_rejected():
    mcwind = _mcw()
    p = gc.problem("box")
    g, _ = mcwind.grid_from_problem(p)
    cw = _coarse(p, spacing=8.0)
    bad = dict(cw)
    h = cw["hagl"].copy()
    h[3, 1, 1] = h[2, 1, 1]  # not increasing
    bad["hagl"] = h
    with pytest.raises(mcwind.MCWError, match="increase"):
        g.interp_wind(_dev_cw(bad))
    low = dict(cw)
    low["z0"] = float(cw["hagl"].min()) * 1.5  # lowest level not above z0
    with pytest.raises(mcwind.MCWError, match="above z0"):
        g.interp_wind(_dev_cw(low))
    one = dict(cw)
    one["hagl"] = np.ascontiguousarray(cw["hagl"][:, :, :1])
    one["wind"] = np.ascontiguousarray(cw["wind"][:, :, :, :1])
    with pytest.raises(mcwind.MCWError, match="ncx"):
        g.interp_wind(_dev_cw(one))
    u = torch.zeros((3, p.dims[2], p.dims[1], p.dims[0]), dtype=torch.float64, device="cuda")
    with pytest.raises(mcwind.MCWError, match="height"):
        g.surface_wind(u, -1.0)


def test_coupled_step_matches_oracle():
    """Coarse wind -> u0 -> mass-consistent wind -> surface wind at 6.1 m."""
    mcwind = _mcw()
    p = gc.problem("ragged")
    cw = _coarse(p, spacing=150.0)
    g, _ = mcwind.grid_from_problem(p, rtol=1e-12)
    u0 = g.interp_wind(_dev_cw(cw))
    lam, u, info = g.solve(u0)
    uv = g.surface_wind(u, 6.1, z0=0.1).cpu().numpy()
    u0_ref = coupling.interp_wind(p.X, p.Y, p.Z, cw)
    q = inputs.Problem("coupled", p.X, p.Y, p.Z, u0_ref, p.a, p.gamma)
    _, u_ref, _ = osolve.solve(q, rtol=1e-14)
    uv_ref = coupling.surface_wind(p.X, p.Y, p.Z, u_ref, 6.1, 0.1)
    assert info["rel_residual"] <= 1e-12
    assert gc.rel_err(uv, uv_ref) < 1e-8
    # the solve changed the wind: the read-out is not the interpolated wind's
    uv0 = coupling.surface_wind(p.X, p.Y, p.Z, u0_ref, 6.1, 0.1)
    assert gc.rel_err(uv0, uv_ref) > 1e-3
