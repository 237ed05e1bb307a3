"""Kernel-by-kernel parity of the HIP path (through the C ABI) with the FP64
oracle: stiffness apply, right-hand side, recovery, divergence, stencils,
hierarchy, Galerkin operators, smoother, residual, transfers, coarsest solve
and one V-cycle."""
import numpy as np
import pytest
import torch

from oracle import fem, multigrid as mg
from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grid(name, **kw):
    from paper_2101_08453_amd import mcwind
    print(f"[case] {name} {kw}", flush=True)
    return mcwind.grid_from_problem(gc.problem(name), **kw)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


@pytest.mark.parametrize("name", gc.CASES)
def test_apply_K_matches_assembled_stiffness(name):
    g, _ = _grid(name)
    p = gc.problem(name)
    x = np.random.default_rng(1).standard_normal(p.X.shape)
    y = g.apply_K(_dev(x)).cpu().numpy().ravel()
    ref = gc.system(name).K_full @ x.ravel()
    assert gc.rel_err(y, ref) < 1e-13


@pytest.mark.parametrize("name", gc.CASES)
def test_rhs_matches_one_point_quadrature(name):
    g, u0 = _grid(name)
    S = gc.system(name)
    f = g.rhs(u0).cpu().numpy().ravel()
    ref = np.where(S.mask, S.f_full, 0.0)
    assert gc.rel_err(f, ref) < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("name", gc.CASES)
def test_solve_recovers_the_wind_as_the_recovery_entry_point(name, precision):
    """The solve recovers u in its divergence-check launch: the same bits as
    mcw_recover on the solve's lambda, and the same divergence as
    mcw_divergence."""
    g, u0 = _grid(name, precision=precision, rtol=1e-10)
    lam, u, info = g.solve(u0)
    assert info["status"] == "MCW_OK"
    assert torch.equal(u, g.recover(u0, lam))
    _, rel = g.divergence(u0, lam)
    assert rel == info["rel_divergence"]


@pytest.mark.parametrize("name", gc.CASES)
def test_recovery_and_divergence(name):
    g, u0 = _grid(name)
    p = gc.problem(name)
    lam = np.random.default_rng(2).standard_normal(p.X.shape) * gc.free_mask(p)
    u = g.recover(u0, _dev(lam)).cpu().numpy()
    assert gc.rel_err(u, fem.recover(p.X, p.Y, p.Z, p.u0, p.a, lam)) < 1e-13
    D, rel = g.divergence(u0, _dev(lam))
    Dref, D0 = fem.weak_divergence(p.X, p.Y, p.Z, p.u0, p.a, lam)
    m = gc.free_mask(p).ravel()
    assert gc.rel_err(D.cpu().numpy().ravel(), np.where(m, Dref, 0.0)) < 1e-12
    assert abs(rel - np.linalg.norm(Dref[m]) / np.linalg.norm(D0[m])) < 1e-12 * rel


@pytest.mark.parametrize("name", gc.CASES)
def test_fine_stencil_matches_assembly(name):
    g, _ = _grid(name, precision="fp64")
    nx, ny, nz = gc.problem(name).dims
    st = g.stencil(0, "fp64").cpu().numpy()
    ref = mg.stencil_array(gc.system(name).K_full, nx, ny, nz)
    assert gc.rel_err(st, ref) < 1e-13


@pytest.mark.parametrize("name", gc.CASES)
@pytest.mark.parametrize("rule", ["operator", "literal", "full", "operator:coarsened"])
def test_hierarchy_and_galerkin_operators(name, rule):
    cmax = 60
    rule, _, spacing = rule.partition(":")
    spacing = spacing or "level"
    g, _ = _grid(name, precision="fp64", coarse_direct_max=cmax, coarsen_rule=rule,
                 merge_spacing=spacing)
    levels = gc.hierarchy(name, coarse_max=cmax, rule=rule, spacing=spacing)
    assert g.num_levels() == len(levels)
    for l, L in enumerate(levels):
        info = g.level(l)
        assert info["dims"] == L.dims
        if l + 1 < len(levels):
            assert info["coarsen_h"] == bool(L.coarsen_h)
            assert info["keep_z"] == list(L.keep_z)
        st = g.stencil(l, "fp64").cpu().numpy()
        ref = mg.stencil_array(L.K_full, *L.dims)
        assert gc.rel_err(st, ref) < 1e-12, f"level {l}"


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_fp32_stencils_round_off_diagonals_and_keep_row_sums(name):
    """The FP32 operator: off-diagonals rounded once from FP64, except the
    coupling to the node below (o = 4), which is the node below's rounded
    coupling to the node above (o = 22; zero on the bottom plane), so the
    column coupling is symmetric; the diagonal is minus the off-diagonal sum
    (FP64 sum, rounded once)."""
    g64, _ = _grid(name, precision="fp64", coarse_direct_max=60)
    g32, _ = _grid(name, precision="fp32_refine", coarse_direct_max=60)
    for l in range(g64.num_levels()):
        s64 = g64.stencil(l, "fp64").cpu().numpy()
        s32 = g32.stencil(l, "fp32_refine").cpu().numpy()
        stored = np.ones(27, dtype=bool)
        stored[[4, 13]] = False
        assert np.array_equal(s32[stored], s64[stored].astype(np.float32)), f"level {l}"
        want4 = np.zeros_like(s32[4])
        want4[1:] = s32[22][:-1]
        assert np.array_equal(s32[4], want4), f"level {l}"
        # K is symmetric, so this is the rounding of its own o = 4 entry up to
        # the FP64 assembly's last bits
        assert np.allclose(s32[4], s64[4], rtol=2.0 ** -23, atol=0.0), f"level {l}"
        off = np.ones(27, dtype=bool)
        off[13] = False
        diag = (-s32[off].astype(np.float64).sum(axis=0)).astype(np.float32)
        assert np.array_equal(s32[13], diag)


def _level_vectors(p, L, seed):
    rng = np.random.default_rng(seed)
    m = L.mask.reshape(L.nz + 1, L.ny + 1, L.nx + 1)
    return rng.standard_normal(m.shape) * m, rng.standard_normal(m.shape) * m, m


@pytest.mark.parametrize("name", gc.CASES)
def test_gauss_seidel_sweep_matches_sequential_order(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60)
    levels = gc.hierarchy(name, coarse_max=60)
    for l in range(min(2, len(levels))):
        L = levels[l]
        x, f, _ = _level_vectors(gc.problem(name), L, 10 + l)
        xg = _dev(x)
        g.smooth(l, xg, _dev(f), sweeps=1)
        ref = mg.gs_sweep_full(L.K_full, L.mask, L.dims, x.ravel(), f.ravel())
        assert gc.rel_err(xg.cpu().numpy().ravel(), ref) < 1e-12, f"level {l}"


@pytest.mark.parametrize("name", gc.CASES)
def test_residual_and_transfers(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60)
    levels = gc.hierarchy(name, coarse_max=60)
    assert len(levels) >= 2
    L, C = levels[0], levels[1]
    x, f, m = _level_vectors(gc.problem(name), L, 3)
    r = g.residual(0, _dev(x), _dev(f)).cpu().numpy().ravel()
    rref = np.where(L.mask, f.ravel() - L.K_full @ x.ravel(), 0.0)
    assert gc.rel_err(r, rref) < 1e-13
    rc = g.restrict(0, _dev(r.reshape(x.shape))).cpu().numpy().ravel()
    rcref = np.where(C.mask, L.P_full.T @ r, 0.0)
    assert gc.rel_err(rc, rcref) < 1e-14
    e = np.random.default_rng(4).standard_normal(C.mask.size) * C.mask
    xg = _dev(x)
    g.prolong(0, _dev(e.reshape(C.nz + 1, C.ny + 1, C.nx + 1)), xg)
    assert gc.rel_err(xg.cpu().numpy().ravel(), x.ravel() + L.P_full @ e) < 1e-14
    # transposition: <P e, r> = <e, P^T r> with the GPU's two operators
    Pe = xg.cpu().numpy().ravel() - x.ravel()
    assert abs(Pe @ r - e @ rc) < 1e-12 * abs(e @ rc)


@pytest.mark.parametrize("name", gc.CASES)
def test_coarsest_direct_solve(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60)
    levels = gc.hierarchy(name, coarse_max=60)
    L = levels[-1]
    r = np.random.default_rng(5).standard_normal(L.mask.size) * L.mask
    e = g.coarse_solve(_dev(r.reshape(L.nz + 1, L.ny + 1, L.nx + 1))).cpu().numpy().ravel()
    ref = np.zeros_like(r)
    ref[L.free] = np.linalg.solve(L.K.toarray(), r[L.free])
    assert gc.rel_err(e, ref) < 1e-11


@pytest.mark.parametrize("name", gc.CASES)
def test_vcycle_matches_oracle_vcycle(name):
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60)
    levels = gc.hierarchy(name, coarse_max=60)
    M = mg.Multigrid(levels)
    L = levels[0]
    x, f, _ = _level_vectors(gc.problem(name), L, 6)
    xg = _dev(x)
    g.vcycle(xg, _dev(f))
    ref = M.vcycle(x.ravel()[L.free], f.ravel()[L.free])
    assert gc.rel_err(xg.cpu().numpy().ravel()[L.free], ref) < 1e-10


@pytest.mark.parametrize("shape", [0, 1, 4])
def test_vcycle_matches_oracle_with_every_pass_shape(shape, tmp_path, monkeypatch):
    """The last pre-smoothing sweep leaves the odd rows' residual both in the
    two-colour launch (shape 0) and after the one-colour passes (1 or 4 rows of
    64 columns per block).  On a 130x100x6 hills grid whose fine level (92 K
    nodes) is forced to each shape through the tuning cache, one FP64 V-cycle
    against the oracle's."""
    from paper_2101_08453_amd import inputs, mcwind
    p = inputs.hills_problem(130, 100, 6, 3, 7, a=(1.0, 1.0, 3.0))
    shp = f"{p.dims[0] + 1}x{p.dims[1] + 1}x{p.dims[2] + 1}"
    cache = tmp_path / "tune.json"
    cache.write_text('{\n  "gfx950|gsf|%s|f64": %d,\n  "gfx950|res|%s|f64": 4\n}\n' % (shp, shape, shp))
    monkeypatch.setenv("MCW_TUNE_CACHE", str(cache))
    print(f"[case] V-cycle, fine pass shape {shape}", flush=True)
    g, _ = mcwind.grid_from_problem(p, precision="fp64", coarse_direct_max=60)
    assert g.tile_rows(0)[0] == shape
    levels = mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=60)
    assert [lv.dims for lv in levels] == [tuple(int(v) - 1 for v in g.level_shape(l)[::-1])
                                          for l in range(g.num_levels())]
    M = mg.Multigrid(levels)
    L = levels[0]
    x, f, _ = _level_vectors(p, L, 23)
    xg = _dev(x)
    g.vcycle(xg, _dev(f))
    ref = M.vcycle(x.ravel()[L.free], f.ravel()[L.free])
    assert gc.rel_err(xg.cpu().numpy().ravel()[L.free], ref) < 1e-10


@pytest.mark.parametrize("nu", [(0, 2), (1, 1), (3, 2)])
@pytest.mark.parametrize("smoother", ["point", "line"])
@pytest.mark.parametrize("name", ["ragged", "tiles"])
def test_vcycle_with_other_smoothing_counts(name, smoother, nu):
    """The last colour pass of the last pre-smoothing sweep writes its columns'
    residual and the residual kernel skips them; with no pre-smoothing the
    residual kernel computes every column.  Each count and smoother against
    the oracle's V-cycle (Sec. 3) of the same counts."""
    g, _ = _grid(name, precision="fp64", coarse_direct_max=60, smoother=smoother,
                 nu_pre=nu[0], nu_post=nu[1])
    levels = gc.hierarchy(name, coarse_max=60)
    M = mg.Multigrid(levels, nu_pre=nu[0], nu_post=nu[1], smoother=smoother)
    L = levels[0]
    x, f, _ = _level_vectors(gc.problem(name), L, 17)
    xg = _dev(x)
    g.vcycle(xg, _dev(f))
    ref = M.vcycle(x.ravel()[L.free], f.ravel()[L.free])
    assert gc.rel_err(xg.cpu().numpy().ravel()[L.free], ref) < 1e-10


def test_inverted_element_is_rejected():
    from paper_2101_08453_amd import mcwind
    p = gc.make("box")
    Z = p.Z.copy()
    Z[3, 5, 6] = Z[4, 5, 6] + 3.0  # node pushed far above the one over it
    assert fem.min_detJ(p.X, p.Y, Z).min() <= 0.0  # the geometry really is invalid
    with pytest.raises(mcwind.MCWError) as ei:
        mcwind.Grid(_dev(p.X), _dev(p.Y), _dev(Z), p.a)
    assert ei.value.status_name == "MCW_BAD_GEOMETRY"
    bad = np.flatnonzero(fem.min_detJ(p.X, p.Y, Z) <= 0.0)[0]
    nx, ny, _ = p.dims
    assert f"element ({bad % nx}, {(bad // nx) % ny}, {bad // (nx * ny)})" in str(ei.value)


def test_element_inverted_only_at_a_gauss_point_is_rejected():
    """A node pushed towards the opposite corner of the element below it, by
    0.8 of that element's edges: det J <= 0 at the Gauss point nearest the
    node but > 0 at the element centre (closed form in the oracle's pin), so
    only the Gauss-point part of the check can reject the grid."""
    from paper_2101_08453_amd import mcwind
    p = gc.make("box")
    X, Y, Z = p.X.copy(), p.Y.copy(), p.Z.copy()
    i, j, k = 7, 6, 4  # node (i, j, k) is corner 7 of element (i-1, j-1, k-1)
    t = 0.8
    X[k, j, i] -= t * (X[k, j, i] - X[k, j, i - 1])
    Y[k, j, i] -= t * (Y[k, j, i] - Y[k, j - 1, i])
    Z[k, j, i] -= t * (Z[k, j, i] - Z[k - 1, j, i])
    dmin = fem.min_detJ(X, Y, Z)
    bad = int(np.flatnonzero(dmin <= 0.0)[0])
    nx, ny, nz = p.dims
    xe = fem.element_coords(X, Y, Z, fem.element_node_ids(nx, ny, nz))
    assert np.linalg.det(fem.jacobian(xe, fem.CENTRE)).min() > 0.0  # every centre is fine
    with pytest.raises(mcwind.MCWError) as ei:
        mcwind.Grid(_dev(X), _dev(Y), _dev(Z), p.a)
    assert ei.value.status_name == "MCW_BAD_GEOMETRY"
    assert f"element ({bad % nx}, {(bad // nx) % ny}, {bad // (nx * ny)})" in str(ei.value)


@pytest.mark.parametrize("name,terrain", [("ragged", True), ("tiles", True), ("distorted", False)])
def test_terrain_following_grids_take_the_short_element_path(name, terrain, capfd):
    """Grids whose node x depends on i only and y on j only use the element
    kernels' terrain-following path; others the general one.  Both match the
    assembled stiffness, the right-hand side and the divergence identity."""
    g, u0 = _grid(name, precision="fp64", verbose=True)
    err = capfd.readouterr().err
    assert f"terrain-following grid: {'yes' if terrain else 'no'}" in err
    p = gc.problem(name)
    x = np.random.default_rng(11).standard_normal(p.X.shape)
    y = g.apply_K(_dev(x)).cpu().numpy().ravel()
    assert gc.rel_err(y, gc.system(name).K_full @ x.ravel()) < 1e-13
    f = g.rhs(u0).cpu().numpy().ravel()
    S = gc.system(name)
    assert gc.rel_err(f, np.where(S.mask, S.f_full, 0.0)) < 1e-13
    lam, _, _ = g.solve(u0)
    D, rel = g.divergence(u0, lam)
    r = (g.rhs(u0) - g.apply_K(lam)).cpu().numpy()
    m = gc.free_mask(p)
    assert np.abs(D.cpu().numpy() + np.where(m, r, 0.0)).max() <= 1e-12 * np.abs(f).max()
