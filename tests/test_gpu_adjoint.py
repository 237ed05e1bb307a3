"""Adjoint of the solve (transpose multigrid solve with the same SPD operator
plus the adjoints of recovery and right-hand side) through
torch.autograd.Function, checked against the FP64 oracle's gradient and
against central finite differences of the GPU forward solve."""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from paper_2101_08453_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mcw():
    from paper_2101_08453_amd import mcwind
    return mcwind


def _loss(u, mask_t):
    return (u[0, 0][mask_t] ** 2).sum() + (u[1, 0][mask_t] ** 2).sum()


def _grad_gpu(p, mask, rtol=1e-12, **kw):
    mcwind = _mcw()
    g, u0 = mcwind.grid_from_problem(p, rtol=rtol, **kw)
    u0 = u0.clone().requires_grad_(True)
    a = torch.tensor(p.a, dtype=torch.float64, device="cuda", requires_grad=True)
    u = mcwind.WindSolve.apply(u0, a, g)
    mask_t = torch.from_numpy(mask).cuda()
    L = _loss(u, mask_t)
    L.backward()
    return g, float(L), u0.grad.cpu().numpy(), a.grad.cpu().numpy()


def _small():
    p = inputs.fractal_problem(24, 20, 6, 120.0, seed=21, a=(1.0, 1.3, 2.0))
    mask = inputs.fire_mask(24, 20, seed=55)
    mask |= inputs.fire_mask(24, 20, seed=57)
    assert mask.sum() > 10
    return p, mask


def test_gradient_matches_oracle():
    p, mask = _small()
    _, L, g_u0, g_a = _grad_gpu(p, mask)
    L_ref, g_u0_ref, g_a_ref = oadj.gradient(p, mask)
    assert abs(L - L_ref) <= 1e-10 * abs(L_ref)
    # dL/du0 is returned in FP32
    assert np.abs(g_u0 - g_u0_ref).max() <= 1e-5 * np.abs(g_u0_ref).max()
    assert np.allclose(g_a, g_a_ref, rtol=1e-8, atol=1e-10 * np.abs(g_a_ref).max())


@pytest.mark.parametrize("kw", [dict(krylov=True), dict(smoother="line"),
                                dict(precision="fp64", krylov=True, smoother="line")])
def test_gradient_with_solver_variants_matches_oracle(kw):
    """The transpose solve runs through the handle's own solver: CG, the line
    smoother and plain FP64 give the same gradient."""
    p, mask = _small()
    _, L, g_u0, g_a = _grad_gpu(p, mask, **kw)
    L_ref, g_u0_ref, g_a_ref = oadj.gradient(p, mask)
    assert abs(L - L_ref) <= 1e-10 * abs(L_ref)
    assert np.abs(g_u0 - g_u0_ref).max() <= 1e-5 * np.abs(g_u0_ref).max()
    assert np.allclose(g_a, g_a_ref, rtol=1e-8, atol=1e-10 * np.abs(g_a_ref).max())


def test_gradient_matches_central_differences_of_gpu_forward():
    """L is exactly quadratic in u0, so central differences along u0 are exact
    up to the solve tolerance; along a they are O(h^2)."""
    mcwind = _mcw()
    p, mask = _small()
    g, L, g_u0, g_a = _grad_gpu(p, mask)
    mask_t = torch.from_numpy(mask).cuda()
    u0 = torch.from_numpy(p.u0).cuda()

    def loss_u0(v):
        _, u, _ = g.solve(v)
        return float(_loss(u, mask_t))

    h = 1e-4
    for d in inputs.random_directions(p.u0.shape, 6, seed=56):
        dt = torch.from_numpy(d).cuda()
        fd = (loss_u0(u0 + h * dt) - loss_u0(u0 - h * dt)) / (2 * h)
        an = float(np.sum(g_u0.astype(np.float64) * d))
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-7 * L

    def loss_a(a):
        q = inputs.Problem("a", p.X, p.Y, p.Z, p.u0, np.asarray(a), p.gamma)
        gg, uu = mcwind.grid_from_problem(q, rtol=1e-12)
        _, u, _ = gg.solve(uu)
        return float(_loss(u, mask_t))

    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (loss_a(p.a + e) - loss_a(p.a - e)) / (2 * h)
        assert abs(fd - g_a[d]) <= 1e-6 * np.abs(g_a).max()


def test_adjoint_dot_product_identity():
    """<g_u, du/du0 . v> = <dL/du0, v> for the linear map u0 -> u (L = <g_u, u>)."""
    mcwind = _mcw()
    p, _ = _small()
    g, u0 = mcwind.grid_from_problem(p, rtol=1e-13, precision="fp64")
    rng = np.random.default_rng(9)
    gu = torch.from_numpy(rng.standard_normal(g.elem_shape)).cuda()
    v = torch.from_numpy(rng.standard_normal(g.elem_shape)).cuda()
    lam_v, u_v, _ = g.solve(v)
    lam0 = torch.zeros(g.node_shape, dtype=torch.float64, device="cuda")
    d_u0, _, _ = g.adjoint(lam0, gu)
    lhs = float((gu * u_v).sum())
    rhs = float((d_u0.double() * v).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_c5_size_gradient_finite_differences():
    """512x512x15 fractal terrain (500 m relief), elliptical fire mask: the
    adjoint gradient against central differences along 20 random u0 directions
    and the three penalty axes."""
    mcwind = _mcw()
    p = inputs.c5()
    mask = inputs.fire_mask(512, 512, seed=55)
    g, L, g_u0, g_a = _grad_gpu(p, mask, rtol=1e-12)
    mask_t = torch.from_numpy(mask).cuda()
    u0 = torch.from_numpy(p.u0).cuda()
    h = 1e-4
    dirs = inputs.random_directions(p.u0.shape, 20, seed=56)
    errs = []
    for d in dirs:
        dt = torch.from_numpy(d).cuda()
        lp = float(_loss(g.solve(u0 + h * dt)[1], mask_t))
        lm = float(_loss(g.solve(u0 - h * dt)[1], mask_t))
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(g_u0.astype(np.float64) * d))
        errs.append(abs(fd - an) / max(abs(an), 1e-30))
    print(f"[c5] L={L:.6e} median rel err {np.median(errs):.2e} max {max(errs):.2e}")
    assert np.median(errs) < 1e-4 and max(errs) < 1e-3
    for dd in range(3):
        e = np.zeros(3)
        e[dd] = h
        vals = []
        for s in (1.0, -1.0):
            q = inputs.Problem("a", p.X, p.Y, p.Z, p.u0, p.a + s * e, p.gamma)
            gg, uu = mcwind.grid_from_problem(q, rtol=1e-12)
            vals.append(float(_loss(gg.solve(uu)[1], mask_t)))
            gg.close()
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g_a[dd]) <= 1e-5 * np.abs(g_a).max()


def test_c5_size_gradient_against_the_oracle():
    """512x512x15 fractal terrain (500 m relief), elliptical fire mask: the
    adjoint's loss, dL/da and the directional derivatives <dL/du0, d> along 20
    seeded directions against the FP64 oracle's (tests/golden/c5_gradient.txt,
    written by the oracle alone), at 1e-6 relative.  L is quadratic in u0 and
    the solves run to 1e-12, so only the FP32 output of dL/du0 and the
    reduction orders separate the two."""
    from tests import golden_cases as gold
    ref = gold.c5_gradient()
    assert len(ref["directional"]) == 20
    p = inputs.c5()
    mask = inputs.fire_mask(512, 512, seed=55)
    print("[case] c5 gradient against the oracle's", flush=True)
    _, L, g_u0, g_a = _grad_gpu(p, mask, rtol=1e-12)
    assert abs(L - ref["loss"]) <= 1e-9 * abs(ref["loss"])
    assert np.allclose(g_a, ref["dL_da"], rtol=1e-6, atol=1e-9 * np.abs(ref["dL_da"]).max())
    dirs = inputs.random_directions(p.u0.shape, 20, seed=56)
    got = np.array([float(np.sum(g_u0.astype(np.float64) * d)) for d in dirs])
    want = np.array(ref["directional"])
    err = np.abs(got - want) / np.abs(want).max()
    print(f"[c5] directional derivatives: max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 1e-6


def test_penalties_other_than_the_grids_are_rejected():
    """dL/da is the derivative at the grid's own penalties; a different a would
    silently get that gradient, so WindSolve refuses it."""
    mcwind = _mcw()
    p, _ = _small()
    print("[case] WindSolve with mismatched a", flush=True)
    g, u0 = mcwind.grid_from_problem(p)
    a = torch.tensor([1.0, 1.3, 2.5], dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(ValueError, match="penalties"):
        mcwind.WindSolve.apply(u0, a, g)
