"""The FP16-stencil option of the FP32 V-cycle (stencil_fp16): the stored
coefficients are the FP64 Galerkin stencils divided by a per-level power of two
and rounded to FP16; the V-cycle computes in FP32 and the
refinement in FP64, so solutions meet the same tolerance and match the oracle.
Also: the fused colour pass equals the four separate passes bit for bit, batches
mix FP16 and FP32 members, and the 3000x3000x15 solve reaches 1e-8."""
import numpy as np
import pytest
import torch

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


@pytest.mark.parametrize("name", gc.CASES)
def test_fp16_stencils_are_the_rounded_galerkin_stencils(name):
    """Every level: off-diagonals = fp16(a / s) * s, rounded once from FP64, with
    s = 2^(floor(log2 max|a|) + 1), and zero where |a / s| < 2^-14 (below the FP16
    normal range); the coupling to the node below (o = 4) is the node below's
    coupling to the node above (o = 22; zero on the bottom plane); the diagonal
    minus their sum (FP64 sum, rounded once)."""
    mcwind = _mcw()
    p = gc.problem(name)
    print(f"[case] fp16 stencil {name}", flush=True)
    g16, _ = mcwind.grid_from_problem(p, stencil_fp16=True, coarse_direct_max=60)
    g64, _ = mcwind.grid_from_problem(p, precision="fp64", coarse_direct_max=60)
    assert g16.num_levels() == g64.num_levels()
    off = np.array([o != 13 for o in range(27)])
    for l in range(g16.num_levels()):
        s64 = g64.stencil(l, "fp64").cpu().numpy().reshape(27, -1)
        s16 = g16.stencil(l).cpu().numpy().reshape(27, -1)
        amax = np.abs(s64[off]).max()
        s = 2.0 ** (np.floor(np.log2(amax)) + 1)
        v = s64[off] / s
        v = np.where(np.abs(v) < 2.0 ** -14, 0.0, v)
        want = v.astype(np.float16).astype(np.float32) * np.float32(s)
        # o = 4 is row 4 of the off-diagonal rows: the o = 22 row (row 21) one plane down
        nxy = g16.level_shape(l)[1] * g16.level_shape(l)[2]
        want[4] = 0.0
        want[4, nxy:] = want[21, :-nxy]
        assert np.array_equal(s16[off], want), f"level {l}"
        diag = (-(want / np.float32(s)).astype(np.float64).sum(axis=0)).astype(np.float32) * np.float32(s)
        assert np.array_equal(s16[13], diag), f"level {l}"


@pytest.mark.parametrize("krylov", [False, True])
@pytest.mark.parametrize("name", gc.CASES)
def test_solution_with_fp16_stencils_matches_oracle(name, krylov):
    mcwind = _mcw()
    p = gc.problem(name)
    lam_ref, u_ref, _ = gc.solution(name)
    print(f"[case] fp16 solve {name} krylov {krylov}", flush=True)
    g, u0 = mcwind.grid_from_problem(p, stencil_fp16=True, krylov=krylov, rtol=1e-12)
    lam, u, info = g.solve(u0)
    assert info["status"] == "MCW_OK" and info["rel_residual"] <= 1e-12
    assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8
    assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8
    assert info["rel_divergence"] < 1e-10


def test_line_smoother_with_fp16_stencils_matches_oracle():
    mcwind = _mcw()
    p = gc.problem("ragged")
    lam_ref, _, _ = gc.solution("ragged")
    g, u0 = mcwind.grid_from_problem(p, stencil_fp16=True, smoother="line", rtol=1e-12)
    lam, _, info = g.solve(u0)
    assert info["status"] == "MCW_OK" and info["rel_residual"] <= 1e-12
    assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8


@pytest.mark.parametrize("dims", [(160, 120, 8), (2100, 5, 5)])
@pytest.mark.parametrize("smoother", ["point", "line"])
def test_fused_fp16_pass_equals_four_separate_passes(tmp_path, monkeypatch, smoother, dims):
    mcwind = _mcw()
    nx, ny, nz = dims
    p = inputs.hills_problem(nx, ny, nz, 4, 5, a=(1.0, 1.0, 2.0))
    key = "gsf" if smoother == "point" else "gsl"
    shp = f"{nx + 1}x{ny + 1}x{nz + 1}"
    grids = []
    for shape in (0, 4):
        cache = tmp_path / f"tune{shape}.json"
        cache.write_text('{\n  "gfx950|%s|%s|h16": %d,\n  "gfx950|res|%s|h16": 4\n}\n'
                         % (key, shp, shape, shp))
        monkeypatch.setenv("MCW_TUNE_CACHE", str(cache))
        g, u0 = mcwind.grid_from_problem(p, stencil_fp16=True, krylov=True, smoother=smoother)
        assert g.tile_rows(0)[0] == shape
        grids.append(g)
    rng = np.random.default_rng(3)
    x0 = torch.from_numpy(rng.standard_normal((nz + 1, ny + 1, nx + 1))).to("cuda", torch.float32)
    f = torch.from_numpy(rng.standard_normal((nz + 1, ny + 1, nx + 1))).to("cuda", torch.float32)
    out = []
    for g in grids:
        x = x0.clone()
        g.smooth(0, x, f, sweeps=2)
        g.smooth(0, x, f, sweeps=-1)
        r = g.residual(0, x, f)
        lam, _, _ = g.solve(u0, want_u=False)
        out.append((x, r, lam))
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert torch.equal(a, b)


def test_batch_mixes_fp16_and_fp32_members():
    mcwind = _mcw()
    names = ["c1", "ragged", "tiles", "box"]
    grids, u0s, refs = [], [], []
    for m, name in enumerate(names):
        p = gc.problem(name)
        g, u0 = mcwind.grid_from_problem(p, stencil_fp16=bool(m % 2), rtol=1e-12)
        grids.append(g)
        u0s.append(u0)
        refs.append(gc.solution(name)[0])
    for krylov in (False, True):
        if krylov:
            grids = [mcwind.grid_from_problem(gc.problem(n), stencil_fp16=bool(m % 2), krylov=True,
                                              rtol=1e-12)[0] for m, n in enumerate(names)]
        print(f"[case] fp16 batch krylov {krylov}", flush=True)
        lams, _, infos, st = mcwind.solve_batch(grids, u0s)
        assert st == "MCW_OK"
        for lam, info, ref in zip(lams, infos, refs):
            assert info["rel_residual"] <= 1e-12
            assert gc.rel_err(lam.cpu().numpy(), ref) < 1e-8
        if krylov:
            # batched CG takes each member's own steps with the single kernels'
            # arithmetic, whichever stencil format the member has
            for g, u0, lam in zip(grids, u0s, lams):
                lam1, _, _ = g.solve(u0.clone(), want_u=False)
                assert torch.equal(lam, lam1)


def test_3000x3000x15_warm_solve_with_fp16_stencils():
    """The benchmark's warm-started solve with FP16 stencils reaches 1e-8 (FP64
    residual) and gives the FP32-stencil lambda to within what the tolerance allows."""
    mcwind = _mcw()
    p = inputs.c3()
    du = inputs.c3_perturbation(p.u0.shape)
    print("[case] 3000x3000x15 warm solve, FP16 stencils", flush=True)
    dev = torch.device("cuda")
    XYZ = [torch.from_numpy(A).to(dev) for A in (p.X, p.Y, p.Z)]
    u0 = torch.from_numpy(p.u0).to(dev)
    u0p = u0 + torch.from_numpy(du).to(dev)
    lams = []
    for fp16 in (False, True):
        g = mcwind.Grid(*XYZ, p.a, rtol=1e-10, stencil_fp16=fp16)
        lam, _, _ = g.solve(u0, want_u=False)
        g.set_tolerance(1e-8)
        lam, _, info = g.solve(u0p, lam=lam, want_u=False)
        assert info["status"] == "MCW_OK" and info["rel_residual"] <= 1e-8
        assert abs(info["rel_divergence"] - info["rel_residual"]) <= 1e-6 * info["rel_residual"]
        lams.append(lam)
        g.close()
        del g
    diff = float((lams[0] - lams[1]).abs().max() / lams[0].abs().max())
    print(f"[case] lambda fp16 vs fp32 stencils: {diff:.2e}", flush=True)
    assert diff < 1e-5


@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("scale", [1e-3, 1e3])
def test_coordinate_scaling_with_either_stencil_format(scale, fp16):
    """Coordinates times s: K scales by s, f by s^2, so lambda by s and u is
    unchanged; the per-level power-of-two scale keeps FP16 stencils (and the
    scaled residual keeps FP32 V-cycles) indifferent to the magnitudes."""
    mcwind = _mcw()
    p = gc.problem("ragged")
    lam_ref, u_ref, _ = gc.solution("ragged")
    print(f"[case] scaled coordinates s={scale} fp16={fp16}", flush=True)
    dev = torch.device("cuda")
    X, Y, Z = (torch.from_numpy(A * scale).to(dev) for A in (p.X, p.Y, p.Z))
    u0 = torch.from_numpy(p.u0).to(dev)
    g = mcwind.Grid(X, Y, Z, p.a, gamma=p.gamma, rtol=1e-12, stencil_fp16=fp16)
    lam, u, info = g.solve(u0)
    assert info["status"] == "MCW_OK" and info["rel_residual"] <= 1e-12
    assert gc.rel_err(lam.cpu().numpy() / scale, lam_ref) < 1e-8
    assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8


@pytest.mark.parametrize("name", gc.CASES)
def test_cg_with_line_smoother_and_fp16_stencils_matches_oracle(name):
    """The three options together (CG preconditioned by the symmetric V-cycle,
    vertical line smoother, FP16 stencils) reach the oracle's solution."""
    mcwind = _mcw()
    p = gc.problem(name)
    lam_ref, u_ref, _ = gc.solution(name)
    print(f"[case] cg + line + fp16 {name}", flush=True)
    g, u0 = mcwind.grid_from_problem(p, krylov=True, smoother="line", stencil_fp16=True, rtol=1e-12)
    lam, u, info = g.solve(u0)
    assert info["status"] == "MCW_OK" and info["rel_residual"] <= 1e-12
    assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8
    assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8
