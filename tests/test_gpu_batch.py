"""Batched solves (mcw_solve_batch): members of uneven sizes, depths and
penalties advanced together by persistent batched kernels and a captured
batched V-cycle, checked against the FP64 oracle and against single solves."""
import numpy as np
import pytest
import torch

from oracle import solve as osolve
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


def _members():
    return [
        inputs.hills_problem(40, 36, 8, 3, 401, a=(1.0, 1.0, 4.0)),
        inputs.hills_problem(70, 70, 12, 5, 402, a=(1.0, 1.0, 1.0)),
        inputs.fractal_problem(33, 47, 16, 90.0, 403, a=(1.0, 1.0, 9.0)),
        gc.make("distorted"),
        inputs.box_problem(9, 7, 3, seed=3),
    ]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_oracle(use_graph):
    mcwind = _mcw()
    probs = _members()
    print(f"[case] batch of {len(probs)} use_graph={use_graph}", flush=True)
    grids, u0s = zip(*[mcwind.grid_from_problem(p, rtol=1e-12, use_graph=use_graph) for p in probs])
    lams, us, infos, status = mcwind.solve_batch(list(grids), list(u0s))
    assert status == "MCW_OK"
    for p, lam, u, info in zip(probs, lams, us, infos):
        lam_ref, u_ref, _ = osolve.solve(p, rtol=1e-14)
        assert info["rel_residual"] <= 1e-12
        assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8
        assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8
        assert info["rel_divergence"] < 1e-10


def test_batch_equals_single_solves_and_isolates_failures():
    mcwind = _mcw()
    probs = _members()[:3]
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p) for p in probs])]
    # a zero-wind member and a non-finite member ride along
    gz, uz = mcwind.grid_from_problem(gc.make("box"))
    uz = torch.zeros_like(uz)
    gn, un = mcwind.grid_from_problem(inputs.hills_problem(20, 20, 6, 2, 9))
    un[1, 2, 3, 4] = float("nan")
    lams, us, infos, status = mcwind.solve_batch(grids + [gz, gn], u0s + [uz, un], check=False)
    assert status == "MCW_NONFINITE"
    assert [i["status"] for i in infos] == ["MCW_OK"] * 4 + ["MCW_NONFINITE"]
    for i, g in enumerate(grids):
        lam1, _, _ = g.solve(u0s[i].clone())
        assert infos[i]["rel_residual"] <= 1e-8
        assert float((lams[i] - lam1).abs().max() / lam1.abs().max()) < 1e-6
    assert float(lams[3].abs().max()) == 0.0 and torch.equal(us[3], uz)
    assert infos[3]["rel_residual"] == 0.0
    ok = ~torch.isnan(un)
    assert torch.equal(us[4][ok], un[ok])


def test_batch_of_ensemble_members_against_fp64_solves():
    """Eight members of the 64-member ensemble (64^2..512^2 x 8..16, a3 in [1,10])."""
    mcwind = _mcw()
    probs = [inputs.c4_member(m) for m in range(8)]
    g32, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p) for p in probs])]
    lams, us, infos, status = mcwind.solve_batch(g32, u0s)
    assert status == "MCW_OK"
    for p, g, u0, lam, info in zip(probs, g32, u0s, lams, infos):
        assert info["rel_residual"] <= 1e-8
        g64 = mcwind.Grid(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.Y).cuda(),
                          torch.from_numpy(p.Z).cuda(), p.a, precision="fp64", rtol=1e-12)
        lam64, _, _ = g64.solve(u0)
        err = float((lam - lam64).abs().max() / lam64.abs().max())
        print(f"[c4] {p.name}: cycles {info['cycles']} rel err vs fp64 {err:.2e}")
        assert err < 1e-5
        g64.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_cg_matches_oracle_and_single_cg(use_graph):
    """Members of uneven sizes and depths advanced together by batched CG (one
    symmetric V-cycle per step); each member stops on its own residual."""
    mcwind = _mcw()
    probs = _members()
    print(f"[case] batched CG of {len(probs)} use_graph={use_graph}", flush=True)
    grids, u0s = zip(*[mcwind.grid_from_problem(p, rtol=1e-12, krylov=True, use_graph=use_graph)
                       for p in probs])
    lams, us, infos, status = mcwind.solve_batch(list(grids), list(u0s))
    assert status == "MCW_OK"
    for p, g, u0, lam, u, info in zip(probs, grids, u0s, lams, us, infos):
        lam_ref, u_ref, _ = osolve.solve(p, rtol=1e-14)
        assert info["rel_residual"] <= 1e-12
        assert gc.rel_err(lam.cpu().numpy(), lam_ref) < 1e-8
        assert gc.rel_err(u.cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8
        lam1, _, info1 = g.solve(u0.clone(), want_u=False)
        assert float((lam - lam1).abs().max() / lam1.abs().max()) < 1e-9
        print(f"[cg] {p.name}: batched {info['cycles']} steps, single {info1['cycles']}", flush=True)


def test_batched_cg_isolates_a_non_finite_member():
    mcwind = _mcw()
    probs = _members()[:2]
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p, krylov=True) for p in probs])]
    gn, un = mcwind.grid_from_problem(inputs.hills_problem(20, 20, 6, 2, 9), krylov=True)
    un[0, 1, 2, 3] = float("inf")
    lams, us, infos, status = mcwind.solve_batch(grids + [gn], u0s + [un], check=False)
    assert status == "MCW_NONFINITE"
    assert [i["status"] for i in infos] == ["MCW_OK", "MCW_OK", "MCW_NONFINITE"]
    for i in range(2):
        assert infos[i]["rel_residual"] <= 1e-8
        lam1, _, _ = grids[i].solve(u0s[i].clone(), want_u=False)
        assert float((lams[i] - lam1).abs().max() / lam1.abs().max()) < 1e-6


def test_batch_mixing_cg_and_multigrid_runs_one_after_another():
    mcwind = _mcw()
    probs = _members()[:2]
    g0, u0 = mcwind.grid_from_problem(probs[0], krylov=True)
    g1, u1 = mcwind.grid_from_problem(probs[1], krylov=False)
    lams, _, infos, status = mcwind.solve_batch([g0, g1], [u0, u1])
    assert status == "MCW_OK"
    for g, u, lam in ((g0, u0, lams[0]), (g1, u1, lams[1])):
        lam1, _, _ = g.solve(u.clone(), want_u=False)
        assert torch.equal(lam, lam1)


def test_members_keep_their_own_tolerance_and_cycle_limit():
    """Members of one batch with different rtol and max_cycles: each stops on
    its own tolerance and runs at most its own cycle limit, taking the same
    cycles as when solved alone."""
    mcwind = _mcw()
    probs = _members()[:3]
    print("[case] batch with per-member rtol and max_cycles", flush=True)
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p) for p in probs])]
    grids[0].set_tolerance(1e-5, 200)
    grids[1].set_tolerance(1e-11, 200)
    grids[2].set_tolerance(1e-11, 3)  # 1e-11 is out of reach in 3 cycles
    lams, us, infos, status = mcwind.solve_batch(grids, u0s, check=False)
    assert status == "MCW_NOT_CONVERGED"
    assert [i["status"] for i in infos] == ["MCW_OK", "MCW_OK", "MCW_NOT_CONVERGED"]
    assert infos[0]["rel_residual"] <= 1e-5 and infos[1]["rel_residual"] <= 1e-11
    assert infos[2]["cycles"] <= 3
    assert infos[0]["cycles"] < infos[1]["cycles"]
    for g, u0, info in zip(grids, u0s, infos):
        _, _, solo = g.solve(u0.clone(), want_u=False, check=False)
        assert solo["cycles"] == info["cycles"] and solo["status"] == info["status"]


def test_member_without_an_output_wind_skips_recovery():
    """u[i] = NULL for one member: its multiplier is still solved, the others
    get their wind."""
    mcwind = _mcw()
    probs = _members()[:3]
    print("[case] batch with a NULL u member", flush=True)
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p, rtol=1e-12) for p in probs])]
    lams, us, infos, status = mcwind.solve_batch(grids, u0s, want_u=[True, False, True])
    assert status == "MCW_OK" and us[1] is None
    for i, p in enumerate(probs):
        lam_ref, u_ref, _ = osolve.solve(p, rtol=1e-14)
        assert infos[i]["rel_residual"] <= 1e-12
        assert gc.rel_err(lams[i].cpu().numpy(), lam_ref) < 1e-8
        if us[i] is not None:
            assert gc.rel_err(us[i].cpu().numpy() - p.u0, u_ref - p.u0) < 1e-8


def test_batched_kernel_timing_entry_point_leaves_solves_unchanged():
    """mcw_run_kernel_batch launches the batched sweep and residual on the
    members' own level buffers (scratch of the V-cycle): a batch solve after
    it gives the same multiplier bit for bit."""
    mcwind = _mcw()
    probs = _members()[:3]
    print("[case] batched kernel timing entry point", flush=True)
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p) for p in probs])]
    lams, _, _, _ = mcwind.solve_batch(grids, u0s, want_u=False)
    ms, launches = mcwind.run_kernel_batch(grids, "smooth", 3)
    assert ms > 0.0 and launches in (2, 4)  # two-colour launches, or one colour per launch
    ms, launches = mcwind.run_kernel_batch(grids, "residual", 2)
    assert ms > 0.0 and launches == 1
    lams2, _, _, _ = mcwind.solve_batch(grids, u0s, want_u=False)
    for a, b in zip(lams, lams2):
        assert torch.equal(a, b)
    with pytest.raises(mcwind.MCWError):
        mcwind.run_kernel_batch(grids, "smooth", 0)


@pytest.mark.parametrize("shape", [0, 2])
def test_batched_colour_passes_match_single_cg_bit_for_bit(tmp_path, monkeypatch, shape):
    """Batched CG takes each member's own steps with the single kernels'
    arithmetic, whether the batch's finest depth runs the two-colour pass (one
    block per row, tile shape 0) or the one-colour tiles (2 rows of 64
    columns): every member's multiplier equals its single CG solve bit for bit.
    The fine levels' shapes are fixed through the tuning cache."""
    mcwind = _mcw()
    probs = [inputs.hills_problem(160, 120, 8, 3, 411, a=(1.0, 1.0, 3.0)),
             inputs.hills_problem(100, 90, 8, 2, 412, a=(1.0, 1.0, 1.0))]
    entries = []
    for p in probs:
        shp = f"{p.dims[0] + 1}x{p.dims[1] + 1}x{p.dims[2] + 1}"
        entries += [f'  "gfx950|gsf|{shp}|f32": {shape}', f'  "gfx950|res|{shp}|f32": 4']
    cache = tmp_path / "tune.json"
    cache.write_text("{\n" + ",\n".join(entries) + "\n}\n")
    monkeypatch.setenv("MCW_TUNE_CACHE", str(cache))
    print(f"[case] batched CG, fine tile shape {shape}", flush=True)
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p, krylov=True, rtol=1e-10)
                                         for p in probs])]
    for g in grids:
        assert g.tile_rows(0)[0] == shape
    singles = [g.solve(u0, want_u=False)[0].clone() for g, u0 in zip(grids, u0s)]
    lams, _, infos, st = mcwind.solve_batch(grids, u0s, want_u=False)
    assert st == "MCW_OK"
    for lam, ref, info in zip(lams, singles, infos):
        assert info["rel_residual"] <= 1e-10
        assert torch.equal(lam, ref)


def test_64_member_ensemble_sampled_against_the_oracle():
    """The benchmark's ensemble (64 seeded members, 64^2..512^2 x 8..16, a3 up
    to 10) in one batch with the benchmark's options and launch shapes, solved
    to 1e-10: every member converges, the seven 64x64x8 members match the
    oracle's direct solve, and on the largest member (512x512x16) the
    oracle's f - K lambda of the GPU's lambda on two windows is small."""
    from tests.test_gpu_solve import _window_residual
    mcwind = _mcw()
    print("[case] 64-member ensemble, sampled", flush=True)
    probs = [inputs.c4_member(m) for m in range(64)]
    grids, u0s = [list(t) for t in zip(*[mcwind.grid_from_problem(p, rtol=1e-10) for p in probs])]
    lams, _, infos, st = mcwind.solve_batch(grids, u0s, want_u=False)
    assert st == "MCW_OK"
    assert max(i["rel_residual"] for i in infos) <= 1e-10
    small = [m for m, p in enumerate(probs) if p.dims == (64, 64, 8)]
    assert len(small) == 7
    for m in small:
        ref, _, _ = osolve.solve(probs[m], rtol=1e-14)
        err = gc.rel_err(lams[m].cpu().numpy(), ref)
        print(f"  member {m}: lambda rel err {err:.1e}", flush=True)
        assert err < 1e-7
    big = max(range(64), key=lambda m: probs[m].n_nodes)
    p = probs[big]
    lam_h = lams[big].cpu().numpy()
    fn = infos[big]["f_norm"]
    for (i0, i1, j0, j1) in [(0, 16, 0, 16), (250, 270, 300, 318)]:
        r, _ = _window_residual(p, lam_h, i0, i1, j0, j1)
        assert np.abs(r).max() <= 1e-10 * fn
    for g in grids:
        g.close()
