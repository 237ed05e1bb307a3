"""mcw_divergence_noalloc (the divergence check for callers that cannot
allocate: no handle, partial sums in the library's fixed device array) against
mcw_divergence on a handle, on two calls in a row, the second with a smaller
grid; and the size limit of the fixed array."""
import numpy as np
import pytest
import torch

from paper_2101_08453_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)


def test_noalloc_divergence_equals_the_handle_call_twice_in_a_row():
    from paper_2101_08453_amd import mcwind
    for p in (inputs.hills_problem(70, 52, 9, 3, 31, a=(1.0, 1.0, 3.0), noise=0.3),
              inputs.distorted_problem(23, 17, 5, seed=8, amp=0.2, a=(1.0, 1.5, 2.0),
                                       gamma=inputs.GAMMA_BOTTOM | inputs.GAMMA_XLO)):
        print(f"[case] noalloc divergence {p.name} gamma {p.gamma}", flush=True)
        X, Y, Z, u0 = (_dev(A) for A in (p.X, p.Y, p.Z, p.u0))
        g = mcwind.Grid(X, Y, Z, p.a, gamma=p.gamma, rtol=1e-10)
        lam, _, _ = g.solve(u0, want_u=False)
        D_ref, rel_ref = g.divergence(u0, lam)
        D, rel = mcwind.divergence_noalloc(X, Y, Z, p.a, u0, lam, gamma=p.gamma)
        torch.cuda.synchronize()
        assert torch.equal(D, D_ref)  # the same kernel and the same deterministic sums
        assert rel == rel_ref and rel <= 1e-10
        # enqueue-only form (no result to the host): D is the same once the stream is done
        D2, none = mcwind.divergence_noalloc(X, Y, Z, p.a, u0, lam, gamma=p.gamma, want_rel=False)
        torch.cuda.synchronize()
        assert none is None and torch.equal(D2, D_ref)
        g.close()


def test_noalloc_divergence_rejects_grids_beyond_its_scratch():
    from paper_2101_08453_amd import mcwind
    n = 15 * 363 - 1  # 363^2 element tiles of 15 x 15 node columns > (2 MiB / 8 - 2) / 2
    print("[case] noalloc size limit (host-side check, no launch)", flush=True)
    Xb = torch.zeros((2, n + 1, n + 1), dtype=torch.float64, device="cuda")
    u0 = torch.zeros((3, 1, n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(mcwind.MCWError) as ei:
        mcwind.divergence_noalloc(Xb, Xb, Xb, (1.0, 1.0, 1.0), u0, Xb)
    assert ei.value.status_name == "MCW_INVALID_ARG" and "scratch" in str(ei.value)
