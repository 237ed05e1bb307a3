"""The HIP path against the text fixtures of tests/golden/: the fine-level FP64
stencil of a uniform cube grid equals the closed form, and the set-up takes the
hand-derived coarsening decisions of Sec. 3 (also the oracle's)."""
import numpy as np
import pytest
import torch

from paper_2101_08453_amd import inputs
from tests import golden_cases as gold

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mcw():
    from paper_2101_08453_amd import mcwind
    return mcwind


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)


@pytest.mark.parametrize("h", [2.5, 30.0])
def test_cube_grid_stencil_equals_golden_closed_form(h):
    mcwind = _mcw()
    n = 8
    X, Y, Z = inputs.terrain_grid(np.zeros((n + 1, n + 1)), h * np.arange(n + 1.0), h, h)
    print(f"[case] golden cube stencil h={h}", flush=True)
    g = mcwind.Grid(_dev(X), _dev(Y), _dev(Z), (1.0, 1.0, 1.0), precision="fp64")
    st = g.stencil(0, "fp64").cpu().numpy()
    for (di, dj, dk), v in gold.cube_stencil().items():
        o = (di + 1) + 3 * (dj + 1) + 9 * (dk + 1)
        # nodes whose 26 neighbours are all free (lambda = 0 on the sides and top)
        got = st[o, 1:n - 1, 2:n - 1, 2:n - 1]
        assert np.abs(got - v * h).max() <= 1e-13 * h, (di, dj, dk)


@pytest.mark.parametrize("case", range(len(gold.coarsening_cases())))
def test_setup_takes_golden_coarsening_decision(case):
    mcwind = _mcw()
    rule, spacing, a, gamma, cmax, (X, Y, Z), want = gold.coarsening_cases()[case]
    print(f"[case] golden coarsening {case} {rule} {spacing}", flush=True)
    g = mcwind.Grid(_dev(X), _dev(Y), _dev(Z), a, gamma=gamma, precision="fp64",
                    coarsen_rule=rule, merge_spacing=spacing, coarse_direct_max=cmax)
    assert g.num_levels() >= 2
    lv = g.level(0)
    assert (lv["coarsen_h"], lv["keep_z"]) == want
