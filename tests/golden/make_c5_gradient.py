"""Write c5_gradient.txt: the FP64 oracle's gradient of the surface-wind loss
on the 512 x 512 x 15 fractal-terrain grid (500 m relief, a = (1, 1, 1)),
whose GPU counterpart is the adjoint through the solve.

Only oracle/ computes: the loss L = sum over the bottom-layer element centres
inside the seeded elliptical fire mask of u_x^2 + u_y^2, dL/da, and the
directional derivatives <dL/du0, d_k> along 20 seeded N(0, 1) directions
(the inputs module draws the grid, the mask and the directions).  Both
solves (lambda and the transpose solve for mu) are the oracle's conjugate
gradients preconditioned by one symmetric V-cycle of the oracle's multigrid
(Sec. 3), run until the recurrence residual is below 1e-14; the true relative
residuals ||f - K x|| / ||f|| are checked below 1e-13 and written out.
Diagonal-preconditioned CG cannot reach 1e-13 on this grid in hours.

Usage: python -m tests.golden.make_c5_gradient   (about ten minutes on one core)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint, multigrid  # noqa: E402
from paper_2101_08453_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_gradient.txt")
N_DIRECTIONS = 20


def main():
    t0 = time.perf_counter()
    p = inputs.c5()
    mask = inputs.fire_mask(512, 512, seed=55)
    levels = multigrid.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=1024)
    M = multigrid.Multigrid(levels, symmetric=True)
    true_res = []

    def solver(K, f):
        x, _ = M.pcg(f, rtol=1e-14, maxiter=60)
        true_res.append(float(np.linalg.norm(f - K @ x) / np.linalg.norm(f)))
        assert true_res[-1] < 1e-13, true_res
        return x

    L, g_u0, g_a = adjoint.gradient(p, mask, rtol=1e-13, solver=solver)
    dirs = inputs.random_directions(p.u0.shape, N_DIRECTIONS, seed=56)
    dd = [float(np.sum(g_u0 * d)) for d in dirs]
    lines = [
        "# Gradient of the surface-wind loss through the solve on the 512x512x15 grid",
        "# (fractal terrain of 500 m relief, seed 5; a = (1, 1, 1); fire mask seed 55;",
        "# directions N(0,1), seed 56), by the FP64 oracle (oracle/adjoint.py, the chain",
        "# rule through eqs. (3) and (5) of Sec. 2), multigrid-preconditioned CG solves;",
        "# true relative residuals " + ", ".join(f"{r:.1e}" for r in true_res) + ".",
        "# Written by tests/golden/make_c5_gradient.py, which calls only oracle/.",
        f"# fire-mask centres: {int(mask.sum())}; oracle time {time.perf_counter() - t0:.0f} s",
        f"loss {L:.17e}",
        "dL_da " + " ".join(f"{v:.17e}" for v in g_a),
    ]
    lines += [f"dL_du0_dot_direction {k} {v:.17e}" for k, v in enumerate(dd)]
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
