"""Gradient of a wind loss through the mass-consistent solve -- FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by tests/ and the smoke check; never by the
product path.

Derivation (chain rule through eqs. (3) and (5) as discretised in Sec. 2):
with G_1 lambda = B_0 lambda_e (centre gradients), W_1 = 8 detJ_0,
K = sum_g G_g^T detJ_g diag(c) G_g, f = -G_1^T W_1 u0 and
u = u0 + diag(c) G_1 lambda, a loss L(u) with g_u = dL/du gives

  g_lambda = G_1^T diag(c) g_u          (restricted to the free nodes)
  K mu = g_lambda                        (K is symmetric: same operator)
  dL/du0 = g_u - W_1 G_1 mu
  dL/dc_d = sum_e g_u[d,e] (B_0 lambda_e)_d
            - sum_e sum_g detJ_g (B_g mu_e)_d (B_g lambda_e)_d
  dL/da_d = -2 a_d^{-3} dL/dc_d         (c_d = a_d^{-2})
"""
from __future__ import annotations

import numpy as np

from . import fem
from .solve import System, solve_system


def surface_loss(u, mask):
    """L = sum over bottom-layer element centres inside mask of u_x^2 + u_y^2, and dL/du."""
    L = float(np.sum(u[0, 0][mask] ** 2 + u[1, 0][mask] ** 2))
    g = np.zeros_like(u)
    g[0, 0][mask] = 2.0 * u[0, 0][mask]
    g[1, 0][mask] = 2.0 * u[1, 0][mask]
    return L, g


def _solve(K, f, rtol, solver):
    if solver is None:
        return solve_system(K, f, rtol=rtol)[0]
    return solver(K, f)


def forward(prob_X, prob_Y, prob_Z, u0, a, gamma, rtol=1e-13, solver=None):
    """solver: None for solve_system's default choice, else a callable
    (K, f) -> x that solves K x = f to the accuracy the caller needs (a large
    grid's Jacobi-PCG cannot reach 1e-13 in reasonable time)."""
    S = System(prob_X, prob_Y, prob_Z, u0, a, gamma)
    x = _solve(S.K, S.f, rtol, solver)
    lam = S.expand(x)
    u = fem.recover(prob_X, prob_Y, prob_Z, u0, a, lam)
    return S, lam, u


def gradient(prob, mask, rtol=1e-13, solver=None):
    """(L, dL/du0 (3,nz,ny,nx), dL/da (3,)) for the surface loss; `solver`
    as in forward, used for both the forward and the transpose solve."""
    X, Y, Z = prob.X, prob.Y, prob.Z
    nx, ny, nz = prob.dims
    a = np.asarray(prob.a, dtype=np.float64)
    c = fem.penalty_coefficients(a)
    S, lam, u = forward(X, Y, Z, prob.u0, a, prob.gamma, rtol, solver)
    L, g_u = surface_loss(u, mask)

    # g_lambda = G_1^T diag(c) g_u, assembled over the elements
    g_lam = np.zeros(X.size)
    dL_du0 = g_u.copy()
    dL_dc = np.zeros(3)
    mu_full = None
    for k in range(nz):
        ids = fem.element_node_ids(nx, ny, nz, layers=[k])
        B0, _ = fem.physical_gradients(fem.element_coords(X, Y, Z, ids), fem.CENTRE)
        gu = np.stack([g_u[d, k].ravel() for d in range(3)], axis=1)
        np.add.at(g_lam, ids.ravel(), np.einsum("eda,ed->ea", B0, c[None, :] * gu).ravel())
    mu_free = _solve(S.K, g_lam[S.free], rtol, solver)
    mu_full = S.expand(mu_free)
    for k in range(nz):
        ids = fem.element_node_ids(nx, ny, nz, layers=[k])
        xe = fem.element_coords(X, Y, Z, ids)
        B0, det0 = fem.physical_gradients(xe, fem.CENTRE)
        gmu = np.einsum("eda,ea->ed", B0, mu_full[ids])
        glam = np.einsum("eda,ea->ed", B0, lam[ids])
        gu = np.stack([g_u[d, k].ravel() for d in range(3)], axis=1)
        for d in range(3):
            dL_du0[d, k] -= (8.0 * det0 * gmu[:, d]).reshape(ny, nx)
        dL_dc += np.sum(gu * glam, axis=0)
        for xi in fem.GAUSS_POINTS:
            B, det = fem.physical_gradients(xe, xi)
            dL_dc -= np.sum(det[:, None] * np.einsum("eda,ea->ed", B, mu_full[ids])
                            * np.einsum("eda,ea->ed", B, lam[ids]), axis=0)
    dL_da = -2.0 * dL_dc / a ** 3
    return L, dL_du0, dL_da


def loss_of(prob, u0, a, mask, rtol=1e-13):
    _, _, u = forward(prob.X, prob.Y, prob.Z, u0, np.asarray(a, dtype=np.float64), prob.gamma, rtol)
    return surface_loss(u, mask)[0]
