"""The discrete solution lambda of K lambda = f and the recovered wind (FP64 oracle).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product path.

The method's result is the exact solution of the symmetric positive definite
linear system that the finite element discretisation of eq. (5) produces
(start of Sec. 3), followed by the recovery of eq. (3).  Multigrid only reaches that
solution faster, so this module solves the system by the most direct route
the size allows: dense Cholesky, sparse LU, or Jacobi-preconditioned CG to a
tight relative residual.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


class System:
    """K and f restricted to the free nodes (lambda = 0 eliminated elsewhere)."""

    def __init__(self, X, Y, Z, u0, a, gamma):
        self.X, self.Y, self.Z = X, Y, Z
        self.u0 = u0
        self.a = np.asarray(a, dtype=np.float64)
        self.gamma = gamma
        self.nx, self.ny, self.nz = fem.dims_of(X)
        self.mask = fem.free_mask(self.nx, self.ny, self.nz, gamma).ravel()
        self.free = np.flatnonzero(self.mask)
        self.K_full = fem.assemble_stiffness(X, Y, Z, self.a)
        self.f_full = fem.assemble_rhs(X, Y, Z, u0)
        self.K = self.K_full[self.free][:, self.free].tocsr()
        self.f = self.f_full[self.free]

    @classmethod
    def of(cls, prob):
        return cls(prob.X, prob.Y, prob.Z, prob.u0, prob.a, prob.gamma)

    def expand(self, x_free):
        """Free-node vector -> full node vector with zeros at fixed nodes."""
        out = np.zeros(self.X.size)
        out[self.free] = x_free
        return out

    def rel_residual(self, lam_full):
        """||f - K lambda||_2 / ||f||_2 over the free nodes."""
        r = self.f - self.K @ np.asarray(lam_full).ravel()[self.free]
        nf = np.linalg.norm(self.f)
        return np.linalg.norm(r) / nf if nf > 0 else np.linalg.norm(r)


def pcg(A, b, x0=None, rtol=1e-12, maxiter=100000, check_every=50):
    """Conjugate gradients preconditioned by diag(A) (Hestenes-Stiefel).

    Stops on the TRUE relative residual ||b - A x|| / ||b|| <= rtol: whenever
    the recurrence residual says so, and every `check_every` steps, it is
    replaced by b - A x, so the answer never relies on a drifted recurrence.
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros(n), 0
    dinv = 1.0 / A.diagonal()
    r = b - A @ x
    if np.linalg.norm(r) <= rtol * nb:
        return x, 0
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for it in range(1, maxiter + 1):
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        if it % check_every == 0 or np.linalg.norm(r) <= rtol * nb:
            r = b - A @ x
            if np.linalg.norm(r) <= rtol * nb:
                return x, it
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxiter


def solve_system(K, f, method="auto", rtol=1e-13, x0=None):
    """Solve the SPD system K x = f; returns (x, method_used, iterations)."""
    n = f.shape[0]
    if method == "auto":
        method = "dense" if n <= 2000 else ("splu" if n <= 60000 else "cg")
    if method == "dense":
        L = np.linalg.cholesky(K.toarray())  # raises if K is not SPD
        return sla.cho_solve((L, True), f), "dense", 0
    if method == "splu":
        return spla.splu(K.tocsc()).solve(f), "splu", 0
    x, it = pcg(K, f, x0=x0, rtol=rtol)
    return x, "cg", it


def solve(prob, method="auto", rtol=1e-13, lam0=None):
    """lambda (full node vector, zeros where fixed), u, and an info dict."""
    t0 = time.perf_counter()
    S = System.of(prob)
    t1 = time.perf_counter()
    x0 = None if lam0 is None else np.asarray(lam0).ravel()[S.free]
    if np.linalg.norm(S.f) == 0.0:
        x, used, it = np.zeros(S.f.shape), "zero rhs", 0
    else:
        x, used, it = solve_system(S.K, S.f, method=method, rtol=rtol, x0=x0)
    t2 = time.perf_counter()
    lam = S.expand(x)
    u = fem.recover(prob.X, prob.Y, prob.Z, prob.u0, prob.a, lam)
    info = {
        "method": used,
        "iterations": it,
        "rel_residual": S.rel_residual(lam),
        "n_free": int(S.free.size),
        "t_assemble": t1 - t0,
        "t_solve": t2 - t1,
    }
    return lam.reshape(prob.X.shape), u, info


def divergence_report(prob, lam):
    """Relative discrete divergence ||D||/||D0|| over the free nodes (see fem.weak_divergence)."""
    D, D0 = fem.weak_divergence(prob.X, prob.Y, prob.Z, prob.u0, prob.a, lam)
    m = fem.free_mask(*prob.dims, prob.gamma).ravel()
    n0 = np.linalg.norm(D0[m])
    return np.linalg.norm(D[m]) / n0 if n0 > 0 else np.linalg.norm(D[m])
