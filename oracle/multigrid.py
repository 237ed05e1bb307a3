"""Multigrid pieces of Sec. 3 of Mandel et al. -- FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product path.

* Coarse grids are subsets of the fine grid nodes: in each coarsened
  direction every other node plus the last one (odd counts leave one coarse
  interval spanning a single fine element).
* Prolongation P interpolates with the weights of linear interpolation on a
  regular grid (1 at kept nodes, 1/2 from each neighbour at dropped nodes),
  as a tensor product over the directions; identity in directions that are
  not coarsened (Sec. 3, base method and semicoarsening paragraphs).
* Coarse operators are variational: K_c = P^T K P, and the coarse right-hand
  side f_c = P^T (f - K u) (eqs. (6)-(7)).
* Smoother: Gauss-Seidel in vertical sweeps from the bottom up, the columns
  split horizontally into 4 red-black groups (i mod 2, j mod 2) visited in
  the order (0,0), (1,0), (0,1), (1,1).
* Coarsening decision (Sec. 3, last paragraph), with the readings used here:
  the vertical-to-horizontal coupling ratio is r = a_3 h_3 / (a_h h_h) for
  the assembled operator (coefficient a_d^{-2}), or the printed
  h_3 / (h_1 a_3) with rule="literal"; coarsen horizontally iff the ratio of
  the bottom layer exceeds 1/3; then walk the layers from the ground up and
  merge layer k with layer k+1 iff the ratio of layer k is below 3 (an
  unpaired top layer stays).  The layer test takes h_h of the level being
  coarsened (spacing="level", the default), so that both thresholds bound
  the coupling anisotropy of the grid the smoother runs on by 9; the paper
  prints the spacing after the horizontal step (spacing="coarsened"), which
  lets a merged pair reach anisotropy 36.  rule="full" is the base method:
  coarsen every direction.  Stop when the free unknowns fit the direct
  solver, or nothing coarsens; if nothing coarsens while the grid is still
  too large, coarsen horizontally anyway.
* Beyond the paper: the symmetric V-cycle (post-smoothing in the reverse
  order) and conjugate gradients preconditioned by it, the textbook method
  (Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.1); and the
  vertical line smoother, the other reading of "vertical sweeps": block
  Gauss-Seidel whose blocks are the free nodes of one column, solved exactly,
  in the same colour order.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem

RULES = ("operator", "literal", "full")
SPACINGS = ("level", "coarsened")
COLOURS = ((0, 0), (1, 0), (0, 1), (1, 1))


# ---------------------------------------------------------------- coarsening

def spacings(X, Y, Z):
    """(h1, h2, h3): mean x and y node spacings of the bottom plane and the mean
    thickness of every layer, shape (nz,)."""
    h1 = float(np.mean(X[0, :, 1:] - X[0, :, :-1]))
    h2 = float(np.mean(Y[0, 1:, :] - Y[0, :-1, :]))
    h3 = np.mean(Z[1:] - Z[:-1], axis=(1, 2))
    return h1, h2, h3


def coupling_ratio(h3, hh, a, rule):
    """Vertical-to-horizontal ratio that the coarsening thresholds compare."""
    ah = math.sqrt(a[0] * a[1])
    if rule == "operator":
        return a[2] * h3 / (ah * hh)
    if rule == "literal":
        return ah * h3 / (hh * a[2])
    raise ValueError(rule)


def n_free(nx, ny, nz, gamma):
    return int(fem.free_mask(nx, ny, nz, gamma).sum())


def decide(X, Y, Z, a, rule, gamma, coarse_max, spacing="level"):
    """Coarsening of one level: (coarsen_horizontally, kept node planes) or None
    when this level is the coarsest.  `spacing` is the horizontal spacing the
    layer test compares with: the level's own ("level") or the one after the
    horizontal step ("coarsened")."""
    if spacing not in SPACINGS:
        raise ValueError(spacing)
    nx, ny, nz = fem.dims_of(X)
    if n_free(nx, ny, nz, gamma) <= coarse_max:
        return None
    can_h = nx >= 3 and ny >= 3
    h1, h2, h3 = spacings(X, Y, Z)
    hh = math.sqrt(h1 * h2)
    if rule == "full":
        ch = can_h
        keep = list(range(0, nz + 1, 2))
        if keep[-1] != nz:
            keep.append(nz)
    else:
        ch = can_h and coupling_ratio(h3[0], hh, a, rule) > 1.0 / 3.0
        hh2 = 2.0 * hh if (ch and spacing == "coarsened") else hh
        keep = [0]
        k = 0
        while k < nz:
            if k + 1 < nz and coupling_ratio(h3[k], hh2, a, rule) < 3.0:
                keep.append(k + 2)
                k += 2
            else:
                keep.append(k + 1)
                k += 1
    # A coarse level keeps a free node: with both z faces fixed, dropping every
    # interior plane would leave none, so then all planes are kept.
    nxc = len(horizontal_keep(nx)) - 1 if ch else nx
    nyc = len(horizontal_keep(ny)) - 1 if ch else ny
    if n_free(nxc, nyc, len(keep) - 1, gamma) == 0:
        keep = list(range(nz + 1))
    if not ch and len(keep) == nz + 1:
        if not can_h:
            return None
        ch = True  # forced: nothing coarsened but the grid is too large
    return ch, keep


def horizontal_keep(n):
    """Kept node indices of a coarsened direction with n elements: evens and the last."""
    keep = list(range(0, n + 1, 2))
    if keep[-1] != n:
        keep.append(n)
    return keep


def interpolation_1d(n, keep):
    """(n+1) x len(keep) regular-grid linear interpolation from the kept nodes."""
    idx = {p: q for q, p in enumerate(keep)}
    rows, cols, vals = [], [], []
    for p in range(n + 1):
        if p in idx:
            rows.append(p); cols.append(idx[p]); vals.append(1.0)
        else:
            rows += [p, p]; cols += [idx[p - 1], idx[p + 1]]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, len(keep)))


class Level:
    def __init__(self, X, Y, Z, K_full, gamma):
        self.X, self.Y, self.Z = X, Y, Z
        self.nx, self.ny, self.nz = fem.dims_of(X)
        self.K_full = K_full
        self.mask = fem.free_mask(self.nx, self.ny, self.nz, gamma).ravel()
        self.free = np.flatnonzero(self.mask)
        self.K = K_full[self.free][:, self.free].tocsr()
        self.P_full = None  # to the next coarser level
        self.P = None
        self.coarsen_h = None
        self.keep_z = None

    @property
    def dims(self):
        return self.nx, self.ny, self.nz


def build_hierarchy(X, Y, Z, a, gamma=1, rule="operator", coarse_max=1024, max_levels=40,
                    spacing="level"):
    """Levels from fine to coarse, with P and K_c = P^T K P at each step."""
    a = np.asarray(a, dtype=np.float64)
    K = fem.assemble_stiffness(X, Y, Z, a)
    levels = [Level(X, Y, Z, K, gamma)]
    while len(levels) < max_levels:
        L = levels[-1]
        d = decide(L.X, L.Y, L.Z, a, rule, gamma, coarse_max, spacing)
        if d is None:
            break
        ch, keep_z = d
        kx = horizontal_keep(L.nx) if ch else list(range(L.nx + 1))
        ky = horizontal_keep(L.ny) if ch else list(range(L.ny + 1))
        Px = interpolation_1d(L.nx, kx)
        Py = interpolation_1d(L.ny, ky)
        Pz = interpolation_1d(L.nz, keep_z)
        P = sp.kron(Pz, sp.kron(Py, Px)).tocsr()
        Kc = (P.T @ L.K_full @ P).tocsr()
        sel = np.ix_(keep_z, ky, kx)
        C = Level(L.X[sel], L.Y[sel], L.Z[sel], Kc, gamma)
        L.P_full = P
        L.P = P[L.free][:, C.free].tocsr()
        L.coarsen_h = ch
        L.keep_z = keep_z
        levels.append(C)
    return levels


# ---------------------------------------------------------------- smoother

def colour_order(nx, ny, nz, mask):
    """Free node numbers in smoothing order: colour groups (i mod 2, j mod 2)
    in the order (0,0),(1,0),(0,1),(1,1); each column bottom to top."""
    order = []
    for ci, cj in COLOURS:
        for j in range(cj, ny + 1, 2):
            for i in range(ci, nx + 1, 2):
                for k in range(nz + 1):
                    n = fem.node_index(i, j, k, nx, ny)
                    if mask[n]:
                        order.append(n)
    return np.asarray(order, dtype=np.int64)


def gs_sweep_full(K_full, mask, dims, x, f, order=None, reverse=False):
    """One Gauss-Seidel sweep on full-length vectors x, f (fixed nodes untouched).

    Updating the nodes one by one in `order` is the same as solving with the
    lower triangle (diagonal included) of K permuted to that order:
    x_pi += tril(K_pi)^{-1} (f - K x)_pi.
    reverse=True visits the nodes in the opposite order (colours (1,1),(0,1),
    (1,0),(0,0), each column top to bottom): the adjoint sweep, which makes a
    V-cycle symmetric when it follows the forward pre-smoothing.
    """
    nx, ny, nz = dims
    if order is None:
        order = colour_order(nx, ny, nz, mask)
    if reverse:
        order = order[::-1]
    x = np.array(x, dtype=np.float64)
    Kp = K_full[order][:, order].tocsr()
    r = f[order] - (K_full @ x)[order]
    x[order] += spla.spsolve_triangular(sp.tril(Kp).tocsr(), r, lower=True)
    return x


def column_blocks(nx, ny, nz, mask, colour):
    """Free node numbers of each column of one colour class (i mod 2, j mod 2)."""
    ci, cj = colour
    cols = []
    for j in range(cj, ny + 1, 2):
        for i in range(ci, nx + 1, 2):
            c = [fem.node_index(i, j, k, nx, ny) for k in range(nz + 1)]
            c = [n for n in c if mask[n]]
            if c:
                cols.append(np.asarray(c, dtype=np.int64))
    return cols


def line_sweep_full(K_full, mask, dims, x, f, reverse=False):
    """One vertical line Gauss-Seidel sweep on full-length vectors (not in the
    paper; the reading of "vertical sweeps" as exact column solves): colour by
    colour, every free column c of the colour solves its own block,
    x_c += K_cc^{-1} (f - K x)_c.  Columns of one colour do not couple, so the
    residual of a colour is taken once.  reverse=True runs the colours in the
    opposite order (the adjoint sweep)."""
    nx, ny, nz = dims
    x = np.array(x, dtype=np.float64)
    order = COLOURS[::-1] if reverse else COLOURS
    K = K_full.tocsr()
    for colour in order:
        r = f - K @ x
        for c in column_blocks(nx, ny, nz, mask, colour):
            x[c] += np.linalg.solve(K[c][:, c].toarray(), r[c])
    return x


class Multigrid:
    """V-cycle on the free-node systems of a hierarchy (eqs. (6)-(7)).

    symmetric=True runs the post-smoothing sweeps in the reverse order (not in
    the paper): with nu_pre == nu_post the V-cycle from zero is then a
    symmetric positive definite operator B, usable as a CG preconditioner."""

    def __init__(self, levels, nu_pre=2, nu_post=2, symmetric=False, smoother="point"):
        self.levels = levels
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.symmetric = symmetric
        self.smoother = smoother
        self._orders = []
        self._tri = []
        self._tri_rev = []
        for L in levels:
            order_full = colour_order(L.nx, L.ny, L.nz, L.mask)
            pos = np.full(L.mask.size, -1, dtype=np.int64)
            pos[L.free] = np.arange(L.free.size)
            order = pos[order_full]  # positions within the free-node vector
            self._orders.append(order)
            self._tri.append(sp.tril(L.K[order][:, order]).tocsr())
            rev = order[::-1]
            self._tri_rev.append(sp.tril(L.K[rev][:, rev]).tocsr())
        self._coarse = np.linalg.cholesky(levels[-1].K.toarray())

    def smooth(self, l, x, f, reverse=False):
        if self.smoother == "line":
            L = self.levels[l]
            xf = np.zeros(L.mask.size)
            ff = np.zeros(L.mask.size)
            xf[L.free] = x
            ff[L.free] = f
            return line_sweep_full(L.K_full, L.mask, L.dims, xf, ff, reverse)[L.free]
        order = self._orders[l][::-1] if reverse else self._orders[l]
        tri = self._tri_rev[l] if reverse else self._tri[l]
        r = f - self.levels[l].K @ x
        x = x.copy()
        x[order] += spla.spsolve_triangular(tri, r[order], lower=True)
        return x

    def coarse_solve(self, f):
        Lc = self._coarse
        y = spla.spsolve_triangular(sp.csr_matrix(Lc), f, lower=True)
        return spla.spsolve_triangular(sp.csr_matrix(Lc.T), y, lower=False)

    def vcycle(self, x, f, l=0):
        L = self.levels[l]
        if l == len(self.levels) - 1:
            return self.coarse_solve(f)
        for _ in range(self.nu_pre):
            x = self.smooth(l, x, f)
        rc = L.P.T @ (f - L.K @ x)
        x = x + L.P @ self.vcycle(np.zeros(rc.shape), rc, l + 1)
        for _ in range(self.nu_post):
            x = self.smooth(l, x, f, reverse=self.symmetric)
        return x

    def precondition(self, r):
        """B r: one V-cycle on K z = r from z = 0."""
        return self.vcycle(np.zeros_like(r), r)

    def pcg(self, f, steps=None, rtol=1e-12, maxiter=500):
        """Conjugate gradients on K x = f from x = 0, preconditioned by one
        V-cycle per step (Hestenes-Stiefel recurrences, Fletcher-Reeves beta).
        Runs `steps` steps if given, else until ||f - K x|| <= rtol ||f||.
        Returns x and the relative residual norms of the recurrence."""
        K = self.levels[0].K
        x = np.zeros_like(f)
        r = f.copy()
        nf = np.linalg.norm(f)
        z = self.precondition(r)
        p = z.copy()
        rz = r @ z
        hist = []
        for it in range(steps if steps is not None else maxiter):
            q = K @ p
            alpha = rz / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            hist.append(np.linalg.norm(r) / nf)
            if steps is None and hist[-1] <= rtol:
                break
            z = self.precondition(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        return x, hist

    def convergence_factor(self, cycles=12, seed=0, skip=4):
        """Asymptotic residual reduction per V-cycle for K e = 0 from a random start."""
        rng = np.random.default_rng(seed)
        K = self.levels[0].K
        x = rng.standard_normal(K.shape[0])
        f = np.zeros_like(x)
        norms = []
        for _ in range(cycles):
            x = self.vcycle(x, f)
            norms.append(np.linalg.norm(K @ x))
        return (norms[-1] / norms[skip - 1]) ** (1.0 / (cycles - skip))

    def solve(self, f, x0=None, rtol=1e-10, max_cycles=200):
        K = self.levels[0].K
        x = np.zeros_like(f) if x0 is None else x0.copy()
        nf = np.linalg.norm(f)
        hist = []
        for _ in range(max_cycles):
            x = self.vcycle(x, f)
            hist.append(np.linalg.norm(f - K @ x) / nf)
            if hist[-1] <= rtol:
                break
        return x, hist


# ---------------------------------------------------------------- layout helper

def stencil_array(K_full, nx, ny, nz):
    """27-point node stencil of a full-grid matrix, shape (27, nz+1, ny+1, nx+1):
    entry o = (di+1) + 3(dj+1) + 9(dk+1) holds K[n, n + offset] (0 off the grid)."""
    N = (nx + 1) * (ny + 1) * (nz + 1)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    out = np.zeros((27, nz + 1, ny + 1, nx + 1))
    Kc = K_full.tocsr()
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                o = (di + 1) + 3 * (dj + 1) + 9 * (dk + 1)
                ii, jj, kk = i + di, j + dj, k + dk
                ok = (ii >= 0) & (ii <= nx) & (jj >= 0) & (jj <= ny) & (kk >= 0) & (kk <= nz)
                rows = fem.node_index(i[ok], j[ok], k[ok], nx, ny)
                cols = fem.node_index(ii[ok], jj[ok], kk[ok], nx, ny)
                vals = np.asarray(Kc[rows, cols]).ravel()
                tmp = np.zeros(N)
                tmp[rows] = vals
                out[o] = tmp.reshape(nz + 1, ny + 1, nx + 1)
    return out
