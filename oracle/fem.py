"""Finite element formulation (Sec. 2 of Mandel et al.) -- FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product path.

What is computed (Sec. 2, eqs. (3) and (5); discretisation paragraph):

* lambda lives at the vertices of isoparametric 8-node hexahedra, the wind at
  element centres.
* Stiffness: K_e = sum over the 2x2x2 Gauss points g of
  detJ_g * B_g^T diag(c) B_g, with B_g = J_g^{-T} grad_xi N (physical
  gradients of the 8 trilinear shape functions) and c_d = a_d^{-2}, i.e. the
  coefficient matrix A^{-1} with A = diag(a_1^2, a_2^2, a_3^2) (eq. (1)).
* Right-hand side of eq. (5) by one-point quadrature at the element centre:
  f_e = -8 detJ_0 B_0^T u0_e (the reference cube [-1,1]^3 has volume 8).
* Recovery, eq. (3), with the gradient taken at the element centre by the
  same derivative code: u_e = u0_e + diag(c) B_0 lambda_e.
* lambda = 0 on the boundary outside Gamma (eq. (4)); nodes on the closure
  of that set are fixed, every other node (Gamma included) is free.

Reference element conventions: local node a = i' + 2 j' + 4 k' with corner
xi_a = (2i'-1, 2j'-1, 2k'-1); N_a(xi) = prod_d (1 + xi_{a,d} xi_d) / 8;
Gauss points (+-1/sqrt(3))^3 with unit weights.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

G = 1.0 / math.sqrt(3.0)

# corners of the reference cube, local node a = i' + 2 j' + 4 k'
REF_NODES = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                      for a in range(8)], dtype=np.float64)
GAUSS_POINTS = np.array([[sx * G, sy * G, sz * G]
                         for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)])
CENTRE = np.zeros(3)


def shape_values(xi):
    """N_a(xi) for the 8 trilinear shape functions, shape (8,)."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.prod(1.0 + REF_NODES * xi[None, :], axis=1) / 8.0


def shape_grad_ref(xi):
    """Reference gradients dN_a/dxi_m at xi, shape (8, 3)."""
    xi = np.asarray(xi, dtype=np.float64)
    f = 1.0 + REF_NODES * xi[None, :]  # (8,3) factors
    d = np.empty((8, 3))
    d[:, 0] = REF_NODES[:, 0] * f[:, 1] * f[:, 2] / 8.0
    d[:, 1] = f[:, 0] * REF_NODES[:, 1] * f[:, 2] / 8.0
    d[:, 2] = f[:, 0] * f[:, 1] * REF_NODES[:, 2] / 8.0
    return d


def dims_of(X):
    nzp, nyp, nxp = X.shape
    return nxp - 1, nyp - 1, nzp - 1


def node_index(i, j, k, nx, ny):
    """Global node number, x fastest."""
    return i + (nx + 1) * (j + (ny + 1) * k)


def element_node_ids(nx, ny, nz, layers=None):
    """Global node numbers of the 8 local nodes of each element, shape (E, 8).

    Elements are numbered e = i + nx (j + ny k), restricted to the given
    element layers k if `layers` is not None.
    """
    ks = np.arange(nz) if layers is None else np.asarray(layers)
    k, j, i = np.meshgrid(ks, np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    ids = np.empty((i.size, 8), dtype=np.int64)
    for a in range(8):
        ids[:, a] = node_index(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1), nx, ny)
    return ids


def element_coords(X, Y, Z, ids):
    """Coordinates of the element nodes, shape (E, 8, 3)."""
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return xyz[ids]


def jacobian(xe, xi):
    """J[e, d, m] = d x_d / d xi_m at reference point xi, shape (E, 3, 3)."""
    return np.einsum("ead,am->edm", xe, shape_grad_ref(xi))


def physical_gradients(xe, xi):
    """(B, detJ): B[e, d, a] = d N_a / d x_d at xi, i.e. J^{-T} grad_xi N."""
    J = jacobian(xe, xi)
    det = np.linalg.det(J)
    dN = shape_grad_ref(xi)  # (8,3)
    # solve J^T B = dN^T for B (3 x 8) per element
    B = np.linalg.solve(np.transpose(J, (0, 2, 1)), np.broadcast_to(dN.T, (xe.shape[0], 3, 8)))
    return B, det


def penalty_coefficients(a):
    """Diagonal of A^{-1}: c_d = a_d^{-2} (A = diag(a_d^2), eq. (1))."""
    a = np.asarray(a, dtype=np.float64)
    return 1.0 / (a * a)


def element_stiffness(xe, c):
    """K_e = sum_g detJ_g B_g^T diag(c) B_g over the 2x2x2 Gauss points, (E, 8, 8)."""
    Ke = np.zeros((xe.shape[0], 8, 8))
    for xi in GAUSS_POINTS:
        B, det = physical_gradients(xe, xi)
        Ke += det[:, None, None] * np.einsum("eda,d,edb->eab", B, c, B)
    return Ke


def element_rhs(xe, u0e):
    """f_e = -8 detJ_0 B_0^T u0_e (one-point quadrature of -int grad mu . u0), (E, 8).

    u0e has shape (E, 3).
    """
    B, det = physical_gradients(xe, CENTRE)
    return -8.0 * det[:, None] * np.einsum("eda,ed->ea", B, u0e)


def min_detJ(X, Y, Z):
    """Smallest Jacobian determinant over the 8 Gauss points and the centre of every element."""
    nx, ny, nz = dims_of(X)
    ids = element_node_ids(nx, ny, nz)
    xe = element_coords(X, Y, Z, ids)
    dets = [np.linalg.det(jacobian(xe, xi)) for xi in list(GAUSS_POINTS) + [CENTRE]]
    return np.min(np.stack(dets, axis=1), axis=1)


def free_mask(nx, ny, nz, gamma):
    """Boolean (nz+1, ny+1, nx+1): True where lambda is an unknown.

    A node is fixed (lambda = 0) iff it lies on a face of the box that is not
    part of Gamma; faces are bit 0 bottom, 1 top, 2 x-low, 3 x-high, 4 y-low,
    5 y-high.  Nodes on an edge shared by Gamma and a fixed face are fixed.
    """
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    fixed = np.zeros(k.shape, dtype=bool)
    faces = [(0, k == 0), (1, k == nz), (2, i == 0), (3, i == nx), (4, j == 0), (5, j == ny)]
    for bit, on_face in faces:
        if not (gamma >> bit) & 1:
            fixed |= on_face
    return ~fixed


def _u0_elements(u0, layers):
    """u0 (3, nz, ny, nx) -> (E_layers, 3) in element order."""
    return np.stack([u0[d][layers].reshape(-1) for d in range(3)], axis=1)


def assemble_stiffness(X, Y, Z, a):
    """Full (unconstrained) stiffness matrix, CSR N x N, summed element by element."""
    nx, ny, nz = dims_of(X)
    N = X.size
    c = penalty_coefficients(a)
    K = sp.csr_matrix((N, N))
    for k in range(nz):
        ids = element_node_ids(nx, ny, nz, layers=[k])
        Ke = element_stiffness(element_coords(X, Y, Z, ids), c)
        rows = np.repeat(ids[:, :, None], 8, axis=2).ravel()
        cols = np.repeat(ids[:, None, :], 8, axis=1).ravel()
        K = K + sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(N, N)).tocsr()
    return K.tocsr()


def assemble_rhs(X, Y, Z, u0):
    """Full right-hand side vector (N,), before imposing lambda = 0."""
    nx, ny, nz = dims_of(X)
    f = np.zeros(X.size)
    for k in range(nz):
        ids = element_node_ids(nx, ny, nz, layers=[k])
        fe = element_rhs(element_coords(X, Y, Z, ids), _u0_elements(u0, [k]))
        np.add.at(f, ids.ravel(), fe.ravel())
    return f


def centre_gradient(X, Y, Z, lam):
    """B_0 lambda_e: gradient of the FE function at each element centre, (3, nz, ny, nx)."""
    nx, ny, nz = dims_of(X)
    lam = np.asarray(lam).ravel()
    out = np.empty((3, nz, ny, nx))
    for k in range(nz):
        ids = element_node_ids(nx, ny, nz, layers=[k])
        B, _ = physical_gradients(element_coords(X, Y, Z, ids), CENTRE)
        g = np.einsum("eda,ea->ed", B, lam[ids])
        for d in range(3):
            out[d, k] = g[:, d].reshape(ny, nx)
    return out


def recover(X, Y, Z, u0, a, lam):
    """u = u0 + A^{-1} grad lambda at element centres (eq. (3))."""
    c = penalty_coefficients(a)
    return u0 + c[:, None, None, None] * centre_gradient(X, Y, Z, lam)


def apply_stiffness_matfree(X, Y, Z, a, lam):
    """K lambda computed element by element without assembling K, (N,)."""
    nx, ny, nz = dims_of(X)
    c = penalty_coefficients(a)
    lam = np.asarray(lam).ravel()
    y = np.zeros(X.size)
    for k in range(nz):
        ids = element_node_ids(nx, ny, nz, layers=[k])
        Ke = element_stiffness(element_coords(X, Y, Z, ids), c)
        np.add.at(y, ids.ravel(), np.einsum("eab,eb->ea", Ke, lam[ids]).ravel())
    return y


def weak_divergence(X, Y, Z, u0, a, lam):
    """Weak divergence of the flux field u0 + A^{-1} grad lambda tested with every nodal
    shape function, each term with its own quadrature:

      D_a = sum_e 8 detJ_0 (B_0^T u0_e)_a + sum_e sum_g detJ_g (B_g^T q_g)_a,
      q_g = diag(c) B_g lambda_e.

    Returns (D, D0) where D0 = sum_e 8 detJ_0 B_0^T u0_e is the term of u0 alone.
    Discrete mass consistency means D = 0 at the free nodes.
    """
    nx, ny, nz = dims_of(X)
    c = penalty_coefficients(a)
    lam = np.asarray(lam).ravel()
    D = np.zeros(X.size)
    D0 = np.zeros(X.size)
    for k in range(nz):
        ids = element_node_ids(nx, ny, nz, layers=[k])
        xe = element_coords(X, Y, Z, ids)
        B0, det0 = physical_gradients(xe, CENTRE)
        t0 = 8.0 * det0[:, None] * np.einsum("eda,ed->ea", B0, _u0_elements(u0, [k]))
        np.add.at(D0, ids.ravel(), t0.ravel())
        t = np.zeros_like(t0)
        for xi in GAUSS_POINTS:
            B, det = physical_gradients(xe, xi)
            q = c[None, :] * np.einsum("eda,ea->ed", B, lam[ids])
            t += det[:, None] * np.einsum("eda,ed->ea", B, q)
        np.add.at(D, ids.ravel(), (t0 + t).ravel())
    return D, D0


def element_volumes(X, Y, Z):
    """Volume of each hexahedron by 2x2x2 Gauss (exact for trilinear maps), (nz, ny, nx)."""
    nx, ny, nz = dims_of(X)
    ids = element_node_ids(nx, ny, nz)
    xe = element_coords(X, Y, Z, ids)
    v = sum(np.linalg.det(jacobian(xe, xi)) for xi in GAUSS_POINTS)
    return v.reshape(nz, ny, nx)
