"""Steps on either side of the solve in a coupled fire-atmosphere model -- FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product path.

The solve replaces the interpolation of the atmospheric model's wind to the
fire model's grid (Sec. 1): before it, the coarse wind (horizontal spacing
300 m - 1 km, terrain-following levels) gives u0 at the fine element centres;
after it, the fire model takes the horizontal wind at a fixed height above
the terrain. The paper names these steps without defining them; the reading
used here:

* Element centre: the mean of the element's 8 corner nodes (the image of the
  reference centre under the trilinear map). Ground under an element column:
  the mean of the column's 4 bottom nodes. Height above ground of a centre:
  its z minus that ground height.
* Coarse wind: ncx x ncy columns at (x0 + I dx, y0 + J dy), nl levels per
  column at heights above the coarse ground hagl[l, J, I] (increasing in l),
  three components per level.
* Interpolation to a centre at (xc, yc) with height zeta above ground: in each
  of the four coarse columns around (xc, yc) (positions clamped to the coarse
  grid), take the wind at height zeta: linear between the two levels around
  zeta; the top level's wind above the top; below the lowest level h1 the
  neutral log law v(h1) ln(zeta/z0) / ln(h1/z0), zero at zeta <= z0. Then
  combine the four columns with bilinear weights.
* Surface wind at height H over an element column: the same vertical rule on
  the column's element centres (linear between the centres around H, the top
  centre's value above, the log law from the lowest centre below).
"""
from __future__ import annotations

import numpy as np


def element_centres(X, Y, Z):
    """Centres (3, nz, ny, nx): mean of the 8 corners of each element."""
    def mean8(A):
        return 0.125 * (A[:-1, :-1, :-1] + A[:-1, :-1, 1:] + A[:-1, 1:, :-1] + A[:-1, 1:, 1:]
                        + A[1:, :-1, :-1] + A[1:, :-1, 1:] + A[1:, 1:, :-1] + A[1:, 1:, 1:])
    return np.stack([mean8(X), mean8(Y), mean8(Z)])


def ground_height(Z):
    """(ny, nx): mean of the 4 bottom nodes of each element column."""
    B = Z[0]
    return 0.25 * (B[:-1, :-1] + B[:-1, 1:] + B[1:, :-1] + B[1:, 1:])


def heights_above_ground(X, Y, Z):
    c = element_centres(X, Y, Z)
    return c, c[2] - ground_height(Z)[None]


def column_profile(h, v, zeta, z0):
    """Value at height zeta of one column with levels h (increasing) and values v
    (..., nl): linear inside, constant above, log law below h[0]."""
    h = np.asarray(h, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    if zeta >= h[-1]:
        return v[..., -1]
    if zeta >= h[0]:
        l = int(np.searchsorted(h, zeta, side="right")) - 1
        l = min(l, len(h) - 2)
        t = (zeta - h[l]) / (h[l + 1] - h[l])
        return (1.0 - t) * v[..., l] + t * v[..., l + 1]
    if zeta <= z0:
        return np.zeros_like(v[..., 0])
    return v[..., 0] * (np.log(zeta / z0) / np.log(h[0] / z0))


def bilinear_cell(pos, origin, spacing, n):
    """Lower coarse index and weight along one axis, the position clamped to
    [origin, origin + (n-1) spacing]."""
    s = (pos - origin) / spacing
    s = min(max(s, 0.0), n - 1.0)
    i = min(int(np.floor(s)), n - 2)
    return i, s - i


def element_centre(X, Y, Z, k, j, i):
    """Centre (x, y, z) of element (i, j, k) and the ground height under it."""
    sl = (slice(k, k + 2), slice(j, j + 2), slice(i, i + 2))
    c = np.array([X[sl].mean(), Y[sl].mean(), Z[sl].mean()])
    return c, Z[0, j:j + 2, i:i + 2].mean()


def interp_wind_element(X, Y, Z, cw, k, j, i):
    """u0 (3,) at the centre of element (i, j, k) from the coarse wind
    cw = dict(x0, y0, dx, dy, hagl (nl, ncy, ncx), wind (3, nl, ncy, ncx), z0)."""
    c, zs = element_centre(X, Y, Z, k, j, i)
    zeta = c[2] - zs
    hagl, wind = cw["hagl"], cw["wind"]
    _, ncy, ncx = hagl.shape
    I, a = bilinear_cell(c[0], cw["x0"], cw["dx"], ncx)
    J, b = bilinear_cell(c[1], cw["y0"], cw["dy"], ncy)
    acc = np.zeros(3)
    for (dI, dJ, w) in ((0, 0, (1 - a) * (1 - b)), (1, 0, a * (1 - b)),
                        (0, 1, (1 - a) * b), (1, 1, a * b)):
        acc += w * column_profile(hagl[:, J + dJ, I + dI], wind[:, :, J + dJ, I + dI], zeta, cw["z0"])
    return acc


def interp_wind(X, Y, Z, cw):
    """u0 (3, nz, ny, nx) at every element centre (loops: for small grids)."""
    nz, ny, nx = (s - 1 for s in X.shape)
    u0 = np.zeros((3, nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                u0[:, k, j, i] = interp_wind_element(X, Y, Z, cw, k, j, i)
    return u0


def surface_wind_column(X, Y, Z, u, height, z0, j, i):
    """(2,): horizontal wind at `height` above ground over element column (i, j),
    from the wind u (3, nz, ny, nx) at the element centres."""
    nz = X.shape[0] - 1
    zeta = np.array([element_centre(X, Y, Z, k, j, i)[0][2] for k in range(nz)])
    zeta -= Z[0, j:j + 2, i:i + 2].mean()
    return column_profile(zeta, u[:2, :, j, i], height, z0)


def surface_wind(X, Y, Z, u, height, z0):
    """(2, ny, nx) over every element column (loops: for small grids)."""
    nz, ny, nx = (s - 1 for s in X.shape)
    out = np.zeros((2, ny, nx))
    for j in range(ny):
        for i in range(nx):
            out[:, j, i] = surface_wind_column(X, Y, Z, u, height, z0, j, i)
    return out
