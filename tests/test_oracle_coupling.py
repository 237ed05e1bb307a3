"""Pins of the oracle's steps around the solve (interpolation of a coarse
atmospheric wind to the element centres, surface wind at a height): exactness
on fields linear in position and height, the log law below the lowest level
in closed form, clamping outside the coarse grid, constant extrapolation above
the top."""
import math

import numpy as np
import pytest

from oracle import coupling
from paper_2101_08453_amd import inputs


def _grid(nx=7, ny=5, nz=4, seed=9, first=5.0):
    p = inputs.hills_problem(nx, ny, nz, 2, seed)
    zeta = inputs.vertical_levels(nz, first=first)
    X, Y, _ = inputs.terrain_grid(np.zeros((ny + 1, nx + 1)), zeta, 30.0, 30.0)
    return X, Y, p.Z


def _coarse(ncx, ncy, nl, x0, y0, d, h_first, seed=1):
    rng = np.random.default_rng(seed)
    base = h_first * 1.3 ** np.arange(nl)
    hagl = base[:, None, None] * rng.uniform(0.9, 1.1, (1, ncy, ncx))
    xs = x0 + d * np.arange(ncx)
    ys = y0 + d * np.arange(ncy)
    return hagl, xs, ys


def test_centres_and_heights_on_a_flat_box():
    X, Y, Z = inputs.terrain_grid(np.zeros((3, 4)), np.array([0.0, 2.0, 6.0]), 10.0, 20.0)
    c, zeta = coupling.heights_above_ground(X, Y, Z)
    assert np.allclose(c[0, 0, 0, :], [5.0, 15.0, 25.0])
    assert np.allclose(c[1, 0, :, 0], [10.0, 30.0])
    assert np.allclose(zeta[:, 0, 0], [1.0, 4.0])


def test_interpolation_is_exact_for_fields_linear_in_position_and_height():
    X, Y, Z = _grid()
    hagl, xs, ys = _coarse(5, 4, 18, -40.0, -35.0, 70.0, 0.5)
    al, be, ga, de = np.array([1.0, -2.0, 0.5]), np.array([0.01, 0.02, -0.03]), \
        np.array([-0.02, 0.005, 0.01]), np.array([0.3, -0.1, 0.05])
    wind = (al[:, None, None, None] + be[:, None, None, None] * xs[None, None, None, :]
            + ga[:, None, None, None] * ys[None, None, :, None] + de[:, None, None, None] * hagl[None])
    cw = dict(x0=-40.0, y0=-35.0, dx=70.0, dy=70.0, hagl=hagl, wind=wind, z0=0.1)
    c, zeta = coupling.heights_above_ground(X, Y, Z)
    assert zeta.min() > hagl[0].max() and zeta.max() < hagl[-1].min()
    u0 = coupling.interp_wind(X, Y, Z, cw)
    ref = (al[:, None, None, None] + be[:, None, None, None] * c[0][None]
           + ga[:, None, None, None] * c[1][None] + de[:, None, None, None] * zeta[None])
    assert np.abs(u0 - ref).max() < 1e-12 * np.abs(ref).max()


def test_log_law_below_the_lowest_level_and_constant_above_the_top():
    X, Y, Z = _grid(nz=6)
    _, zeta = coupling.heights_above_ground(X, Y, Z)
    nl, h1, z0 = 3, 20.0, 0.2
    hagl = np.broadcast_to(np.array([h1, 30.0, 40.0])[:, None, None], (nl, 3, 3)).copy()
    v = np.array([4.0, -1.0, 0.25])
    wind = np.zeros((3, nl, 3, 3))
    wind[:, 0] = v[:, None, None]
    wind[:, 1:] = 7.0
    cw = dict(x0=0.0, y0=0.0, dx=200.0, dy=200.0, hagl=hagl, wind=wind, z0=z0)
    u0 = coupling.interp_wind(X, Y, Z, cw)
    below = zeta < h1
    above = zeta >= 40.0
    assert below.any() and above.any()
    fac = np.log(zeta[below] / z0) / math.log(h1 / z0)
    for d in range(3):
        assert np.allclose(u0[d][below], v[d] * fac, rtol=1e-13, atol=1e-13)
        assert np.allclose(u0[d][above], 7.0, rtol=1e-14, atol=0)
    # the closed form at the geometric mean of z0 and h1 is one half
    assert coupling.column_profile([h1, 30.0], np.array([[2.0, 5.0]]), math.sqrt(z0 * h1), z0)[0] \
        == pytest.approx(1.0, rel=1e-14)
    assert coupling.column_profile([h1, 30.0], np.array([[2.0, 5.0]]), 0.5 * z0, z0)[0] == 0.0


def test_positions_outside_the_coarse_grid_take_the_edge_columns():
    X, Y, Z = _grid(nx=6, ny=6)
    ncx = ncy = 3
    hagl = np.broadcast_to((0.5 * 1.5 ** np.arange(8))[:, None, None], (8, ncy, ncx)).copy()
    wind = np.zeros((3, 8, ncy, ncx))
    wind[0] = np.array([1.0, 2.0, 3.0])[None, None, :]   # varies along x only
    wind[1] = np.array([5.0, 6.0, 9.0])[None, :, None]   # varies along y only
    # coarse columns at x, y = 40, 60, 80 m: centres at x < 40 clamp to the first column
    cw = dict(x0=40.0, y0=40.0, dx=20.0, dy=20.0, hagl=hagl, wind=wind, z0=0.1)
    c, _ = coupling.heights_above_ground(X, Y, Z)
    u0 = coupling.interp_wind(X, Y, Z, cw)
    lo, hi = c[0] <= 40.0, c[0] >= 80.0
    assert np.allclose(u0[0][lo], 1.0, rtol=1e-14, atol=0)
    assert np.allclose(u0[0][hi], 3.0, rtol=1e-14, atol=0)
    lo, hi = c[1] <= 40.0, c[1] >= 80.0
    assert np.allclose(u0[1][lo], 5.0, rtol=1e-14, atol=0)
    assert np.allclose(u0[1][hi], 9.0, rtol=1e-14, atol=0)
    mid = (c[0] > 40.0) & (c[0] < 60.0)
    assert np.allclose(u0[0][mid], 1.0 + (c[0][mid] - 40.0) / 20.0, rtol=1e-14)


def test_surface_wind_linear_between_centres_log_below_constant_above():
    X, Y, Z = _grid(nz=5)
    _, zeta = coupling.heights_above_ground(X, Y, Z)
    a, b = 1.5, 0.2
    u = np.zeros((3,) + zeta.shape)
    u[0] = a + b * zeta
    u[1] = -2.0 * (a + b * zeta)
    H = 0.5 * (zeta[1] + zeta[2]).mean()
    assert np.all((zeta[1] <= H) & (H < zeta[2]))
    out = coupling.surface_wind(X, Y, Z, u, H, 0.1)
    assert np.allclose(out[0], a + b * H, rtol=1e-13)
    assert np.allclose(out[1], -2.0 * (a + b * H), rtol=1e-13)
    h_low = 0.5 * zeta[0].min()
    out = coupling.surface_wind(X, Y, Z, u, h_low, 0.1)
    ref = u[0, 0] * np.log(h_low / 0.1) / np.log(zeta[0] / 0.1)
    assert np.allclose(out[0], ref, rtol=1e-13)
    out = coupling.surface_wind(X, Y, Z, u, 1e4, 0.1)
    assert np.all(out[0] == u[0, -1]) and np.all(out[1] == u[1, -1])


def test_coarse_wind_generator_shapes_and_levels():
    cw = inputs.coarse_wind(3000.0, 2000.0, spacing=600.0, nl=20)
    nl, ncy, ncx = cw["hagl"].shape
    assert (nl, ncx, ncy) == (20, 7, 6)
    assert cw["wind"].shape == (3, 20, 6, 7)
    assert np.all(np.diff(cw["hagl"], axis=0) > 0) and cw["hagl"].min() > cw["z0"]
    assert cw["x0"] + cw["dx"] * (ncx - 1) >= 3000.0 and cw["x0"] <= 0.0
