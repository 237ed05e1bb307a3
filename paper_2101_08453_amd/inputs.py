"""Seeded synthetic inputs for the mass-consistent wind solve.

This module builds terrain-following hexahedral grids, initial wind fields
u0 and penalty constants for the workloads the solver is measured on.  It
holds none of the method's arithmetic (no shape functions, quadrature,
stiffness, multigrid or recovery): both the FP64 CPU checker and the GPU
path take their inputs from here, and nothing else is shared between them.

Conventions (Sec. 2 of Mandel et al., "Simple finite elements and multigrid
for efficient mass-consistent wind downscaling..."):

* Node arrays X, Y, Z have shape (nz+1, ny+1, nx+1), x fastest.  Node
  (i, j, k) sits at X[k, j, i], Y[k, j, i], Z[k, j, i].
* The wind is represented at element centres (Sec. 2, last paragraph), so
  u0 has shape (3, nz, ny, nx): components (u, v, w) of element (i, j, k).
* Grids are terrain following: Z = z_s(x, y) + zeta_k with zeta_0 = 0 and
  layer thicknesses first * ratio**m, horizontally uniform spacing dx, dy.
* The log wind profile S(z) = S_ref * ln(z / 0.1) / ln(10 / 0.1) is taken at
  the height above ground of each element centre, (zeta_k + zeta_{k+1}) / 2.
* Gamma (the surface where u.n = 0 is imposed) is given as a bit mask of
  grid faces: bit 0 bottom (k = 0), bit 1 top (k = nz), bit 2 x-low (i = 0),
  bit 3 x-high (i = nx), bit 4 y-low (j = 0), bit 5 y-high (j = ny).  The
  paper's setting is Gamma = bottom.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA_BOTTOM = 1
GAMMA_TOP = 2
GAMMA_XLO = 4
GAMMA_XHI = 8
GAMMA_YLO = 16
GAMMA_YHI = 32
GAMMA_ALL = 63


@dataclasses.dataclass
class Problem:
    """One solve: grid node coordinates, initial wind, penalties, Gamma."""

    name: str
    X: np.ndarray  # (nz+1, ny+1, nx+1) float64
    Y: np.ndarray
    Z: np.ndarray
    u0: np.ndarray  # (3, nz, ny, nx) float64
    a: np.ndarray  # (3,) float64 penalty constants a_1..a_3
    gamma: int = GAMMA_BOTTOM
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def dims(self):
        nzp, nyp, nxp = self.X.shape
        return nxp - 1, nyp - 1, nzp - 1

    @property
    def n_nodes(self):
        return int(self.X.size)


def vertical_levels(nz, first=5.0, ratio=1.2):
    """Heights above ground of the node planes: 0, then thicknesses first*ratio**m."""
    th = first * ratio ** np.arange(nz, dtype=np.float64)
    return np.concatenate([[0.0], np.cumsum(th)])


def log_profile(z, s_ref):
    """Neutral log-law speed with roughness 0.1 m, equal to s_ref at 10 m."""
    return s_ref * np.log(np.asarray(z) / 0.1) / math.log(10.0 / 0.1)


def terrain_grid(zs, zeta, dx, dy):
    """Node coordinates of the terrain-following grid Z = z_s + zeta_k."""
    nyp, nxp = zs.shape
    nzp = zeta.shape[0]
    x = dx * np.arange(nxp, dtype=np.float64)
    y = dy * np.arange(nyp, dtype=np.float64)
    X = np.broadcast_to(x[None, None, :], (nzp, nyp, nxp)).copy()
    Y = np.broadcast_to(y[None, :, None], (nzp, nyp, nxp)).copy()
    Z = zs[None, :, :] + zeta[:, None, None]
    return X, Y, np.ascontiguousarray(Z)


def centre_heights(zeta):
    """Height above ground of element centres in each layer."""
    return 0.5 * (zeta[:-1] + zeta[1:])


def gaussian_hills(nx, ny, dx, dy, heights, widths, cx, cy):
    """Sum of isotropic Gaussian hills sampled at the nodes."""
    x = dx * np.arange(nx + 1, dtype=np.float64)
    y = dy * np.arange(ny + 1, dtype=np.float64)
    zs = np.zeros((ny + 1, nx + 1))
    for h, w, x0, y0 in zip(heights, widths, cx, cy):
        gx = np.exp(-((x - x0) ** 2) / (2.0 * w * w))
        gy = np.exp(-((y - y0) ** 2) / (2.0 * w * w))
        zs += h * gy[:, None] * gx[None, :]
    return zs


def fractal_terrain(nx, ny, relief, rng, slope=1.75):
    """Power-law random terrain on the (ny+1, nx+1) node grid.

    White N(0,1) noise is filtered in Fourier space by |k|**(-slope), the
    k = 0 mode removed, and the result rescaled to [0, relief] metres.
    slope = 1.75 gives a 1D radial spectrum E(k) ~ k**-2.5.
    """
    noise = rng.standard_normal((ny + 1, nx + 1))
    F = np.fft.rfft2(noise)
    ky = np.fft.fftfreq(ny + 1)[:, None]
    kx = np.fft.rfftfreq(nx + 1)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    k[0, 0] = 1.0
    F *= k ** (-slope)
    F[0, 0] = 0.0
    zs = np.fft.irfft2(F, s=(ny + 1, nx + 1))
    zs -= zs.min()
    zs *= relief / zs.max()
    return zs


def _log_wind(nx, ny, nz, zeta, s_ref, theta):
    """u0 = S(z)(cos theta, sin theta, 0) at element centres; theta scalar or (nx,) array."""
    zc = centre_heights(zeta)
    s = log_profile(zc, s_ref)[:, None, None]
    th = np.broadcast_to(np.asarray(theta, dtype=np.float64), (nx,))[None, None, :]
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = s * np.cos(th)
    u0[1] = s * np.sin(th)
    return u0


def c1(seed=1):
    """32x32x8, dx 30 m, one Gaussian hill (200 m, width 250 m) at the centre,
    westerly log profile (5 m/s at 10 m) plus N(0, 0.2) noise, a = (1,1,1)."""
    nx = ny = 32
    nz = 8
    dx = 30.0
    rng = np.random.default_rng(seed)
    zeta = vertical_levels(nz)
    zs = gaussian_hills(nx, ny, dx, dx, [200.0], [250.0], [480.0], [480.0])
    X, Y, Z = terrain_grid(zs, zeta, dx, dx)
    u0 = _log_wind(nx, ny, nz, zeta, 5.0, 0.0)
    u0 += rng.normal(0.0, 0.2, size=u0.shape)
    return Problem("32x32x8 gaussian hill", X, Y, Z, u0, np.array([1.0, 1.0, 1.0]))


def hills_problem(nx, ny, nz, n_hills, seed, a=(1.0, 1.0, 1.0), noise=0.0, s_ref=8.0,
                  dx=30.0, name=None):
    """Seeded sum of Gaussian hills (heights U(50,400) m, widths U(100,1500) m,
    centres uniform over the domain), log-profile wind of random direction."""
    rng = np.random.default_rng(seed)
    Lx, Ly = nx * dx, ny * dx
    h = rng.uniform(50.0, 400.0, n_hills)
    w = rng.uniform(100.0, 1500.0, n_hills)
    cx = rng.uniform(0.0, Lx, n_hills)
    cy = rng.uniform(0.0, Ly, n_hills)
    theta = rng.uniform(0.0, 2.0 * math.pi)
    zeta = vertical_levels(nz)
    zs = gaussian_hills(nx, ny, dx, dx, h, w, cx, cy)
    X, Y, Z = terrain_grid(zs, zeta, dx, dx)
    u0 = _log_wind(nx, ny, nz, zeta, s_ref, theta)
    if noise > 0.0:
        u0 += rng.normal(0.0, noise, size=u0.shape)
    return Problem(name or f"{nx}x{ny}x{nz} {n_hills} hills", X, Y, Z, u0,
                   np.asarray(a, dtype=np.float64), meta={"theta": theta})


def c2(seed=2, n=256, nz=16):
    """256x256x16, 40 hills, log profile 8 m/s of random direction, N(0,0.5) noise."""
    return hills_problem(n, n, nz, 40, seed, noise=0.5,
                         name=f"{n}x{n}x{nz} 40 gaussian hills")


def fractal_problem(nx, ny, nz, relief, seed, a=(1.0, 1.0, 1.0), veer=False,
                    s_ref=8.0, dx=30.0, name=None):
    """Fractal terrain; log profile wind, either of random direction or with a
    +-30 degree sinusoidal veer of 20 km wavelength along x."""
    rng = np.random.default_rng(seed)
    zeta = vertical_levels(nz)
    zs = fractal_terrain(nx, ny, relief, rng)
    X, Y, Z = terrain_grid(zs, zeta, dx, dx)
    if veer:
        xc = dx * (np.arange(nx) + 0.5)
        theta = (math.pi / 6.0) * np.sin(2.0 * math.pi * xc / 20000.0)
    else:
        theta = rng.uniform(0.0, 2.0 * math.pi)
    u0 = _log_wind(nx, ny, nz, zeta, s_ref, theta)
    return Problem(name or f"{nx}x{ny}x{nz} fractal", X, Y, Z, u0,
                   np.asarray(a, dtype=np.float64))


def c3(seed=3, n=3000, nz=15):
    """3000x3000x15 (90 km at 30 m), fractal terrain of 800 m relief, veering
    log-profile wind, a = (1, 1, 10)."""
    return fractal_problem(n, n, nz, 800.0, seed, a=(1.0, 1.0, 10.0), veer=True,
                           name=f"{n}x{n}x{nz} fractal 800 m, a3=10")


def c3_perturbation(shape, seed=33, sigma=0.3):
    """The next-time-step wind perturbation N(0, 0.3) on every component."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=shape)


def c4_member(m, seed_base=400):
    """Member m of the 64-member ensemble: size from {64,128,256,512}^2 x {8,12,16},
    1-10 hills, log profile without noise, a3 ~ U(1, 10)."""
    rng = np.random.default_rng(seed_base + m)
    n = int(rng.choice([64, 128, 256, 512]))
    nz = int(rng.choice([8, 12, 16]))
    n_hills = int(rng.integers(1, 11))
    a3 = float(rng.uniform(1.0, 10.0))
    sub = int(rng.integers(0, 2**31 - 1))
    return hills_problem(n, n, nz, n_hills, sub, a=(1.0, 1.0, a3),
                         name=f"member {m}: {n}x{n}x{nz}, a3={a3:.2f}")


def c4(count=64):
    return [c4_member(m) for m in range(count)]


def c5(seed=5, n=512, nz=15):
    """512x512x15 fractal terrain of 500 m relief, log profile of random direction."""
    return fractal_problem(n, n, nz, 500.0, seed, name=f"{n}x{n}x{nz} fractal 500 m")


def coarse_wind(Lx, Ly, spacing=600.0, nl=30, seed=60, s_ref=8.0, first=25.0, ratio=1.15,
                z0=0.1, noise=0.3):
    """A stand-in for the atmospheric model's wind over a Lx x Ly domain:
    columns every `spacing` m from -spacing/2 (the domain lies inside the
    column grid), nl terrain-following levels from `first` m above ground
    growing by `ratio`, scaled per column by a smooth factor in [0.9, 1.1];
    log-law speed (s_ref at 10 m, roughness z0) turning 30 degrees from the
    ground to the top and veering +-20 degrees across the domain, vertical
    component 0, plus N(0, noise) in every component.
    Returns dict(x0, y0, dx, dy, hagl (nl, ncy, ncx), wind (3, nl, ncy, ncx), z0)."""
    rng = np.random.default_rng(seed)
    ncx = int(math.ceil(Lx / spacing)) + 2
    ncy = int(math.ceil(Ly / spacing)) + 2
    x0 = y0 = -0.5 * spacing
    xs = x0 + spacing * np.arange(ncx)
    ys = y0 + spacing * np.arange(ncy)
    base = first * np.cumprod(np.concatenate([[1.0], np.full(nl - 1, ratio)]))
    phase = rng.uniform(0.0, 2.0 * math.pi, 2)
    fac = 1.0 + 0.1 * np.sin(2.0 * math.pi * xs[None, :] / 7000.0 + phase[0]) \
        * np.cos(2.0 * math.pi * ys[:, None] / 9000.0 + phase[1])
    hagl = base[:, None, None] * fac[None]
    speed = s_ref * np.log(hagl / z0) / math.log(10.0 / z0)
    turn = (math.pi / 6.0) * (hagl - hagl[0]) / (hagl[-1] - hagl[0])
    veer = (math.pi / 9.0) * np.sin(2.0 * math.pi * xs / max(Lx, spacing))[None, None, :]
    theta = rng.uniform(0.0, 2.0 * math.pi) + turn + veer
    wind = np.zeros((3, nl, ncy, ncx))
    wind[0] = speed * np.cos(theta)
    wind[1] = speed * np.sin(theta)
    wind += rng.normal(0.0, noise, size=wind.shape)
    return {"x0": x0, "y0": y0, "dx": spacing, "dy": spacing,
            "hagl": np.ascontiguousarray(hagl), "wind": np.ascontiguousarray(wind), "z0": z0}


def fire_mask(nx, ny, dx=30.0, dy=30.0, seed=55):
    """Elliptical fire-perimeter mask over the bottom-layer element centres, (ny, nx) bool."""
    rng = np.random.default_rng(seed)
    Lx, Ly = nx * dx, ny * dy
    cx = rng.uniform(0.25, 0.75) * Lx
    cy = rng.uniform(0.25, 0.75) * Ly
    sa = rng.uniform(0.05, 0.2) * Lx
    sb = rng.uniform(0.05, 0.2) * Ly
    ang = rng.uniform(0.0, math.pi)
    xc = dx * (np.arange(nx) + 0.5)
    yc = dy * (np.arange(ny) + 0.5)
    Xc, Yc = np.meshgrid(xc, yc)
    px = (Xc - cx) * math.cos(ang) + (Yc - cy) * math.sin(ang)
    py = -(Xc - cx) * math.sin(ang) + (Yc - cy) * math.cos(ang)
    return (px / sa) ** 2 + (py / sb) ** 2 <= 1.0


def random_directions(shape, count, seed=56):
    """count N(0,1) directions of the given shape (for finite-difference checks)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((count,) + tuple(shape))


def box_problem(nx, ny, nz, hx=1.0, hy=1.0, hz=1.0, a=(1.0, 1.0, 1.0), seed=0,
                gamma=GAMMA_BOTTOM, z_ratio=1.0):
    """Flat box grid (uniform, or with geometric vertical stretching) with a
    random N(0,1) wind: the setting of textbook Poisson multigrid checks."""
    rng = np.random.default_rng(seed)
    zeta = vertical_levels(nz, first=hz, ratio=z_ratio)
    zs = np.zeros((ny + 1, nx + 1))
    X, Y, Z = terrain_grid(zs, zeta, hx, hy)
    u0 = rng.standard_normal((3, nz, ny, nx))
    return Problem(f"box {nx}x{ny}x{nz}", X, Y, Z, u0, np.asarray(a, dtype=np.float64),
                   gamma=gamma)


def distorted_problem(nx, ny, nz, seed=0, amp=0.2, a=(1.0, 1.0, 1.0), gamma=GAMMA_BOTTOM):
    """Unit-spacing grid whose nodes are all randomly displaced by up to amp
    (kept < 0.25 so that every element stays right-handed): a general
    isoparametric mesh, not terrain following."""
    rng = np.random.default_rng(seed)
    zeta = np.arange(nz + 1, dtype=np.float64)
    zs = np.zeros((ny + 1, nx + 1))
    X, Y, Z = terrain_grid(zs, zeta, 1.0, 1.0)
    X = X + rng.uniform(-amp, amp, X.shape)
    Y = Y + rng.uniform(-amp, amp, Y.shape)
    Z = Z + rng.uniform(-amp, amp, Z.shape)
    u0 = rng.standard_normal((3, nz, ny, nx))
    return Problem(f"distorted {nx}x{ny}x{nz}", X, Y, Z, u0, np.asarray(a, dtype=np.float64),
                   gamma=gamma)


CONFIGS = {
    "c1": c1,
    "c2": c2,
    "c3": c3,
    "c5": c5,
}
