"""Python binding of libmcwind (ctypes).  Argument marshalling only: every
numerical step runs in the library's HIP kernels on the GPU.

Tensors are torch tensors on the ROCm device (PyTorch provides device memory
and streams).  Layouts follow include/mcwind.h:

* node arrays X, Y, Z, lambda: float64, shape (nz+1, ny+1, nx+1), x fastest;
* element arrays u0, u: float64, shape (3, nz, ny, nx).

The library must have been built (python -m paper_2101_08453_amd.build);
importing this module on a machine without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcwind.so")

MCW_OK = 0
STATUS_NAMES = ["MCW_OK", "MCW_INVALID_ARG", "MCW_BAD_GEOMETRY", "MCW_SINGULAR", "MCW_NONFINITE",
                "MCW_NOT_CONVERGED", "MCW_OOM", "MCW_HIP_ERROR"]
FP64 = 0
FP32_REFINE = 1
PRECISIONS = {"fp64": FP64, "fp32_refine": FP32_REFINE}
RULES = {"operator": 0, "literal": 1, "full": 2}
MERGE_SPACINGS = {"level": 0, "coarsened": 1}
SMOOTHERS = {"point": 0, "line": 1}
MAX_LEVELS = 24
HISTORY = 64

GAMMA_BOTTOM, GAMMA_TOP, GAMMA_XLO, GAMMA_XHI, GAMMA_YLO, GAMMA_YHI = 1, 2, 4, 8, 16, 32


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                ("a", ctypes.c_double * 3), ("gamma_faces", ctypes.c_uint32)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("max_cycles", ctypes.c_int32), ("nu_pre", ctypes.c_int32),
                ("nu_post", ctypes.c_int32), ("inner_cycles", ctypes.c_int32),
                ("coarsen_rule", ctypes.c_int32), ("coarse_direct_max", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("autotune", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("stencil_fp16", ctypes.c_int32), ("merge_spacing", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class Info(ctypes.Structure):
    _fields_ = [("outer_steps", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("rel_divergence", ctypes.c_double),
                ("rho", ctypes.c_double), ("f_norm", ctypes.c_double),
                ("n_levels", ctypes.c_int32), ("level_dims", (ctypes.c_int32 * 3) * MAX_LEVELS),
                ("n_history", ctypes.c_int32), ("history", ctypes.c_double * HISTORY),
                ("ms_total", ctypes.c_float), ("ms_rhs", ctypes.c_float),
                ("ms_cycles", ctypes.c_float), ("ms_outer", ctypes.c_float),
                ("ms_finish", ctypes.c_float), ("status", ctypes.c_int32)]

    def to_dict(self):
        return {
            "outer_steps": self.outer_steps, "cycles": self.cycles,
            "rel_residual": self.rel_residual, "rel_divergence": self.rel_divergence,
            "rho": self.rho, "f_norm": self.f_norm,
            "levels": [tuple(self.level_dims[l]) for l in range(self.n_levels)],
            "history": [self.history[i] for i in range(self.n_history)],
            "ms_total": self.ms_total, "ms_rhs": self.ms_rhs, "ms_cycles": self.ms_cycles,
            "ms_outer": self.ms_outer, "ms_finish": self.ms_finish,
            "status": STATUS_NAMES[self.status] if 0 <= self.status < len(STATUS_NAMES) else str(self.status),
        }


class CoarseWind(ctypes.Structure):
    _fields_ = [("ncx", ctypes.c_int32), ("ncy", ctypes.c_int32), ("nl", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("z0", ctypes.c_double), ("hagl", ctypes.c_void_p),
                ("wind", ctypes.c_void_p)]


class MCWError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.status_name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{self.status_name}: {message}")


_lib = None
P = ctypes.c_void_p
H = ctypes.c_void_p
I32 = ctypes.c_int32

# name -> (restype, argtypes), mirrors include/mcwind.h
SIGNATURES = {
    "mcw_default_options": (None, [ctypes.POINTER(Options)]),
    "mcw_create": (I32, [ctypes.POINTER(GridDesc), ctypes.POINTER(Options), P, ctypes.POINTER(H)]),
    "mcw_destroy": (None, [H]),
    "mcw_set_tolerance": (I32, [H, ctypes.c_double, I32]),
    "mcw_solve": (I32, [H, P, P, P, ctypes.POINTER(Info)]),
    "mcw_solve_batch": (I32, [I32, ctypes.POINTER(H), ctypes.POINTER(P), ctypes.POINTER(P),
                              ctypes.POINTER(P), ctypes.POINTER(Info)]),
    "mcw_adjoint": (I32, [H, P, P, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Info)]),
    "mcw_apply_K": (I32, [H, P, P]),
    "mcw_rhs": (I32, [H, P, P]),
    "mcw_recover": (I32, [H, P, P, P]),
    "mcw_divergence": (I32, [H, P, P, P, ctypes.POINTER(ctypes.c_double)]),
    "mcw_divergence_noalloc": (I32, [ctypes.POINTER(GridDesc), P, P, P,
                                     ctypes.POINTER(ctypes.c_double), P]),
    "mcw_num_levels": (I32, [H]),
    "mcw_level_info": (I32, [H, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                             ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "mcw_get_stencil": (I32, [H, I32, I32, P]),
    "mcw_smooth": (I32, [H, I32, P, P, I32]),
    "mcw_residual": (I32, [H, I32, P, P, P]),
    "mcw_restrict": (I32, [H, I32, P, P]),
    "mcw_prolong": (I32, [H, I32, P, P]),
    "mcw_coarse_solve": (I32, [H, P, P]),
    "mcw_vcycle": (I32, [H, P, P]),
    "mcw_run_kernel": (I32, [H, I32, I32, I32]),
    "mcw_run_kernel_batch": (I32, [I32, ctypes.POINTER(H), I32, I32, ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(I32)]),
    "mcw_interp_wind": (I32, [H, ctypes.POINTER(CoarseWind), P]),
    "mcw_surface_wind": (I32, [H, P, ctypes.c_double, ctypes.c_double, P]),
    "mcw_tile_shape": (I32, [H, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "mcw_status_string": (ctypes.c_char_p, [I32]),
    "mcw_last_error": (ctypes.c_char_p, [H]),
}


def lib():
    """Load libmcwind.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2101_08453_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_options():
    o = Options()
    lib().mcw_default_options(ctypes.byref(o))
    return o


def _ptr(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """A set-up grid (mcw_create): hierarchy, operators and workspace on the GPU."""

    def __init__(self, X, Y, Z, a, gamma=GAMMA_BOTTOM, precision="fp32_refine", rtol=1e-8,
                 max_cycles=200, nu_pre=2, nu_post=2, inner_cycles=0, coarsen_rule="operator",
                 coarse_direct_max=1024, use_graph=True, verbose=False, autotune=True,
                 krylov=False, smoother="point", stencil_fp16=False, merge_spacing="level",
                 tune_cache=None):
        L = lib()
        self._h = H()
        nzp, nyp, nxp = X.shape
        self.nx, self.ny, self.nz = nxp - 1, nyp - 1, nzp - 1
        self.device = X.device
        node = (nzp, nyp, nxp)
        d = GridDesc()
        d.nx, d.ny, d.nz = self.nx, self.ny, self.nz
        d.X = _ptr(X, torch.float64, node, "X")
        d.Y = _ptr(Y, torch.float64, node, "Y")
        d.Z = _ptr(Z, torch.float64, node, "Z")
        a = [float(v) for v in a]
        d.a[0], d.a[1], d.a[2] = a
        d.gamma_faces = int(gamma)
        self.a = np.array(a)
        self.gamma = int(gamma)
        o = default_options()
        o.precision = PRECISIONS[precision]
        o.rtol = rtol
        o.max_cycles = max_cycles
        o.nu_pre, o.nu_post = nu_pre, nu_post
        o.inner_cycles = inner_cycles
        o.coarsen_rule = RULES[coarsen_rule]
        o.coarse_direct_max = coarse_direct_max
        o.use_graph = 1 if use_graph else 0
        o.autotune = 1 if autotune else 0
        o.krylov = 1 if krylov else 0
        o.smoother = SMOOTHERS[smoother]
        o.stencil_fp16 = 1 if stencil_fp16 else 0
        o.merge_spacing = MERGE_SPACINGS[merge_spacing]
        o.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
        o.verbose = 1 if (verbose or os.environ.get("MCW_LOG")) else 0
        self.precision = precision
        self.vdtype = torch.float32 if precision == "fp32_refine" else torch.float64
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        st = L.mcw_create(ctypes.byref(d), ctypes.byref(o), stream, ctypes.byref(self._h))
        if st != MCW_OK:
            raise MCWError(st, L.mcw_last_error(None).decode())

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mcw_destroy(self._h)
            self._h = H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != MCW_OK:
            raise MCWError(st, lib().mcw_last_error(self._h).decode())

    # ------------------------------------------------------------ shapes
    @property
    def node_shape(self):
        return (self.nz + 1, self.ny + 1, self.nx + 1)

    @property
    def elem_shape(self):
        return (3, self.nz, self.ny, self.nx)

    def level_shape(self, l):
        nx, ny, nz = self.level(l)["dims"]
        return (nz + 1, ny + 1, nx + 1)

    def _node(self, dtype=torch.float64, l=0):
        return torch.zeros(self.level_shape(l), dtype=dtype, device=self.device)

    # ------------------------------------------------------------ solve
    def set_tolerance(self, rtol, max_cycles=200):
        self._check(lib().mcw_set_tolerance(self._h, float(rtol), int(max_cycles)))

    def solve(self, u0, lam=None, want_u=True, check=True):
        """(lambda, u, info).  lam, if given, is the warm start and is overwritten."""
        if lam is None:
            lam = self._node()
        u = torch.empty(self.elem_shape, dtype=torch.float64, device=self.device) if want_u else None
        info = Info()
        st = lib().mcw_solve(self._h, _ptr(u0, torch.float64, self.elem_shape, "u0"),
                             _ptr(lam, torch.float64, self.node_shape, "lambda"),
                             _ptr(u, torch.float64, self.elem_shape, "u") if want_u else None,
                             ctypes.byref(info))
        out = info.to_dict()
        out["status"] = STATUS_NAMES[st]
        if check:
            self._check(st)
        return lam, u, out

    def adjoint(self, lam, g_u):
        """(dL/du0 float32, dL/da float64[3], info) for dL/du = g_u."""
        d_u0 = torch.empty(self.elem_shape, dtype=torch.float32, device=self.device)
        d_a = (ctypes.c_double * 3)()
        info = Info()
        self._check(lib().mcw_adjoint(self._h, _ptr(lam, torch.float64, self.node_shape, "lambda"),
                                      _ptr(g_u, torch.float64, self.elem_shape, "g_u"),
                                      _ptr(d_u0, torch.float32, self.elem_shape, "dL_du0"), d_a,
                                      ctypes.byref(info)))
        return d_u0, np.array(list(d_a)), info.to_dict()

    # ------------------------------------------------------------ single steps
    def apply_K(self, x):
        y = self._node()
        self._check(lib().mcw_apply_K(self._h, _ptr(x, torch.float64, self.node_shape, "x"),
                                      _ptr(y, torch.float64, self.node_shape, "y")))
        return y

    def rhs(self, u0):
        f = self._node()
        self._check(lib().mcw_rhs(self._h, _ptr(u0, torch.float64, self.elem_shape, "u0"),
                                  _ptr(f, torch.float64, self.node_shape, "f")))
        return f

    def recover(self, u0, lam):
        u = torch.empty(self.elem_shape, dtype=torch.float64, device=self.device)
        self._check(lib().mcw_recover(self._h, _ptr(u0, torch.float64, self.elem_shape, "u0"),
                                      _ptr(lam, torch.float64, self.node_shape, "lambda"),
                                      _ptr(u, torch.float64, self.elem_shape, "u")))
        return u

    def divergence(self, u0, lam):
        D = self._node()
        rel = ctypes.c_double()
        self._check(lib().mcw_divergence(self._h, _ptr(u0, torch.float64, self.elem_shape, "u0"),
                                         _ptr(lam, torch.float64, self.node_shape, "lambda"),
                                         _ptr(D, torch.float64, self.node_shape, "D"),
                                         ctypes.byref(rel)))
        return D, rel.value

    # ------------------------------------------------------------ around the solve
    def interp_wind(self, cw):
        """u0 (3, nz, ny, nx) at the element centres from a coarse wind given as a
        dict with x0, y0, dx, dy, z0 (floats) and device float64 tensors hagl
        (nl, ncy, ncx) and wind (3, nl, ncy, ncx)."""
        hagl, wind = cw["hagl"], cw["wind"]
        nl, ncy, ncx = hagl.shape
        c = CoarseWind()
        c.ncx, c.ncy, c.nl = ncx, ncy, nl
        c.x0, c.y0, c.dx, c.dy, c.z0 = (float(cw[k]) for k in ("x0", "y0", "dx", "dy", "z0"))
        c.hagl = _ptr(hagl, torch.float64, (nl, ncy, ncx), "hagl")
        c.wind = _ptr(wind, torch.float64, (3, nl, ncy, ncx), "wind")
        u0 = torch.empty(self.elem_shape, dtype=torch.float64, device=self.device)
        self._check(lib().mcw_interp_wind(self._h, ctypes.byref(c),
                                          _ptr(u0, torch.float64, self.elem_shape, "u0")))
        return u0

    def surface_wind(self, u, height, z0=0.1):
        """(2, ny, nx): horizontal wind at `height` above ground over each column."""
        uv = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=self.device)
        self._check(lib().mcw_surface_wind(self._h, _ptr(u, torch.float64, self.elem_shape, "u"),
                                           float(height), float(z0),
                                           _ptr(uv, torch.float64, (2, self.ny, self.nx), "uv")))
        return uv

    def num_levels(self):
        return int(lib().mcw_num_levels(self._h))

    def level(self, l):
        dims = (I32 * 3)()
        ch = I32()
        nk = I32()
        keep = (I32 * 8192)()
        self._check(lib().mcw_level_info(self._h, l, dims, ctypes.byref(ch), keep, ctypes.byref(nk)))
        return {"dims": tuple(dims), "coarsen_h": bool(ch.value),
                "keep_z": [keep[i] for i in range(nk.value)]}

    def levels(self):
        return [self.level(l) for l in range(self.num_levels())]

    def tile_rows(self, l):
        """Tile rows per block the autotuner chose for level l: (colour pass, residual)."""
        gs, res = I32(), I32()
        self._check(lib().mcw_tile_shape(self._h, l, ctypes.byref(gs), ctypes.byref(res)))
        return gs.value, res.value

    def stencil(self, l, precision=None):
        """(27, NZ, NY, NX) coefficients of level l in natural node order."""
        precision = precision or self.precision
        dt = torch.float64 if precision == "fp64" else torch.float32
        out = torch.empty((27,) + self.level_shape(l), dtype=dt, device=self.device)
        self._check(lib().mcw_get_stencil(self._h, l, PRECISIONS[precision],
                                          ctypes.c_void_p(out.data_ptr())))
        return out

    def smooth(self, l, x, f, sweeps=1):
        """sweeps > 0 forward Gauss-Seidel sweeps, < 0 reverse (adjoint) sweeps."""
        s = self.level_shape(l)
        self._check(lib().mcw_smooth(self._h, l, _ptr(x, self.vdtype, s, "x"),
                                     _ptr(f, self.vdtype, s, "f"), sweeps))
        return x

    def residual(self, l, x, f):
        s = self.level_shape(l)
        r = torch.empty(s, dtype=self.vdtype, device=self.device)
        self._check(lib().mcw_residual(self._h, l, _ptr(x, self.vdtype, s, "x"),
                                       _ptr(f, self.vdtype, s, "f"), _ptr(r, self.vdtype, s, "r")))
        return r

    def restrict(self, l, r):
        rc = torch.empty(self.level_shape(l + 1), dtype=self.vdtype, device=self.device)
        self._check(lib().mcw_restrict(self._h, l, _ptr(r, self.vdtype, self.level_shape(l), "r"),
                                       _ptr(rc, self.vdtype, self.level_shape(l + 1), "rc")))
        return rc

    def prolong(self, l, e, x):
        self._check(lib().mcw_prolong(self._h, l, _ptr(e, self.vdtype, self.level_shape(l + 1), "e"),
                                      _ptr(x, self.vdtype, self.level_shape(l), "x")))
        return x

    def coarse_solve(self, r):
        L = self.num_levels() - 1
        e = torch.zeros(self.level_shape(L), dtype=self.vdtype, device=self.device)
        self._check(lib().mcw_coarse_solve(self._h, _ptr(r, self.vdtype, self.level_shape(L), "r"),
                                           _ptr(e, self.vdtype, self.level_shape(L), "e")))
        return e

    KERNELS = {"smooth": 0, "residual": 1, "restrict": 2, "prolong": 3, "residual64": 4}

    def run_kernel(self, l, kernel, reps=1):
        """Launch one multigrid kernel `reps` times on level l's own buffers (timing)."""
        self._check(lib().mcw_run_kernel(self._h, l, self.KERNELS[kernel], reps))

    def vcycle(self, x, f):
        s = self.level_shape(0)
        self._check(lib().mcw_vcycle(self._h, _ptr(x, self.vdtype, s, "x"),
                                     _ptr(f, self.vdtype, s, "f")))
        return x


def solve_batch(grids, u0s, lams=None, want_u=True, check=True):
    """Solve several problems together (mcw_solve_batch); returns (lams, us, infos, status).

    want_u: True / False for every member, or one bool per member (a member
    without it gets None in us and skips recovery).  With check=False a failing
    member does not raise: status names the first failing member's status and
    each member's own outcome is in its info."""
    m = len(grids)
    if lams is None:
        lams = [g._node() for g in grids]
    per = [bool(w) for w in want_u] if isinstance(want_u, (list, tuple)) else [bool(want_u)] * m
    if len(per) != m:
        raise ValueError("want_u needs one entry per member")
    us = [torch.empty(g.elem_shape, dtype=torch.float64, device=g.device) if w else None
          for g, w in zip(grids, per)]
    hs = (H * m)(*[g._h.value for g in grids])
    pu0 = (P * m)(*[_ptr(u, torch.float64, g.elem_shape, "u0").value for g, u in zip(grids, u0s)])
    pl = (P * m)(*[_ptr(l, torch.float64, g.node_shape, "lambda").value for g, l in zip(grids, lams)])
    pu = (P * m)(*[u.data_ptr() if u is not None else None for u in us]) if any(per) else None
    if not any(per):
        us = None
    infos = (Info * m)()
    st = lib().mcw_solve_batch(m, hs, pu0, pl, pu, infos)
    if check and st != MCW_OK:
        raise MCWError(st, lib().mcw_last_error(None).decode())
    return lams, us, [infos[i].to_dict() for i in range(m)], STATUS_NAMES[st]


def divergence_noalloc(X, Y, Z, a, u0, lam, gamma=GAMMA_BOTTOM, want_rel=True):
    """(D, rel) by mcw_divergence_noalloc: the divergence check on a grid given by
    its node coordinates, with no handle and no device allocation by the library
    (D is allocated here, by torch)."""
    nzp, nyp, nxp = X.shape
    node = (nzp, nyp, nxp)
    elem = (3, nzp - 1, nyp - 1, nxp - 1)
    d = GridDesc()
    d.nx, d.ny, d.nz = nxp - 1, nyp - 1, nzp - 1
    d.X = _ptr(X, torch.float64, node, "X")
    d.Y = _ptr(Y, torch.float64, node, "Y")
    d.Z = _ptr(Z, torch.float64, node, "Z")
    d.a[0], d.a[1], d.a[2] = (float(v) for v in a)
    d.gamma_faces = int(gamma)
    D = torch.empty(node, dtype=torch.float64, device=X.device)
    rel = ctypes.c_double(float("nan"))
    stream = ctypes.c_void_p(torch.cuda.current_stream(X.device).cuda_stream)
    st = lib().mcw_divergence_noalloc(ctypes.byref(d), _ptr(u0, torch.float64, elem, "u0"),
                                      _ptr(lam, torch.float64, node, "lambda"),
                                      _ptr(D, torch.float64, node, "D"),
                                      ctypes.byref(rel) if want_rel else None, stream)
    if st != MCW_OK:
        raise MCWError(st, lib().mcw_last_error(None).decode())
    return D, (rel.value if want_rel else None)


def run_kernel_batch(grids, kernel, reps=1):
    """Launch one batched phase over the finest level of every grid `reps` times
    (mcw_run_kernel_batch; "smooth" = one sweep, "residual"), for timing.
    Returns (device ms per repetition, launches per repetition and format)."""
    m = len(grids)
    hs = (H * m)(*[g._h.value for g in grids])
    ms, launches = ctypes.c_float(0.0), I32(0)
    st = lib().mcw_run_kernel_batch(m, hs, {"smooth": 0, "residual": 1}[kernel], int(reps),
                                    ctypes.byref(ms), ctypes.byref(launches))
    if st != MCW_OK:
        raise MCWError(st, lib().mcw_last_error(None).decode())
    return ms.value, launches.value


def grid_from_problem(prob, device="cuda", **kw):
    """Upload a paper_2101_08453_amd.inputs.Problem and set up its Grid; returns (grid, u0)."""
    X = torch.from_numpy(prob.X).to(device)
    Y = torch.from_numpy(prob.Y).to(device)
    Z = torch.from_numpy(prob.Z).to(device)
    u0 = torch.from_numpy(np.ascontiguousarray(prob.u0)).to(device)
    torch.cuda.synchronize()
    g = Grid(X, Y, Z, prob.a, gamma=prob.gamma, **kw)
    return g, u0


class WindSolve(torch.autograd.Function):
    """u = mass-consistent wind of u0 on `grid`, differentiable in u0 and a.

    forward(u0, a, grid): a is a (3,) float64 tensor equal to the grid's
    penalties (the grid is set up for them; it is an input only so that
    autograd can return dL/da).  backward runs the hand-written adjoint.
    """

    @staticmethod
    def forward(ctx, u0, a, grid):
        a_host = np.asarray(a.detach().cpu().numpy(), dtype=np.float64).reshape(-1)
        if a_host.shape != (3,) or not np.array_equal(a_host, grid.a):
            raise ValueError(f"a = {a_host.tolist()} differs from the grid's penalties "
                             f"{grid.a.tolist()}: set up a Grid for these penalties")
        lam, u, info = grid.solve(u0.detach().contiguous())
        ctx.grid = grid
        ctx.save_for_backward(lam)
        ctx.a_dtype = a.dtype
        ctx.a_device = a.device
        return u

    @staticmethod
    def backward(ctx, g_u):
        (lam,) = ctx.saved_tensors
        d_u0, d_a, _ = ctx.grid.adjoint(lam, g_u.contiguous().to(torch.float64))
        return (d_u0.to(torch.float64), torch.tensor(d_a, dtype=ctx.a_dtype, device=ctx.a_device),
                None)
