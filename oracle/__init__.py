"""FP64 CPU oracle for scattered-sounding gridding (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg are the only callers.  The product package
never imports this module, and this module imports nothing from the product.

Every function wraps ``liboracle.so`` built from ``auv_oracle.c`` (plain C, IEEE
double, ``-ffp-contract=off``).  See that file for the step-by-step definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "auv_oracle.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


@dataclass(frozen=True)
class Grid:
    """Pixel-centre grid: node (a, b) at (x0+(b+.5)dx, y0+(a+.5)dy)."""
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int

    def c(self) -> _Grid:
        return _Grid(self.x0, self.y0, self.dx, self.dy, self.nx, self.ny)

    def node_xy(self):
        xs = self.x0 + (np.arange(self.nx) + 0.5) * self.dx
        ys = self.y0 + (np.arange(self.ny) + 0.5) * self.dy
        return xs, ys


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.orc_bin_dims.argtypes = [P(_Grid), d, i32, P(i32), P(i32), P(i32)]
        lib.orc_bin.argtypes = [P(_Grid), vp, vp, vp, i64, d, i32, vp, vp,
                                P(i64), P(i64), P(i64)]
        lib.orc_idw.argtypes = [P(_Grid), vp, vp, vp, i64, d, d, i32, i32, i32,
                                vp, i64, vp, vp, vp, i32]
        lib.orc_idw_bounds.argtypes = [P(_Grid), vp, vp, vp, i64, d, i32, i32, vp, i64,
                                       vp, vp, i32]
        lib.orc_nearest.argtypes = [P(_Grid), vp, vp, vp, i64, d, i32, vp, i64,
                                    vp, vp, i32]
        lib.orc_bilinear.argtypes = [P(_Grid), vp, P(_Grid), vp, i32]
        lib.orc_bicubic.argtypes = [P(_Grid), vp, P(_Grid), vp, i32]
        lib.orc_kriging.argtypes = [P(_Grid), vp, P(_Grid), d, vp, i32]
        lib.orc_variogram.argtypes = [P(_Grid), vp, i32, vp, vp, vp, vp]
        lib.orc_fit_exponential.argtypes = [vp, vp, vp, i32, P(d), P(d)]
        for f in (lib.orc_bin_dims, lib.orc_bin, lib.orc_idw, lib.orc_idw_bounds, lib.orc_nearest,
                  lib.orc_bilinear, lib.orc_bicubic, lib.orc_kriging, lib.orc_variogram,
                  lib.orc_fit_exponential):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def bin_dims(grid: Grid, radius: float, bin_log2: int):
    lib = _load()
    nbx, nby, h = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.orc_bin_dims(ctypes.byref(grid.c()), radius, bin_log2,
                            ctypes.byref(nbx), ctypes.byref(nby), ctypes.byref(h)),
           "orc_bin_dims")
    return nbx.value, nby.value, h.value


def bin_points(grid: Grid, x, y, z, radius: float, bin_log2: int):
    """O4: returns (cell_start, perm, n_invalid, n_outside)."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    nbx, nby, _ = bin_dims(grid, radius, bin_log2)
    cs = np.zeros(nbx * nby + 1, dtype=np.int32)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    nb, ni, no = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.orc_bin(ctypes.byref(grid.c()), _ptr(x), _ptr(y), _ptr(z), n,
                       radius, bin_log2, _ptr(cs), _ptr(perm), ctypes.byref(nb),
                       ctypes.byref(ni), ctypes.byref(no)), "orc_bin")
    return cs, perm[: nb.value].copy(), ni.value, no.value


def idw(grid: Grid, x, y, z, radius: float, power: float = 2.0, min_pts: int = 1,
        max_pts: int = 0, bin_log2: int = -1, nodes=None, nthreads: int = 0):
    """O1: returns (z_out float64, cnt int32, nn int32); nodes=None -> [ny, nx]."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    if nodes is None:
        m = grid.nx * grid.ny
        nd = None
    else:
        nd = np.ascontiguousarray(nodes, dtype=np.int64)
        m = nd.shape[0]
    zo = np.empty(max(m, 1), dtype=np.float64)
    co = np.empty(max(m, 1), dtype=np.int32)
    no = np.empty(max(m, 1), dtype=np.int32)
    _check(lib.orc_idw(ctypes.byref(grid.c()), _ptr(x), _ptr(y), _ptr(z), n,
                       radius, power, min_pts, max_pts, bin_log2, _ptr(nd),
                       m if nd is not None else 0, _ptr(zo), _ptr(co), _ptr(no),
                       nthreads), "orc_idw")
    zo, co, no = zo[:m], co[:m], no[:m]
    if nodes is None:
        shape = (grid.ny, grid.nx)
        return zo.reshape(shape), co.reshape(shape), no.reshape(shape)
    return zo, co, no


def idw_bounds(grid: Grid, x, y, z, radius: float, max_pts: int = 0, bin_log2: int = -1,
               nodes=None, nthreads: int = 0):
    """Smallest and largest depth over O1's selected set (NaN where it is
    empty): returns (lo, hi) float64; nodes=None -> [ny, nx]."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    if nodes is None:
        m = grid.nx * grid.ny
        nd = None
    else:
        nd = np.ascontiguousarray(nodes, dtype=np.int64)
        m = nd.shape[0]
    lo = np.empty(max(m, 1), dtype=np.float64)
    hi = np.empty(max(m, 1), dtype=np.float64)
    _check(lib.orc_idw_bounds(ctypes.byref(grid.c()), _ptr(x), _ptr(y), _ptr(z), n, radius,
                              max_pts, bin_log2, _ptr(nd), m if nd is not None else 0,
                              _ptr(lo), _ptr(hi), nthreads), "orc_idw_bounds")
    lo, hi = lo[:m], hi[:m]
    if nodes is None:
        return lo.reshape(grid.ny, grid.nx), hi.reshape(grid.ny, grid.nx)
    return lo, hi


def nearest(grid: Grid, x, y, z, radius: float, bin_log2: int = -1, nodes=None,
            nthreads: int = 0):
    """O2: returns (idx int32, z float64); nodes=None -> [ny, nx]."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    if nodes is None:
        m = grid.nx * grid.ny
        nd = None
    else:
        nd = np.ascontiguousarray(nodes, dtype=np.int64)
        m = nd.shape[0]
    io = np.empty(max(m, 1), dtype=np.int32)
    zo = np.empty(max(m, 1), dtype=np.float64)
    _check(lib.orc_nearest(ctypes.byref(grid.c()), _ptr(x), _ptr(y), _ptr(z), n,
                           radius, bin_log2, _ptr(nd),
                           m if nd is not None else 0, _ptr(io), _ptr(zo),
                           nthreads), "orc_nearest")
    io, zo = io[:m], zo[:m]
    if nodes is None:
        return io.reshape(grid.ny, grid.nx), zo.reshape(grid.ny, grid.nx)
    return io, zo


def bilinear(src_grid: Grid, src, dst_grid: Grid, nthreads: int = 0):
    """O3: returns the destination grid [ny, nx] float64."""
    lib = _load()
    s = _f64(src).reshape(-1)
    if s.shape[0] != src_grid.nx * src_grid.ny:
        raise ValueError("source size does not match its grid")
    d = np.empty(dst_grid.nx * dst_grid.ny, dtype=np.float64)
    _check(lib.orc_bilinear(ctypes.byref(src_grid.c()), _ptr(s),
                            ctypes.byref(dst_grid.c()), _ptr(d), nthreads),
           "orc_bilinear")
    return d.reshape(dst_grid.ny, dst_grid.nx)


def bicubic(src_grid: Grid, src, dst_grid: Grid, nthreads: int = 0):
    """O5: Catmull-Rom resample with bilinear fallback; [ny, nx] float64."""
    lib = _load()
    s = _f64(src).reshape(-1)
    if s.shape[0] != src_grid.nx * src_grid.ny:
        raise ValueError("source size does not match its grid")
    d = np.empty(dst_grid.nx * dst_grid.ny, dtype=np.float64)
    _check(lib.orc_bicubic(ctypes.byref(src_grid.c()), _ptr(s),
                           ctypes.byref(dst_grid.c()), _ptr(d), nthreads),
           "orc_bicubic")
    return d.reshape(dst_grid.ny, dst_grid.nx)


def kriging(src_grid: Grid, src, dst_grid: Grid, range_m: float, nthreads: int = 0):
    """O6: ordinary kriging (5 x 5 neighbourhood, exponential variogram)."""
    lib = _load()
    s = _f64(src).reshape(-1)
    if s.shape[0] != src_grid.nx * src_grid.ny:
        raise ValueError("source size does not match its grid")
    d = np.empty(dst_grid.nx * dst_grid.ny, dtype=np.float64)
    _check(lib.orc_kriging(ctypes.byref(src_grid.c()), _ptr(s), ctypes.byref(dst_grid.c()),
                           float(range_m), _ptr(d), nthreads), "orc_kriging")
    return d.reshape(dst_grid.ny, dst_grid.nx)


def variogram(grid: Grid, src, nlags: int):
    """O7: empirical semivariogram along the axes; returns (gamma_x, gamma_y,
    pairs_x, pairs_y) for lags 1..nlags (lag k is k dx along x, k dy along y)."""
    lib = _load()
    s = _f64(src).reshape(-1)
    if s.shape[0] != grid.nx * grid.ny:
        raise ValueError("source size does not match its grid")
    gx = np.empty(nlags, dtype=np.float64)
    gy = np.empty(nlags, dtype=np.float64)
    px = np.empty(nlags, dtype=np.int64)
    py = np.empty(nlags, dtype=np.int64)
    _check(lib.orc_variogram(ctypes.byref(grid.c()), _ptr(s), int(nlags), _ptr(gx), _ptr(gy),
                             _ptr(px), _ptr(py)), "orc_variogram")
    return gx, gy, px, py


def fit_exponential(h, gamma, w):
    """O8: weighted least-squares exponential variogram fit; returns
    (range, sill, status) with status ORC_ERANGE (-2) when no sill was found
    inside the scanned interval."""
    lib = _load()
    h, g, w = _f64(h), _f64(gamma), _f64(w)
    a, c = ctypes.c_double(), ctypes.c_double()
    rc = lib.orc_fit_exponential(_ptr(h), _ptr(g), _ptr(w), int(h.shape[0]), ctypes.byref(a),
                                 ctypes.byref(c))
    if rc not in (0, -2):
        _check(rc, "orc_fit_exponential")
    return a.value, c.value, rc


def fit_grid_range(grid: Grid, src, nlags: int):
    """O7 then O8 on both axes, weighted by pair counts: (range, sill, status)."""
    gx, gy, px, py = variogram(grid, src, nlags)
    k = np.arange(1, nlags + 1, dtype=np.float64)
    h = np.concatenate([k * grid.dx, k * grid.dy])
    return fit_exponential(h, np.concatenate([gx, gy]),
                           np.concatenate([px, py]).astype(np.float64))
