"""auvgrid: gridding scattered multibeam soundings on one MI355X (gfx950).

Thin Python binding of ``libauvgrid.so`` (C ABI declared in
``include/auvgrid.h``).  Every function has the name of the C entry point it
marshals arguments for; all work runs in the library's HIP kernels.  PyTorch
only supplies device memory and streams.  There is no fallback: if the shared
library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libauvgrid.so")

AUV_OK = 0
AUV_ERR_INVALID = -1
AUV_ERR_RANGE = -2
AUV_ERR_BUDGET = -3
AUV_ERR_HIP = -4
AUV_ERR_STATE = -5

AUV_P_FP32_REBASE = 0
AUV_P_FP16_OFFSETS = 1
AUV_P_FP32_ABSOLUTE = 2

AUV_ALGO_AUTO = 0
AUV_ALGO_SPARSE = 1
AUV_ALGO_DENSE = 2
AUV_ALGO_SPAN = 3


class AuvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"auvgrid status {status}: {msg}")
        self.status = status


class auv_grid_desc(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class auv_idw_params(ctypes.Structure):
    _fields_ = [("power", ctypes.c_double), ("radius", ctypes.c_double),
                ("min_pts", ctypes.c_int32), ("max_pts", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("algo", ctypes.c_int32)]


class auv_batch_item(ctypes.Structure):
    _fields_ = [("grid", auv_grid_desc),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("n", ctypes.c_int64),
                ("params", auv_idw_params),
                ("z_out", ctypes.c_void_p), ("cnt_out", ctypes.c_void_p),
                ("nn_idx_out", ctypes.c_void_p), ("nn_z_out", ctypes.c_void_p)]


AUV_SERVE_FIFO = 0
AUV_SERVE_BATCHED = 1
AUV_T_QUEUED, AUV_T_RUNNING, AUV_T_DONE, AUV_T_FAILED = 0, 1, 2, 3


class auv_session_desc(ctypes.Structure):
    _fields_ = [("n_vehicles", ctypes.c_int32),
                ("grids", ctypes.POINTER(auv_grid_desc)),
                ("z_ref", ctypes.POINTER(ctypes.c_double)),
                ("params", auv_idw_params),
                ("max_request", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class auv_ticket_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("vehicle", ctypes.c_int32), ("n", ctypes.c_int64),
                ("t_arrival", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libauvgrid.so and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libauvgrid.so not found at {path}: build it with "
            "`python -m paper_2505_22675_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "auv_version": ([], ctypes.c_char_p),
        "auv_last_error": ([], ctypes.c_char_p),
        "auv_grid_create": ([P(auv_grid_desc), P(vp)], ctypes.c_int),
        "auv_grid_destroy": ([vp], None),
        "auv_bin_workspace_size": ([vp, i64, d, i32, P(ctypes.c_size_t)], ctypes.c_int),
        "auv_bin_points": ([vp, vp, vp, vp, i64, d, i32, vp, ctypes.c_size_t, vp, P(vp)],
                           ctypes.c_int),
        "auv_bins_info": ([vp, P(i32), P(i32), P(i32), P(i32)], ctypes.c_int),
        "auv_bins_export": ([vp, vp, vp, P(i64), vp], ctypes.c_int),
        "auv_bins_destroy": ([vp], None),
        "auv_interp_idw": ([vp, vp, P(auv_idw_params), vp, vp, vp, vp, vp], ctypes.c_int),
        "auv_interp_nearest": ([vp, vp, d, vp, vp, vp], ctypes.c_int),
        "auv_variogram_workspace_size": ([P(auv_grid_desc), i32, P(ctypes.c_size_t)],
                                         ctypes.c_int),
        "auv_variogram": ([vp, P(auv_grid_desc), i32, vp, ctypes.c_size_t, vp, vp, vp, vp, vp],
                          ctypes.c_int),
        "auv_fit_exponential": ([vp, vp, vp, i32, P(d), P(d)], ctypes.c_int),
        "auv_grid_idw_noalloc": ([vp, vp, vp, vp, i64, i32, P(auv_idw_params), vp, vp, vp, vp,
                                  vp], ctypes.c_int),
        "auv_resample_bilinear": ([vp, P(auv_grid_desc), vp, P(auv_grid_desc), vp],
                                  ctypes.c_int),
        "auv_resample_bicubic": ([vp, P(auv_grid_desc), vp, P(auv_grid_desc), vp],
                                 ctypes.c_int),
        "auv_resample_kriging": ([vp, P(auv_grid_desc), vp, P(auv_grid_desc), d, vp],
                                 ctypes.c_int),
        "auv_batch_plan": ([P(auv_batch_item), i32, ctypes.c_char_p, P(vp)], ctypes.c_int),
        "auv_batch_workspace_size": ([vp, P(ctypes.c_size_t)], ctypes.c_int),
        "auv_batch_launch": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "auv_batch_launch_plain": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "auv_batch_autotune": ([P(auv_batch_item), i32, vp, ctypes.c_size_t, vp,
                                ctypes.c_char_p], ctypes.c_int),
        "auv_batch_item_plan": ([vp, i32, P(i32), P(i32), P(i32), P(i32)], ctypes.c_int),
        "auv_batch_destroy": ([vp], None),
        "auv_session_budget": ([P(auv_session_desc), P(ctypes.c_size_t), P(ctypes.c_size_t)],
                               ctypes.c_int),
        "auv_session_create": ([P(auv_session_desc), vp, ctypes.c_size_t, P(vp)], ctypes.c_int),
        "auv_session_submit": ([vp, i32, vp, vp, vp, i64, d, P(ctypes.c_uint64)], ctypes.c_int),
        "auv_session_poll": ([vp, ctypes.c_uint64, P(auv_ticket_info)], ctypes.c_int),
        "auv_session_drain": ([vp], ctypes.c_int),
        "auv_session_read_grid": ([vp, i32, vp, vp, vp], ctypes.c_int),
        "auv_session_retire": ([vp, i32], ctypes.c_int),
        "auv_session_now": ([vp], d),
        "auv_session_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != AUV_OK:
        raise AuvError(rc, _lib.auv_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, name, numel=None):
    """Device pointer of a contiguous tensor of the given dtype (or None)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def auv_version() -> str:
    return load_library().auv_version().decode()


def auv_last_error() -> str:
    return load_library().auv_last_error().decode()


class Grid:
    """Owning wrapper of an ``auv_grid*``."""

    def __init__(self, desc: auv_grid_desc, handle: ctypes.c_void_p):
        self.desc = desc
        self._h = handle

    @property
    def nx(self):
        return self.desc.nx

    @property
    def ny(self):
        return self.desc.ny

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.auv_grid_destroy(self._h)
            self._h = None


def make_desc(x0, y0, dx, dy, nx, ny) -> auv_grid_desc:
    return auv_grid_desc(float(x0), float(y0), float(dx), float(dy), int(nx), int(ny))


def auv_grid_create(desc) -> Grid:
    """desc: auv_grid_desc or any object with x0, y0, dx, dy, nx, ny."""
    lib = load_library()
    if not isinstance(desc, auv_grid_desc):
        desc = make_desc(desc.x0, desc.y0, desc.dx, desc.dy, desc.nx, desc.ny)
    h = ctypes.c_void_p()
    _check(lib.auv_grid_create(ctypes.byref(desc), ctypes.byref(h)))
    return Grid(desc, h)


def auv_grid_destroy(grid: Grid):
    if grid._h:
        load_library().auv_grid_destroy(grid._h)
        grid._h = None


def auv_bin_workspace_size(grid: Grid, n: int, radius: float, bin_log2: int = 0) -> int:
    lib = load_library()
    out = ctypes.c_size_t()
    _check(lib.auv_bin_workspace_size(grid.handle, int(n), float(radius), int(bin_log2),
                                      ctypes.byref(out)))
    return out.value


@dataclass
class Bins:
    """Owning wrapper of an ``auv_bins*``; keeps its workspace and inputs alive."""
    handle: ctypes.c_void_p
    grid: Grid
    ws: torch.Tensor
    n: int
    radius: float
    keep: tuple = ()

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.auv_bins_destroy(self.handle)
            self.handle = None


def auv_bin_points(grid: Grid, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor,
                   radius: float, bin_log2: int = 0, ws: torch.Tensor | None = None,
                   stream=None) -> Bins:
    """Bin float64 device soundings; allocates the workspace when ws is None."""
    lib = load_library()
    n = int(x.numel())
    px = _dev(x, torch.float64, "x")
    py = _dev(y, torch.float64, "y", n)
    pz = _dev(z, torch.float64, "z", n)
    need = auv_bin_workspace_size(grid, n, radius, bin_log2)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    pw = _dev(ws, torch.uint8, "ws", need)
    h = ctypes.c_void_p()
    _check(lib.auv_bin_points(grid.handle, px, py, pz, n, float(radius), int(bin_log2),
                              pw, ws.numel(), _stream(stream), ctypes.byref(h)))
    return Bins(h, grid, ws, n, float(radius), keep=(x, y, z))


def auv_bins_info(bins: Bins):
    """Returns (nbx, nby, halo, bin_log2)."""
    lib = load_library()
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib.auv_bins_info(bins.handle, *[ctypes.byref(t) for t in v]))
    return tuple(t.value for t in v)


def auv_bins_export(bins: Bins, stream=None):
    """Returns (cell_start, perm, (n_binned, n_invalid, n_outside)) as device
    tensors; synchronises the stream."""
    lib = load_library()
    nbx, nby, _, _ = auv_bins_info(bins)
    dev = bins.ws.device
    cs = torch.empty(nbx * nby + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(max(bins.n, 1), dtype=torch.int32, device=dev)
    counts = (ctypes.c_int64 * 3)()
    _check(lib.auv_bins_export(bins.handle, _dev(cs, torch.int32, "cell_start"),
                               _dev(perm, torch.int32, "perm"), counts, _stream(stream)))
    nb = counts[0]
    return cs, perm[:nb], (counts[0], counts[1], counts[2])


def idw_params(power=2.0, radius=6.0, min_pts=1, max_pts=0, precision=AUV_P_FP32_REBASE,
               algo=AUV_ALGO_AUTO):
    return auv_idw_params(float(power), float(radius), int(min_pts), int(max_pts),
                          int(precision), int(algo))


def auv_interp_idw(grid: Grid, bins: Bins, params: auv_idw_params, z_out: torch.Tensor,
                   cnt_out=None, nn_idx_out=None, nn_z_out=None, stream=None):
    lib = load_library()
    m = grid.nx * grid.ny
    _check(lib.auv_interp_idw(grid.handle, bins.handle, ctypes.byref(params),
                              _dev(z_out, torch.float32, "z_out", m),
                              _dev(cnt_out, torch.int32, "cnt_out", m),
                              _dev(nn_idx_out, torch.int32, "nn_idx_out", m),
                              _dev(nn_z_out, torch.float32, "nn_z_out", m),
                              _stream(stream)))


def auv_grid_idw_noalloc(grid: Grid, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor,
                         bin_log2: int, params: auv_idw_params, z_out: torch.Tensor,
                         cnt_out=None, nn_idx_out=None, nn_z_out=None, stream=None):
    """Binning + IDW with the bins in the library's static device scratch
    (no device allocation; AUV_NOALLOC_SCRATCH_BYTES bytes per GPU)."""
    lib = load_library()
    n = int(x.numel())
    m = grid.nx * grid.ny
    _check(lib.auv_grid_idw_noalloc(grid.handle, _dev(x, torch.float64, "x", n),
                                    _dev(y, torch.float64, "y", n),
                                    _dev(z, torch.float64, "z", n), n, int(bin_log2),
                                    ctypes.byref(params),
                                    _dev(z_out, torch.float32, "z_out", m),
                                    _dev(cnt_out, torch.int32, "cnt_out", m),
                                    _dev(nn_idx_out, torch.int32, "nn_idx_out", m),
                                    _dev(nn_z_out, torch.float32, "nn_z_out", m),
                                    _stream(stream)))


AUV_NOALLOC_SCRATCH_BYTES = 160 << 20


def auv_variogram(src: torch.Tensor, s_desc, nlags: int, stream=None):
    """Empirical semivariogram along the axes: (gamma_x, gamma_y, pairs_x,
    pairs_y) as numpy arrays for lags 1..nlags (workspace allocated here)."""
    import numpy as np
    lib = load_library()
    if not isinstance(s_desc, auv_grid_desc):
        s_desc = make_desc(s_desc.x0, s_desc.y0, s_desc.dx, s_desc.dy, s_desc.nx, s_desc.ny)
    nb = ctypes.c_size_t()
    _check(lib.auv_variogram_workspace_size(ctypes.byref(s_desc), int(nlags), ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=src.device)
    gx = np.empty(nlags, dtype=np.float64)
    gy = np.empty(nlags, dtype=np.float64)
    px = np.empty(nlags, dtype=np.int64)
    py = np.empty(nlags, dtype=np.int64)
    _check(lib.auv_variogram(_dev(src, torch.float32, "src", s_desc.nx * s_desc.ny),
                             ctypes.byref(s_desc), int(nlags), ctypes.c_void_p(ws.data_ptr()),
                             nb.value, gx.ctypes.data, gy.ctypes.data, px.ctypes.data,
                             py.ctypes.data, _stream(stream)))
    return gx, gy, px, py


def auv_fit_exponential(h, gamma, w):
    """Exponential variogram fit: (range, sill, status); status AUV_ERR_RANGE
    when no sill lies inside the searched interval."""
    import numpy as np
    lib = load_library()
    h, g, w = (np.ascontiguousarray(v, dtype=np.float64) for v in (h, gamma, w))
    a, c = ctypes.c_double(), ctypes.c_double()
    rc = lib.auv_fit_exponential(h.ctypes.data, g.ctypes.data, w.ctypes.data, int(h.shape[0]),
                                 ctypes.byref(a), ctypes.byref(c))
    if rc not in (AUV_OK, AUV_ERR_RANGE):
        _check(rc)
    return a.value, c.value, rc


def fit_variogram_range(src: torch.Tensor, s_desc, nlags: int, stream=None):
    """auv_variogram on both axes, then auv_fit_exponential weighted by the
    pair counts: (range, sill, status)."""
    import numpy as np
    gx, gy, px, py = auv_variogram(src, s_desc, nlags, stream)
    k = np.arange(1, nlags + 1, dtype=np.float64)
    h = np.concatenate([k * s_desc.dx, k * s_desc.dy])
    return auv_fit_exponential(h, np.concatenate([gx, gy]),
                               np.concatenate([px, py]).astype(np.float64))


def auv_interp_nearest(grid: Grid, bins: Bins, radius: float, idx_out: torch.Tensor,
                       z_out=None, stream=None):
    lib = load_library()
    m = grid.nx * grid.ny
    _check(lib.auv_interp_nearest(grid.handle, bins.handle, float(radius),
                                  _dev(idx_out, torch.int32, "idx_out", m),
                                  _dev(z_out, torch.float32, "z_out", m),
                                  _stream(stream)))


def auv_resample_bilinear(src: torch.Tensor, s_desc, dst: torch.Tensor, d_desc, stream=None):
    lib = load_library()
    if not isinstance(s_desc, auv_grid_desc):
        s_desc = make_desc(s_desc.x0, s_desc.y0, s_desc.dx, s_desc.dy, s_desc.nx, s_desc.ny)
    if not isinstance(d_desc, auv_grid_desc):
        d_desc = make_desc(d_desc.x0, d_desc.y0, d_desc.dx, d_desc.dy, d_desc.nx, d_desc.ny)
    _check(lib.auv_resample_bilinear(
        _dev(src, torch.float32, "src", s_desc.nx * s_desc.ny), ctypes.byref(s_desc),
        _dev(dst, torch.float32, "dst", d_desc.nx * d_desc.ny), ctypes.byref(d_desc),
        _stream(stream)))


def auv_resample_bicubic(src: torch.Tensor, s_desc, dst: torch.Tensor, d_desc, stream=None):
    lib = load_library()
    if not isinstance(s_desc, auv_grid_desc):
        s_desc = make_desc(s_desc.x0, s_desc.y0, s_desc.dx, s_desc.dy, s_desc.nx, s_desc.ny)
    if not isinstance(d_desc, auv_grid_desc):
        d_desc = make_desc(d_desc.x0, d_desc.y0, d_desc.dx, d_desc.dy, d_desc.nx, d_desc.ny)
    _check(lib.auv_resample_bicubic(
        _dev(src, torch.float32, "src", s_desc.nx * s_desc.ny), ctypes.byref(s_desc),
        _dev(dst, torch.float32, "dst", d_desc.nx * d_desc.ny), ctypes.byref(d_desc),
        _stream(stream)))


def auv_resample_kriging(src: torch.Tensor, s_desc, dst: torch.Tensor, d_desc, range_m: float,
                         stream=None):
    lib = load_library()
    if not isinstance(s_desc, auv_grid_desc):
        s_desc = make_desc(s_desc.x0, s_desc.y0, s_desc.dx, s_desc.dy, s_desc.nx, s_desc.ny)
    if not isinstance(d_desc, auv_grid_desc):
        d_desc = make_desc(d_desc.x0, d_desc.y0, d_desc.dx, d_desc.dy, d_desc.nx, d_desc.ny)
    _check(lib.auv_resample_kriging(
        _dev(src, torch.float32, "src", s_desc.nx * s_desc.ny), ctypes.byref(s_desc),
        _dev(dst, torch.float32, "dst", d_desc.nx * d_desc.ny), ctypes.byref(d_desc),
        float(range_m), _stream(stream)))


# ------------------------------------------------------------ conveniences --

def grid_idw(grid: Grid, bins: Bins, power=2.0, radius=None, min_pts=1, max_pts=0,
             with_counts=False, with_nearest=False, precision=AUV_P_FP32_REBASE,
             algo=AUV_ALGO_AUTO, stream=None):
    """Allocate outputs and run auv_interp_idw; returns a dict of tensors."""
    dev = bins.ws.device
    shape = (grid.ny, grid.nx)
    out = {"z": torch.empty(shape, dtype=torch.float32, device=dev)}
    if with_counts:
        out["cnt"] = torch.empty(shape, dtype=torch.int32, device=dev)
    if with_nearest:
        out["nn_idx"] = torch.empty(shape, dtype=torch.int32, device=dev)
        out["nn_z"] = torch.empty(shape, dtype=torch.float32, device=dev)
    p = idw_params(power, bins.radius if radius is None else radius, min_pts, max_pts,
                   precision, algo)
    auv_interp_idw(grid, bins, p, out["z"], out.get("cnt"), out.get("nn_idx"),
                   out.get("nn_z"), stream)
    return out


# ------------------------------------------------------------------ batches


def batch_item(desc: auv_grid_desc, x, y, z, params: auv_idw_params, z_out, cnt_out=None,
               nn_idx_out=None, nn_z_out=None) -> auv_batch_item:
    """Fill an ``auv_batch_item`` from device tensors (which the caller keeps alive
    and in place for as long as the batch is launched)."""
    n = int(x.numel())
    cells = desc.nx * desc.ny
    it = auv_batch_item()
    it.grid = desc
    it.x = _dev(x, torch.float64, "x", n)
    it.y = _dev(y, torch.float64, "y", n)
    it.z = _dev(z, torch.float64, "z", n)
    it.n = n
    it.params = params
    it.z_out = _dev(z_out, torch.float32, "z_out", cells)
    it.cnt_out = _dev(cnt_out, torch.int32, "cnt_out", cells)
    it.nn_idx_out = _dev(nn_idx_out, torch.int32, "nn_idx_out", cells)
    it.nn_z_out = _dev(nn_z_out, torch.float32, "nn_z_out", cells)
    return it


def _items_array(items):
    arr = (auv_batch_item * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


class Batch:
    """Owning wrapper of an ``auv_batch*`` plus its device workspace."""

    def __init__(self, items, tune_path: str | None = None, device=None):
        lib = load_library()
        self.items = list(items)
        arr = _items_array(self.items)
        h = ctypes.c_void_p()
        path = tune_path.encode() if tune_path else None
        _check(lib.auv_batch_plan(arr, len(self.items), path, ctypes.byref(h)))
        self._h = h
        nbytes = ctypes.c_size_t()
        _check(lib.auv_batch_workspace_size(h, ctypes.byref(nbytes)))
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        # 256-byte aligned (the caching allocator hands out 512-byte aligned blocks)
        self.ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
        self.ws_bytes = int(nbytes.value)

    def launch(self, stream=None):
        """auv_batch_launch: capture on first use, replay afterwards."""
        _check(_lib.auv_batch_launch(self._h, ctypes.c_void_p(self.ws.data_ptr()),
                                     self.ws_bytes, _stream(stream)))

    def launch_plain(self, stream=None):
        """auv_batch_launch_plain: item after item, default sizes, no graph."""
        _check(_lib.auv_batch_launch_plain(self._h, ctypes.c_void_p(self.ws.data_ptr()),
                                           self.ws_bytes, _stream(stream)))

    def item_plan(self, i: int):
        """(bin_log2, algo) the batched form uses for item i."""
        return self.item_plan_full(i)[:2]

    def item_plan_full(self, i: int):
        """(bin_log2, algo, tile_w, tile_h) the batched form uses for item i."""
        s, a, tw, th = (ctypes.c_int32() for _ in range(4))
        _check(_lib.auv_batch_item_plan(self._h, i, ctypes.byref(s), ctypes.byref(a),
                                        ctypes.byref(tw), ctypes.byref(th)))
        return s.value, a.value, tw.value, th.value

    def close(self):
        if self._h:
            _lib.auv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def auv_batch_autotune(items, ws: torch.Tensor, tune_path: str, stream=None):
    """Time (bin size, kernel form) candidates per item class; write tune_path."""
    lib = load_library()
    arr = _items_array(items)
    _check(lib.auv_batch_autotune(arr, len(items), _dev(ws, torch.uint8, "ws"), ws.numel(),
                                  _stream(stream), tune_path.encode()))


# ------------------------------------------------------------------ serving


def session_desc(grids, power=2.0, radius=6.0, min_pts=1, max_request=50000, slots=32,
                 mode=AUV_SERVE_BATCHED, max_batch=0, z_ref=None) -> auv_session_desc:
    """Build an ``auv_session_desc``; grids: objects with x0, y0, dx, dy, nx, ny.
    The returned struct keeps its arrays alive (``_keep``)."""
    g = (auv_grid_desc * len(grids))()
    for i, gr in enumerate(grids):
        g[i] = gr if isinstance(gr, auv_grid_desc) else make_desc(gr.x0, gr.y0, gr.dx, gr.dy,
                                                                   gr.nx, gr.ny)
    d = auv_session_desc()
    d.n_vehicles = len(grids)
    d.grids = g
    zr = None
    if z_ref is not None:
        zr = (ctypes.c_double * len(grids))(*[float(v) for v in z_ref])
        d.z_ref = zr
    d.params = idw_params(power, radius, min_pts, 0)
    d.max_request = int(max_request)
    d.slots = int(slots)
    d.mode = int(mode)
    d.max_batch = int(max_batch)
    d._keep = (g, zr)
    return d


def auv_session_budget(desc: auv_session_desc):
    """(fixed bytes, bytes per admitted vehicle)."""
    lib = load_library()
    f, v = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.auv_session_budget(ctypes.byref(desc), ctypes.byref(f), ctypes.byref(v)))
    return int(f.value), int(v.value)


def _host_f64(a, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 1:
        raise ValueError(f"{name} must be one-dimensional")
    return a


class Session:
    """Owning wrapper of an ``auv_session*``; the arena is a uint8 device tensor."""

    def __init__(self, desc: auv_session_desc, arena: torch.Tensor):
        lib = load_library()
        self.desc = desc
        self.arena = arena
        if not arena.is_cuda or arena.dtype != torch.uint8:
            raise ValueError("arena must be a uint8 device tensor")
        h = ctypes.c_void_p()
        _check(lib.auv_session_create(ctypes.byref(desc), ctypes.c_void_p(arena.data_ptr()),
                                      arena.numel(), ctypes.byref(h)))
        self._h = h
        self.grids = [desc.grids[i] for i in range(desc.n_vehicles)]

    def now(self) -> float:
        return float(_lib.auv_session_now(self._h))

    def submit(self, vehicle: int, x, y, z, t_arrival=None) -> int:
        x, y, z = _host_f64(x, "x"), _host_f64(y, "y"), _host_f64(z, "z")
        n = x.shape[0]
        if y.shape[0] != n or z.shape[0] != n:
            raise ValueError("x, y, z lengths differ")
        t = ctypes.c_uint64()
        ta = self.now() if t_arrival is None else float(t_arrival)
        _check(_lib.auv_session_submit(self._h, int(vehicle), x.ctypes.data, y.ctypes.data,
                                       z.ctypes.data, n, ta, ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int) -> auv_ticket_info:
        info = auv_ticket_info()
        _check(_lib.auv_session_poll(self._h, ticket, ctypes.byref(info)))
        return info

    def drain(self):
        _check(_lib.auv_session_drain(self._h))

    def read_grid(self, vehicle: int, with_counts=True, stream=None):
        g = self.grids[vehicle]
        dev = self.arena.device
        z = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)
        c = torch.empty((g.ny, g.nx), dtype=torch.int32, device=dev) if with_counts else None
        _check(_lib.auv_session_read_grid(self._h, int(vehicle), ctypes.c_void_p(z.data_ptr()),
                                          ctypes.c_void_p(c.data_ptr()) if c is not None else None,
                                          _stream(stream)))
        return z, c

    def retire(self, vehicle: int):
        _check(_lib.auv_session_retire(self._h, int(vehicle)))

    def close(self):
        if self._h:
            _lib.auv_session_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
