"""Python binding of libkde, the MI355X KDE heat-map library (arXiv 2004.13653).

Thin ctypes marshalling over the C ABI in include/kde.h: every step of the map is
computed by the HIP kernels in libkde.so; PyTorch only supplies device memory and
the current stream.  There is no CPU fallback: if libkde.so is missing, every call
raises.

Build the library with ``python -m paper_2004_13653_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple

import numpy as np

__all__ = ["KERNELS", "PRECISIONS", "KDEError", "Grid", "lib", "eval", "backward", "lscv", "kde_map", "kde_lscv",
           "eval_batched", "to_grid_units", "bandwidth_units", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkde.so")

KERNELS = {"uniform": 0, "triangular": 1, "epanechnikov": 2, "quartic": 3, "triweight": 4, "tricube": 5,
           "gaussian": 6, "cosine": 7}
PRECISIONS = {"fp32": 0, "fp16": 1, "bf16": 2, "fp16x3": 3, "bf16x3": 4}
RAW_SUM = 1

KDE_OK, KDE_EINVAL, KDE_ENOMEM, KDE_EHIP, KDE_EUNSUPPORTED = 0, -1, -2, -3, -4
_STATUS = {KDE_EINVAL: "EINVAL", KDE_ENOMEM: "ENOMEM", KDE_EHIP: "EHIP", KDE_EUNSUPPORTED: "EUNSUPPORTED"}


class KDEError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class MapDesc(ctypes.Structure):
    """ctypes image of struct kde_map (one descriptor of kde_eval_batched)."""

    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("kernel_id", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("grid", ctypes.c_void_p), ("out", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libkde.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libkde.so not found at {LIB_PATH}; build it with "
                               "'python -m paper_2004_13653_amd.build'")
        # PyTorch ships its own HIP runtime with the same soname as the system one.
        # Loading torch first makes libkde bind to that copy, so the process holds
        # a single HIP runtime (two runtimes in one process cannot share a device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u32, d, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
        sig = {
            "kde_create_grid": (ctypes.c_int, [d, d, d, d, i32, i32, ctypes.POINTER(p)]),
            "kde_destroy_grid": (None, [p]),
            "kde_grid_shape": (ctypes.c_int, [p, p, p, p, p]),
            "kde_to_grid_units": (ctypes.c_int, [p, p, i64, p]),
            "kde_bandwidth_units": (ctypes.c_int, [p, d, d, p, p]),
            "kde_eval": (ctypes.c_int, [p, i64, i32, d, d, p, p, i32, u32, p]),
            "kde_eval_noalloc": (ctypes.c_int, [p, i64, i32, d, d, p, p, i32, u32, p]),
            "kde_eval_batched": (ctypes.c_int, [p, i32, u32, p]),
            "kde_backward": (ctypes.c_int, [p, i64, i32, d, d, p, p, p, p, u32, p]),
            "kde_lscv": (ctypes.c_int, [p, i64, i32, d, d, p, p, p, p]),
            "kde_bin_counts": (ctypes.c_int, [p, i64, p, p, p, p, p]),
            "kde_conv_counts": (ctypes.c_int, [p, p, p, i32, d, d, i32, i32, p, u32, p]),
            "kde_eval_binned": (ctypes.c_int, [p, i64, p, i32, d, d, i32, i32, p, p, u32, p]),
            "kde_dp_compress": (ctypes.c_int, [p, i64, p, i64, d, p, p, p, p, p, p]),
            "kde_compression_metrics": (ctypes.c_int, [p, i64, p, p, i64, p, i64, p, p, p,
                                                       ctypes.POINTER(TrackMetrics), p]),
            "kde_time_next_main_kernel": (ctypes.c_int, [p, p]),
            "kde_autotune_enable": (ctypes.c_int, [i32]),
            "kde_autotune_force": (ctypes.c_int, [i32]),
            "kde_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
            "kde_autotune_save": (ctypes.c_int, [ctypes.c_char_p]),
            "kde_autotune_dump": (ctypes.c_int, [p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
            "kde_autotune_clear": (ctypes.c_int, []),
            "kde_last_error": (ctypes.c_char_p, []),
            "kde_shutdown": (None, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != KDE_OK:
        raise KDEError(status, lib().kde_last_error().decode())


def _kernel_id(kernel) -> int:
    if isinstance(kernel, str):
        return KERNELS[kernel.lower()]
    return int(kernel)


class Grid:
    """Library-owned node grid (kde_create_grid): nx x ny nodes spanning
    [xmin, xmax] x [ymin, ymax], both edges on nodes."""

    def __init__(self, xmin: float, xmax: float, ymin: float, ymax: float, nx: int, ny: int):
        h = ctypes.c_void_p()
        _check(lib().kde_create_grid(xmin, xmax, ymin, ymax, nx, ny, ctypes.byref(h)))
        self._h = h
        self.bounds = (float(xmin), float(xmax), float(ymin), float(ymax))
        nx_, ny_ = ctypes.c_int32(), ctypes.c_int32()
        dx, dy = ctypes.c_double(), ctypes.c_double()
        _check(lib().kde_grid_shape(h, ctypes.byref(nx_), ctypes.byref(ny_), ctypes.byref(dx), ctypes.byref(dy)))
        self.nx, self.ny, self.dx, self.dy = nx_.value, ny_.value, dx.value, dy.value

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.kde_destroy_grid(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_grid_units(xy, grid: Grid) -> np.ndarray:
    """World points [n, 2] (FP64) to FP32 grid units on the host (kde_to_grid_units)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    out = np.empty(xy.shape, dtype=np.float32)
    _check(lib().kde_to_grid_units(grid.handle, xy.ctypes.data, xy.shape[0], out.ctypes.data))
    return out


def bandwidth_units(hx: float, hy: float, grid: Grid) -> tuple[np.float32, np.float32]:
    Hx, Hy = ctypes.c_float(), ctypes.c_float()
    _check(lib().kde_bandwidth_units(grid.handle, hx, hy, ctypes.byref(Hx), ctypes.byref(Hy)))
    return np.float32(Hx.value), np.float32(Hy.value)


def _stream(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_points(points, torch):
    if not (points.is_cuda and points.dtype == torch.float32 and points.dim() == 2 and points.shape[1] == 2):
        raise ValueError("points must be a CUDA float32 tensor of shape [n, 2]")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous")


TRUNCATE = 8


def eval(points, kernel, hx: float, hy: float, grid: Grid, out=None, precision: str = "fp32",
         raw: bool = False, truncate: bool = False):
    """The heat map of `points` ([n, 2] FP32 grid units on the GPU) on `grid`:
    returns (or fills) an [ny, nx] FP32 tensor (kde_eval).  truncate: the
    Gaussian cut at 8 bandwidths (binned on the FP32 path, banded on the
    matrix-core paths)."""
    return _eval("kde_eval", points, kernel, hx, hy, grid, out, precision, raw, truncate)


# Device scratch of the allocation-free entry point (KDE_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 128 << 20


def eval_noalloc(points, kernel, hx: float, hy: float, grid: Grid, out, precision: str = "fp32",
                 raw: bool = False, truncate: bool = False):
    """eval through kde_eval_noalloc: fills the caller's `out` using the
    library's fixed per-GPU scratch array instead of allocated workspace (no
    device allocation in the call; maps needing more scratch are rejected)."""
    return _eval("kde_eval_noalloc", points, kernel, hx, hy, grid, out, precision, raw, truncate)


def _eval(entry, points, kernel, hx, hy, grid, out, precision, raw, truncate):
    import torch
    _check_points(points, torch)
    if out is None:
        out = torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=points.device)
    elif not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.numel() == grid.nx * grid.ny):
        raise ValueError("out must be a contiguous CUDA float32 tensor with ny*nx elements")
    with torch.cuda.device(points.device):
        _check(getattr(lib(), entry)(points.data_ptr() if points.numel() else None, points.shape[0],
                                     _kernel_id(kernel), hx, hy, grid.handle, out.data_ptr(), PRECISIONS[precision],
                                     (RAW_SUM if raw else 0) | (TRUNCATE if truncate else 0),
                                     _stream(torch, points.device)))
    return out


def _check_labels(labels, n, torch):
    if labels is None:
        return None
    if not (labels.is_cuda and labels.dtype == torch.int32 and labels.dim() == 1 and labels.shape[0] == n
            and labels.is_contiguous()):
        raise ValueError("labels must be a contiguous CUDA int32 tensor of shape [n]")
    return labels.data_ptr()


def bin_counts(points, labels, grid: Grid, counts=None, total=None):
    """The paper's count matrix (kde_bin_counts): ceil projection of the points
    and, with trajectory labels ([n] int32 CUDA tensor), the gap cells between
    consecutive points.  Returns (counts [ny, nx] int32 tensor holding the
    uint32 counts, total [1] int64 tensor holding the number of counted cells)."""
    import torch
    _check_points(points, torch)
    dev = points.device
    if counts is None:
        counts = torch.empty((grid.ny, grid.nx), dtype=torch.int32, device=dev)
    if total is None:
        total = torch.empty(1, dtype=torch.int64, device=dev)
    lab = _check_labels(labels, points.shape[0], torch)
    with torch.cuda.device(dev):
        _check(lib().kde_bin_counts(points.data_ptr() if points.numel() else None, points.shape[0], lab, grid.handle,
                                    counts.data_ptr(), total.data_ptr(), _stream(torch, dev)))
    return counts, total


def conv_counts(counts, total, kernel, hx: float, hy: float, a: int, b: int, grid: Grid, out=None,
                raw: bool = False):
    """Eq. (7) convolution of a count matrix (kde_conv_counts); density scaled
    by the number of counted cells in `total` unless raw."""
    import torch
    if out is None:
        out = torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=counts.device)
    with torch.cuda.device(counts.device):
        _check(lib().kde_conv_counts(counts.data_ptr(), total.data_ptr() if total is not None else None,
                                     grid.handle, _kernel_id(kernel), hx, hy, int(a), int(b), out.data_ptr(),
                                     RAW_SUM if raw else 0, _stream(torch, counts.device)))
    return out


def eval_binned(points, labels, kernel, hx: float, hy: float, a: int, b: int, grid: Grid, out=None,
                raw: bool = False):
    """The paper's binned heat map in one call (kde_eval_binned)."""
    import torch
    _check_points(points, torch)
    if out is None:
        out = torch.empty((grid.ny, grid.nx), dtype=torch.float32, device=points.device)
    lab = _check_labels(labels, points.shape[0], torch)
    with torch.cuda.device(points.device):
        _check(lib().kde_eval_binned(points.data_ptr() if points.numel() else None, points.shape[0], lab,
                                     _kernel_id(kernel), hx, hy, int(a), int(b), grid.handle, out.data_ptr(),
                                     RAW_SUM if raw else 0, _stream(torch, points.device)))
    return out


def paper_taps(kernel, varpi: int, grid: Grid) -> tuple[float, float, int, int]:
    """The paper's table of odd size varpi (Eq. (7)-(8)) in this library's terms:
    (hx, hy, a, b) with a = b = (varpi - 1) / 2 cells; compact kernels reach
    exactly a cells (H = a), the Gaussian has sigma = one cell (H = 1)."""
    if varpi < 1 or varpi % 2 == 0:
        raise ValueError("varpi must be a positive odd integer")
    r = (varpi - 1) // 2
    H = 1.0 if _kernel_id(kernel) == KERNELS["gaussian"] else float(max(r, 1))
    return H * grid.dx, H * grid.dy, r, r


class DpResult(NamedTuple):
    keep: object     # [n] uint8, 1 for kept points
    xy: object       # [n_kept, 2] kept points in order, or None
    lengths: object  # [n_tracks] kept points per track, or None
    start: object    # [n_tracks + 1] offsets of the compressed tracks, or None


def dp_compress(xy, track_start, eps: float, compact: bool = True) -> DpResult:
    """Douglas-Peucker compression of merged tracks on the GPU (kde_dp_compress).
    xy: [n, 2] float64 CUDA tensor (planar, e.g. Mercator metres); track_start:
    [n_tracks + 1] int64 CUDA tensor of offsets.  With compact=False only the
    keep mask is produced."""
    import torch
    if not (xy.is_cuda and xy.dtype == torch.float64 and xy.dim() == 2 and xy.shape[1] == 2 and xy.is_contiguous()):
        raise ValueError("xy must be a contiguous CUDA float64 tensor of shape [n, 2]")
    if not (track_start.is_cuda and track_start.dtype == torch.int64 and track_start.dim() == 1
            and track_start.is_contiguous()):
        raise ValueError("track_start must be a contiguous CUDA int64 tensor")
    n, nt = xy.shape[0], track_start.shape[0] - 1
    keep = torch.empty(n, dtype=torch.uint8, device=xy.device)
    out = torch.empty_like(xy) if compact else None
    lens = torch.empty(max(nt, 0), dtype=torch.int64, device=xy.device) if compact else None
    starts = torch.empty(max(nt, 0) + 1, dtype=torch.int64, device=xy.device) if compact else None
    kept = ctypes.c_int64()
    with torch.cuda.device(xy.device):
        _check(lib().kde_dp_compress(xy.data_ptr() if n else None, n, track_start.data_ptr(), nt, float(eps),
                                     keep.data_ptr() if n else None, out.data_ptr() if compact and n else None,
                                     lens.data_ptr() if compact and nt > 0 else None,
                                     starts.data_ptr() if compact else None, ctypes.byref(kept),
                                     _stream(torch, xy.device)))
    if compact:
        out = out[:kept.value]
    return DpResult(keep, out, lens, starts)


class TrackMetrics(ctypes.Structure):
    """kde_track_metrics: totals of the compression-quality measures."""
    _fields_ = [("n_original", ctypes.c_int64), ("n_compressed", ctypes.c_int64), ("cr_percent", ctypes.c_double),
                ("length_original", ctypes.c_double), ("length_compressed", ctypes.c_double),
                ("rll", ctypes.c_double), ("dtw_mean", ctypes.c_double), ("dtw_std", ctypes.c_double)]


def _track_set(xy, start, what):
    import torch
    if not (xy.is_cuda and xy.dtype == torch.float64 and xy.dim() == 2 and xy.shape[1] == 2 and xy.is_contiguous()):
        raise ValueError(f"{what} points must be a contiguous CUDA float64 tensor of shape [n, 2]")
    if not (start.is_cuda and start.dtype == torch.int64 and start.dim() == 1 and start.shape[0] >= 1
            and start.is_contiguous()):
        raise ValueError(f"{what} offsets must be a contiguous CUDA int64 tensor of length n_tracks + 1")


def compression_metrics(xy_o, start_o, xy_c, start_c, per_track: bool = True) -> dict:
    """Compression quality of tracks against their compressed versions on the
    GPU (kde_compression_metrics, Sec. V-B): CR, RLL, and the mean and
    population standard deviation of the per-track DTW distances.  xy_*: [n, 2]
    float64 CUDA tensors; start_*: [n_tracks + 1] int64 CUDA offsets (e.g. the
    xy and start of dp_compress).  With per_track the dict also holds the
    per-track tensors len_o, len_c and dtw."""
    import torch
    _track_set(xy_o, start_o, "original")
    _track_set(xy_c, start_c, "compressed")
    nt = start_o.shape[0] - 1
    if start_c.shape[0] - 1 != nt:
        raise ValueError("both track sets must hold the same number of tracks")
    dev = xy_o.device
    lo = lc = dt = None
    if per_track:
        lo, lc, dt = (torch.empty(nt, dtype=torch.float64, device=dev) for _ in range(3))
    tot = TrackMetrics()
    with torch.cuda.device(dev):
        _check(lib().kde_compression_metrics(xy_o.data_ptr() if xy_o.shape[0] else None, xy_o.shape[0],
                                             start_o.data_ptr(), xy_c.data_ptr() if xy_c.shape[0] else None,
                                             xy_c.shape[0], start_c.data_ptr(), nt,
                                             lo.data_ptr() if per_track and nt else None,
                                             lc.data_ptr() if per_track and nt else None,
                                             dt.data_ptr() if per_track and nt else None, ctypes.byref(tot),
                                             _stream(torch, dev)))
    out = {name: getattr(tot, name) for name, _ in TrackMetrics._fields_}
    if per_track:
        out.update(len_o=lo, len_c=lc, dtw=dt)
    return out


def autotune(enabled: bool | None = None, force: int | None = None, load: str | None = None,
             save: str | None = None, clear: bool = False) -> dict:
    """Tile-shape autotuner of the FP32 direct path (kde_autotune_*): switch
    tuning on or off, force a register block (2, 4, 8; 0 ends forcing), merge or
    write a JSON cache file, empty the cache.  Returns the cache's entries
    {key: {"choice": ..., "ms": {...}}}."""
    L = lib()
    if clear:
        _check(L.kde_autotune_clear())
    if enabled is not None:
        _check(L.kde_autotune_enable(1 if enabled else 0))
    if force is not None:
        _check(L.kde_autotune_force(int(force)))
    if load is not None:
        _check(L.kde_autotune_load(os.fsencode(load)))
    if save is not None:
        _check(L.kde_autotune_save(os.fsencode(save)))
    need = ctypes.c_size_t()
    _check(L.kde_autotune_dump(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(L.kde_autotune_dump(buf, need.value, ctypes.byref(need)))
    import json
    return json.loads(buf.value.decode())["entries"]


def time_next_main_kernel(start, stop) -> None:
    """Arms kde_time_next_main_kernel with two torch.cuda.Event objects (created
    with enable_timing=True): the next `eval` on this thread records them around
    its main kernel, so start.elapsed_time(stop) is that kernel's duration."""
    import torch
    if start is None and stop is None:
        _check(lib().kde_time_next_main_kernel(None, None))
        return
    for e in (start, stop):
        if e.cuda_event == 0:  # torch creates the HIP event on its first record
            e.record(torch.cuda.current_stream())
    _check(lib().kde_time_next_main_kernel(start.cuda_event, stop.cuda_event))


GRID_UNIT_GRADS = 2
VJP_FP32 = 16


def backward(points, kernel, hx: float, hy: float, grid: Grid, grad_out, raw: bool = False,
             grid_units: bool = False, want_points: bool = True, want_h: bool = True, fp32: bool = False):
    """Vector-Jacobian product of `eval` (kde_backward).  Returns (grad_points
    [n, 2] FP32 tensor or None, (dL/dhx, dL/dhy) floats or None).  fp32: the
    Gaussian's sums pair by pair in FP32 instead of on matrix cores."""
    import torch
    _check_points(points, torch)
    if not (grad_out.is_cuda and grad_out.dtype == torch.float32 and grad_out.is_contiguous()
            and grad_out.numel() == grid.nx * grid.ny):
        raise ValueError("grad_out must be a contiguous CUDA float32 tensor with ny*nx elements")
    gp = torch.empty_like(points) if want_points else None
    gh = (ctypes.c_double * 2)() if want_h else None
    flags = (RAW_SUM if raw else 0) | (GRID_UNIT_GRADS if grid_units else 0) | (VJP_FP32 if fp32 else 0)
    with torch.cuda.device(points.device):
        _check(lib().kde_backward(points.data_ptr() if points.numel() else None, points.shape[0],
                                  _kernel_id(kernel), hx, hy, grid.handle, grad_out.data_ptr(),
                                  gp.data_ptr() if gp is not None and points.numel() else None, gh, flags,
                                  _stream(torch, points.device)))
    return gp, ((gh[0], gh[1]) if gh is not None else None)


def lscv(points, kernel, hx: float, hy: float, grid: Grid):
    """Least-squares cross-validation score and its gradient w.r.t. (hx, hy)
    (kde_lscv).  Returns (value, (dLSCV/dhx, dLSCV/dhy))."""
    import torch
    _check_points(points, torch)
    v = ctypes.c_double()
    gh = (ctypes.c_double * 2)()
    with torch.cuda.device(points.device):
        _check(lib().kde_lscv(points.data_ptr(), points.shape[0], _kernel_id(kernel), hx, hy, grid.handle,
                              ctypes.byref(v), gh, _stream(torch, points.device)))
    return v.value, (gh[0], gh[1])


def _autograd():
    import torch

    class KDEMap(torch.autograd.Function):
        """out = eval(points, kernel, hx, hy, grid); gradients w.r.t. the grid-unit
        points and the world-unit bandwidths come from kde_backward."""

        @staticmethod
        def forward(ctx, points, hx, hy, kernel, grid, raw):
            ctx.save_for_backward(points)
            ctx.args = (kernel, float(hx), float(hy), grid, raw)
            return eval(points, kernel, float(hx), float(hy), grid, raw=raw)

        @staticmethod
        def backward(ctx, grad_out):
            (points,) = ctx.saved_tensors
            kernel, hx, hy, grid, raw = ctx.args
            want_h = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
            gp, gh = backward(points, kernel, hx, hy, grid, grad_out.contiguous(), raw=raw, grid_units=True,
                              want_points=ctx.needs_input_grad[0], want_h=want_h)
            ghx = torch.tensor(gh[0], dtype=torch.float64) if want_h else None
            ghy = torch.tensor(gh[1], dtype=torch.float64) if want_h else None
            return gp, ghx, ghy, None, None, None

    class KDELSCV(torch.autograd.Function):
        """LSCV(hx, hy) of fixed points; gradient w.r.t. the bandwidths."""

        @staticmethod
        def forward(ctx, points, hx, hy, kernel, grid):
            value, grad = lscv(points, kernel, float(hx), float(hy), grid)
            ctx.grad = grad
            return torch.tensor(value, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            gx, gy = ctx.grad
            return None, g * gx, g * gy, None, None

    return KDEMap, KDELSCV


def kde_map(points, hx, hy, kernel, grid: Grid, raw: bool = False):
    """Differentiable heat map: points [n, 2] grid units (CUDA FP32), hx, hy world
    units (Python floats or 0-d tensors)."""
    KDEMap, _ = _autograd()
    return KDEMap.apply(points, hx, hy, kernel, grid, raw)


def kde_lscv(points, hx, hy, kernel, grid: Grid):
    """Differentiable LSCV score as a 0-d FP64 tensor (gradients w.r.t. hx, hy)."""
    _, KDELSCV = _autograd()
    return KDELSCV.apply(points, hx, hy, kernel, grid)


BATCH_EAGER = 4


def eval_batched(maps, raw: bool = False, eager: bool = False, stream_device=None):
    """Many maps in one call (kde_eval_batched).  `maps` is a list of (points
    [n, 2] CUDA FP32 grid units, kernel, hx, hy, Grid, out [ny, nx] CUDA FP32)
    tuples, optionally followed by a precision name (default "fp32": the
    persistent launch) and a truncate flag; outputs are written in place."""
    import torch
    descs = (MapDesc * len(maps))()
    dev = None
    for d, m in zip(descs, maps):
        pts, kernel, hx, hy, grid, out = m[:6]
        precision = m[6] if len(m) > 6 else "fp32"
        truncate = bool(m[7]) if len(m) > 7 else False
        _check_points(pts, torch)
        if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                and out.numel() == grid.nx * grid.ny):
            raise ValueError("out must be a contiguous CUDA float32 tensor with ny*nx elements")
        dev = pts.device if dev is None else dev
        d.points = pts.data_ptr() if pts.numel() else None
        d.n = pts.shape[0]
        d.kernel_id = _kernel_id(kernel)
        d.precision = PRECISIONS[precision]
        d.hx, d.hy = float(hx), float(hy)
        d.grid = grid.handle.value
        d.out = out.data_ptr()
        d.flags = TRUNCATE if truncate else 0
        d.reserved = 0
    if dev is None:
        return
    flags = (RAW_SUM if raw else 0) | (BATCH_EAGER if eager else 0)
    with torch.cuda.device(dev):
        _check(lib().kde_eval_batched(descs, len(maps), flags, _stream(torch, dev)))
