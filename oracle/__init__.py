"""FP64 CPU oracle for the KDE heat map (arXiv 2004.13653, Sec. III-C, Eq. (7)-(8),
Table I), plus the map's vector-Jacobian product and the LSCV bandwidth objective.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the bench's CPU-baseline leg
may import this package; the product library never does.  It shares no code with
the HIP path.

The arithmetic lives in kde_oracle.c (plain loops, FP64, per-output sums in index
order).  This module loads it (building it with gcc if the shared object is
missing) and adds two things:

* to_units / bandwidth_units: the FP64 -> FP32 pixel-coordinate conditioning,
  written out independently of the library's own;
* map_units_separable / vjp_units_separable: the same sums as the C loops in the
  factored form D = Gy @ Gx^T (Table I kernels are products k(s) k(t)), with a
  library matmul as the contraction step, for windows too large for the plain
  loops.  They are pinned against the plain loops in the tests.

Parity unpinned: none (every function is pinned by a test in tests/test_oracle_*).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

KERNELS = ("uniform", "triangular", "epanechnikov", "quartic", "triweight", "tricube", "gaussian", "cosine")
GAUSSIAN = 6
GAUSS_TRUNC = 8  # the Gaussian truncated at |u| <= 8 (not in Table I)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kde_oracle.c")
_SO = os.path.join(_HERE, "libkde_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile kde_oracle.c with gcc (no fast-math) into libkde_oracle.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        d, i, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        f = ctypes.c_float
        L.ko_num_threads.restype = ctypes.c_int
        L.ko_num_threads.argtypes = []
        L.ko_set_num_threads.restype = None
        L.ko_set_num_threads.argtypes = [ctypes.c_int]
        L.ko_k.restype = d
        L.ko_k.argtypes = [i, d]
        L.ko_dk.restype = d
        L.ko_dk.argtypes = [i, d]
        for name in ("ko_k_array", "ko_dk_array", "ko_kbar_array", "ko_dkbar_array"):
            getattr(L, name).argtypes = [i, p, i64, p]
            getattr(L, name).restype = None
        L.ko_map_world.argtypes = [p, i64, i, d, d, d, d, d, d, i, i, i, i, i, i, i, p]
        L.ko_map_units.argtypes = [p, i64, i, f, f, i, i, i, i, p]
        L.ko_map_units_at.argtypes = [p, i64, i, f, f, p, i64, p]
        L.ko_vjp_units.argtypes = [p, i64, i, f, f, i, i, p, p, i64, p, p]
        L.ko_lscv_world.argtypes = [p, i64, i, d, d, p, p]
        L.ko_lscv_units.argtypes = [p, i64, i, f, f, p, p]
        L.ko_bin_counts.argtypes = [p, i64, p, i, i, p, p]
        L.ko_conv_counts.argtypes = [p, i, i, i, f, f, i, i, i, i, i, i, p]
        L.ko_dp_keep.argtypes = [p, i64, p, i64, d, p]
        L.ko_dp_keep.restype = i64
        L.ko_track_length.argtypes = [p, i64]
        L.ko_track_length.restype = d
        L.ko_dtw.argtypes = [p, i64, p, i64]
        L.ko_dtw.restype = d
        L.ko_track_metrics.argtypes = [p, p, p, p, i64, p, p, p]
        L.ko_track_metrics.restype = None
        for name in ("ko_map_world", "ko_map_units", "ko_map_units_at", "ko_vjp_units", "ko_lscv_world",
                     "ko_lscv_units", "ko_bin_counts", "ko_conv_counts"):
            getattr(L, name).restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP)."""
    return int(lib().ko_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's parallel loops (results do not depend on it)."""
    lib().ko_set_num_threads(int(n))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _apply(name: str, kernel: int, u) -> np.ndarray:
    u = _f64(u)
    out = np.empty_like(u)
    getattr(lib(), name)(int(kernel), _ptr(u), u.size, _ptr(out))
    return out


def k(kernel: int, u) -> np.ndarray:
    """1-D factor k(u) of Table I (support |u| <= 1; Gaussian unbounded)."""
    return _apply("ko_k_array", kernel, u)


def dk(kernel: int, u) -> np.ndarray:
    return _apply("ko_dk_array", kernel, u)


def kbar(kernel: int, u) -> np.ndarray:
    """Autoconvolution (k * k)(u) of a Table I factor."""
    return _apply("ko_kbar_array", kernel, u)


def dkbar(kernel: int, u) -> np.ndarray:
    return _apply("ko_dkbar_array", kernel, u)


# --------------------------------------------------------------------------- grid
class Grid:
    """Node grid of Eq. (5)-(6): nx x ny nodes spanning [xmin, xmax] x [ymin, ymax]
    with both edges on nodes, spacing (max - min)/(count - 1)."""

    def __init__(self, xmin, xmax, ymin, ymax, nx, ny):
        self.xmin, self.xmax, self.ymin, self.ymax = float(xmin), float(xmax), float(ymin), float(ymax)
        self.nx, self.ny = int(nx), int(ny)

    @property
    def dx(self) -> float:
        return (self.xmax - self.xmin) / (self.nx - 1)

    @property
    def dy(self) -> float:
        return (self.ymax - self.ymin) / (self.ny - 1)

    def nodes(self):
        return self.xmin + np.arange(self.nx) * self.dx, self.ymin + np.arange(self.ny) * self.dy


def to_units(xy, grid: Grid) -> np.ndarray:
    """X_p = fl32((x_p - xmin)/dx), Y_p likewise: FP64 subtract and divide, one
    round-to-nearest-even to FP32."""
    xy = _f64(xy).reshape(-1, 2)
    out = np.empty(xy.shape, dtype=np.float32)
    out[:, 0] = ((xy[:, 0] - grid.xmin) / grid.dx).astype(np.float32)
    out[:, 1] = ((xy[:, 1] - grid.ymin) / grid.dy).astype(np.float32)
    return out


def bandwidth_units(hx: float, hy: float, grid: Grid) -> tuple[np.float32, np.float32]:
    """Hx = fl32(hx/dx), Hy = fl32(hy/dy)."""
    return np.float32(hx / grid.dx), np.float32(hy / grid.dy)


def density_scale(n: int, hx: float, hy: float) -> float:
    """Density normalisation 1/(n hx hy) in world units."""
    return 1.0 / (n * hx * hy)


# --------------------------------------------------------------------------- maps
def map_world(xy, kernel: int, hx: float, hy: float, grid: Grid, window=None, raw: bool = False) -> np.ndarray:
    """Density (or raw sum) at the grid nodes from FP64 world points; window =
    (i0, i1, j0, j1) half-open, default the whole grid.  Returns [rows, cols]."""
    xy = _f64(xy).reshape(-1, 2)
    i0, i1, j0, j1 = window if window is not None else (0, grid.nx, 0, grid.ny)
    out = np.empty((j1 - j0, i1 - i0))
    lib().ko_map_world(_ptr(xy), xy.shape[0], int(kernel), float(hx), float(hy), grid.xmin, grid.xmax,
                       grid.ymin, grid.ymax, grid.nx, grid.ny, i0, i1, j0, j1, int(raw), _ptr(out))
    return out


def map_units(XY, kernel: int, Hx, Hy, window) -> np.ndarray:
    """Raw sum S over window (i0, i1, j0, j1) from FP32 pixel coordinates."""
    XY = _f32(XY).reshape(-1, 2)
    i0, i1, j0, j1 = window
    out = np.empty((j1 - j0, i1 - i0))
    lib().ko_map_units(_ptr(XY), XY.shape[0], int(kernel), np.float32(Hx), np.float32(Hy), i0, i1, j0, j1,
                       _ptr(out))
    return out


def map_units_at(XY, kernel: int, Hx, Hy, ij) -> np.ndarray:
    """Raw sums at pixels ij[m, 2] = (i, j)."""
    XY = _f32(XY).reshape(-1, 2)
    ij = np.ascontiguousarray(ij, dtype=np.int32).reshape(-1, 2)
    out = np.empty(ij.shape[0])
    lib().ko_map_units_at(_ptr(XY), XY.shape[0], int(kernel), np.float32(Hx), np.float32(Hy), _ptr(ij),
                          ij.shape[0], _ptr(out))
    return out


def _factors(kernel: int, nodes: np.ndarray, coord: np.ndarray, H: np.float32, deriv: bool = False) -> np.ndarray:
    """[len(nodes), len(coord)] table of k((node - c)/H) (or k'), support test on
    the exact difference for compact kernels."""
    d = nodes[:, None].astype(np.float64) - coord[None, :].astype(np.float64)
    u = d / np.float64(H)
    val = (dk if deriv else k)(kernel, u)
    if kernel == GAUSS_TRUNC:
        val = np.where(np.abs(d) <= 8.0 * np.float64(H), val, 0.0)
    elif kernel != GAUSSIAN:
        val = np.where(np.abs(d) <= np.float64(H), val, 0.0)
    return val


def map_units_separable(XY, kernel: int, Hx, Hy, window, chunk: int = 1 << 15) -> np.ndarray:
    """Same raw sum as map_units, as sum over point chunks of Gy @ Gx^T."""
    XY = _f32(XY).reshape(-1, 2)
    i0, i1, j0, j1 = window
    cols, rows = np.arange(i0, i1), np.arange(j0, j1)
    out = np.zeros((j1 - j0, i1 - i0))
    for c0 in range(0, XY.shape[0], chunk):
        P = XY[c0:c0 + chunk]
        gx = _factors(kernel, cols, P[:, 0], Hx)
        gy = _factors(kernel, rows, P[:, 1], Hy)
        out += gy @ gx.T
    return out


# --------------------------------------------------------------------------- adjoint
def vjp_units(XY, kernel: int, Hx, Hy, gbar, sel=None):
    """Plain-loop VJP of the raw map: returns (g[m, 2] = dL/d(X_p, Y_p), gh[m, 2] =
    per-point shares of dL/d(Hx, Hy)) for points sel (default all)."""
    XY = _f32(XY).reshape(-1, 2)
    gbar = _f64(gbar)
    ny, nx = gbar.shape
    sel = np.arange(XY.shape[0], dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    g = np.empty((sel.size, 2))
    gh = np.empty((sel.size, 2))
    lib().ko_vjp_units(_ptr(XY), XY.shape[0], int(kernel), np.float32(Hx), np.float32(Hy), nx, ny, _ptr(gbar),
                       _ptr(sel), sel.size, _ptr(g), _ptr(gh))
    return g, gh


def vjp_units_separable(XY, kernel: int, Hx, Hy, gbar, chunk: int = 1 << 14):
    """Same as vjp_units for all points in factored form: with Kx[i,p], Ky[j,p]
    and derivatives Dx, Dy,
      dL/dX_p = -(1/Hx) sum_j Ky[j,p] (gbar @ Dx)[j,p],
      dL/dY_p = -(1/Hy) sum_i Kx[i,p] (gbar^T @ Dy)[i,p],
      share of dL/dHx = -(1/Hx) sum_j Ky[j,p] (gbar @ (s*Dx))[j,p], s = (i - X_p)/Hx."""
    XY = _f32(XY).reshape(-1, 2)
    gbar = _f64(gbar)
    ny, nx = gbar.shape
    cols, rows = np.arange(nx), np.arange(ny)
    n = XY.shape[0]
    g = np.empty((n, 2))
    gh = np.empty((n, 2))
    for c0 in range(0, n, chunk):
        P = XY[c0:c0 + chunk]
        kx = _factors(kernel, cols, P[:, 0], Hx)
        ky = _factors(kernel, rows, P[:, 1], Hy)
        dxk = _factors(kernel, cols, P[:, 0], Hx, deriv=True)
        dyk = _factors(kernel, rows, P[:, 1], Hy, deriv=True)
        s = (cols[:, None] - P[None, :, 0].astype(np.float64)) / np.float64(Hx)
        t = (rows[:, None] - P[None, :, 1].astype(np.float64)) / np.float64(Hy)
        zx = gbar @ dxk  # [ny, m]
        zy = gbar.T @ dyk  # [nx, m]
        zhx = gbar @ (s * dxk)
        zhy = gbar.T @ (t * dyk)
        m = P.shape[0]
        g[c0:c0 + m, 0] = -(ky * zx).sum(0) / np.float64(Hx)
        g[c0:c0 + m, 1] = -(kx * zy).sum(0) / np.float64(Hy)
        gh[c0:c0 + m, 0] = -(ky * zhx).sum(0) / np.float64(Hx)
        gh[c0:c0 + m, 1] = -(kx * zhy).sum(0) / np.float64(Hy)
    return g, gh


# --------------------------------------------------------------------------- LSCV
def lscv_world(xy, kernel: int, hx: float, hy: float):
    """(LSCV(hx, hy), [dLSCV/dhx, dLSCV/dhy]) from FP64 world points."""
    xy = _f64(xy).reshape(-1, 2)
    v = np.zeros(1)
    g = np.zeros(2)
    lib().ko_lscv_world(_ptr(xy), xy.shape[0], int(kernel), float(hx), float(hy), _ptr(v), _ptr(g))
    return float(v[0]), g


def lscv_units(XY, kernel: int, Hx, Hy):
    """LSCV and its bandwidth gradient in grid units from FP32 pixel coordinates."""
    XY = _f32(XY).reshape(-1, 2)
    v = np.zeros(1)
    g = np.zeros(2)
    lib().ko_lscv_units(_ptr(XY), XY.shape[0], int(kernel), np.float32(Hx), np.float32(Hy), _ptr(v), _ptr(g))
    return float(v[0]), g


# --------------------------------------------------------------------------- errors
def bin_counts(XY, labels, nx: int, ny: int):
    """The paper's count matrix (Eq. (5)-(6) ceil projection, Eq. (12)-(13) gap
    filling between consecutive points with equal labels; labels None: no
    filling): (counts uint32 [ny, nx], number of counted cells)."""
    XY = _f32(XY).reshape(-1, 2)
    counts = np.zeros((ny, nx), dtype=np.uint32)
    total = ctypes.c_int64()
    lab = None
    if labels is not None:
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        assert lab.shape == (XY.shape[0],)
    lib().ko_bin_counts(_ptr(XY), XY.shape[0], _ptr(lab) if lab is not None else None, nx, ny, _ptr(counts),
                        ctypes.byref(total))
    return counts, int(total.value)


def conv_counts(counts, kernel: int, Hx, Hy, a: int, b: int, window=None) -> np.ndarray:
    """Eq. (7): raw convolution of a count matrix with the taps k(s/Hx) k(t/Hy),
    |s| <= a, |t| <= b, over window (i0, i1, j0, j1) (default: whole grid)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    ny, nx = counts.shape
    i0, i1, j0, j1 = window if window is not None else (0, nx, 0, ny)
    out = np.empty((j1 - j0, i1 - i0), dtype=np.float64)
    lib().ko_conv_counts(_ptr(counts), nx, ny, kernel, float(np.float32(Hx)), float(np.float32(Hy)), int(a),
                         int(b), i0, i1, j0, j1, _ptr(out))
    return out


def dp_keep(xy_m, lengths, eps: float):
    """Douglas-Peucker keep mask (uint8 [n]) of tracks given by their lengths,
    points in metres (FP64 [n, 2]); see ko_dp_keep for the decision rule."""
    xy = _f64(xy_m).reshape(-1, 2)
    start = np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))]).astype(np.int64)
    assert start[-1] == xy.shape[0]
    keep = np.zeros(xy.shape[0], dtype=np.uint8)
    lib().ko_dp_keep(_ptr(xy), xy.shape[0], _ptr(start), len(start) - 1, float(eps), _ptr(keep))
    return keep


def track_length(xy) -> float:
    """|T| = sum of |P_n P_{n+1}| over consecutive points (Eq. (15))."""
    xy = _f64(xy).reshape(-1, 2)
    return float(lib().ko_track_length(_ptr(xy), xy.shape[0]))


def dtw(a, b) -> float:
    """Squared-Euclidean DTW distance sqrt(D[N_o, N_c]) of Eq. (16)-(18)."""
    a = _f64(a).reshape(-1, 2)
    b = _f64(b).reshape(-1, 2)
    return float(lib().ko_dtw(_ptr(a), a.shape[0], _ptr(b), b.shape[0]))


def _starts(lengths):
    return np.concatenate([[0], np.cumsum(np.asarray(lengths, dtype=np.int64))]).astype(np.int64)


def track_metrics(xy_o, lengths_o, xy_c, lengths_c) -> dict:
    """Compression quality of M tracks against their compressed versions
    (Sec. V-B): per track |T_m|, |T'_m| and DTW(T_m, T'_m); over the set
    N_o, N_c, CR = (1 - N_c / N_o) * 100 (Eq. (14)), RLL = (sum |T| - sum |T'|)
    / sum |T| (Eq. (15), a fraction), the mean mu and population standard
    deviation delta of the DTW distances (Eq. (19)-(20)).  The sums over tracks
    are exactly rounded (math.fsum); delta is taken about the computed mu."""
    import math
    xo = _f64(xy_o).reshape(-1, 2)
    xc = _f64(xy_c).reshape(-1, 2)
    so, sc = _starts(lengths_o), _starts(lengths_c)
    m = len(so) - 1
    assert len(sc) - 1 == m and so[-1] == xo.shape[0] and sc[-1] == xc.shape[0]
    lo, lc, dw = (np.zeros(m) for _ in range(3))
    lib().ko_track_metrics(_ptr(xo), _ptr(so), _ptr(xc), _ptr(sc), m, _ptr(lo), _ptr(lc), _ptr(dw))
    n_o, n_c = int(xo.shape[0]), int(xc.shape[0])
    tot_o, tot_c = math.fsum(lo), math.fsum(lc)
    nan = float("nan")
    mu = math.fsum(dw) / m if m else nan
    delta = math.sqrt(math.fsum((v - mu) ** 2 for v in dw) / m) if m else nan
    return {"len_o": lo, "len_c": lc, "dtw": dw, "n_original": n_o, "n_compressed": n_c,
            "cr_percent": (1.0 - n_c / n_o) * 100.0 if n_o else nan,
            "length_original": tot_o, "length_compressed": tot_c,
            "rll": (tot_o - tot_c) / tot_o if tot_o != 0.0 else nan,
            "dtw_mean": mu, "dtw_std": delta}


def errors(y, r) -> dict:
    """Peak-normalised max error e_inf = max|y - r| / max|r|, relative L2 error
    e_2 = ||y - r|| / ||r||, and the max per-pixel relative error over pixels
    with r >= 1e-3 max r."""
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    peak = np.max(np.abs(r))
    diff = np.abs(y - r)
    e_inf = float(diff.max() / peak) if peak > 0 else float(diff.max())
    nr = np.linalg.norm(r)
    e_2 = float(np.linalg.norm(y - r) / nr) if nr > 0 else float(np.linalg.norm(y - r))
    mask = np.abs(r) >= 1e-3 * peak
    e_rel = float((diff[mask] / np.abs(r[mask])).max()) if mask.any() else 0.0
    return {"e_inf": e_inf, "e_2": e_2, "e_rel": e_rel}
