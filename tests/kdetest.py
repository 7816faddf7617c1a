"""Shared helpers of the GPU parity tests: seeded workloads in grid units, GPU
evaluation through the C ABI, and pixel samples for full-size checks."""
from __future__ import annotations

import functools
import sys

import numpy as np

import oracle
import paper_2004_13653_amd as kde
import synth

FP32_GATE = 1e-5  # peak-normalised max error of the FP32 paths against FP64


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def device():
    import torch
    return torch.device("cuda:0")


@functools.lru_cache(maxsize=None)
def lanes(n_tracks: int, pts: int, seed_index: int = 1) -> synth.Tracks:
    return synth.workload_lanes(n_tracks=n_tracks, pts=pts, seed_index=seed_index)


@functools.lru_cache(maxsize=None)
def lanes_dp(n_tracks: int, pts: int, eps: float, seed_index: int = 1) -> synth.Tracks:
    return synth.dp_compress(lanes(n_tracks, pts, seed_index), eps)


def grids(box: synth.Box, nx: int, ny: int):
    """(library grid, oracle grid) over the same box."""
    return kde.Grid(box.lon0, box.lon1, box.lat0, box.lat1, nx, ny), \
        oracle.Grid(box.lon0, box.lon1, box.lat0, box.lat1, nx, ny)


def to_device(XY: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(XY, dtype=np.float32)).to(device())


def gpu_map(XY: np.ndarray, kernel: int, hx: float, hy: float, grid: kde.Grid, precision: str = "fp32",
            raw: bool = False) -> np.ndarray:
    import torch
    pts = to_device(XY)
    out = kde.eval(pts, kernel, hx, hy, grid, precision=precision, raw=raw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def oracle_density_window(XY, kernel, hx, hy, og: oracle.Grid, window, separable: bool = False) -> np.ndarray:
    Hx, Hy = oracle.bandwidth_units(hx, hy, og)
    f = oracle.map_units_separable if separable else oracle.map_units
    return f(XY, kernel, Hx, Hy, window) * oracle.density_scale(XY.shape[0], hx, hy)


def oracle_density_at(XY, kernel, hx, hy, og: oracle.Grid, ij) -> np.ndarray:
    Hx, Hy = oracle.bandwidth_units(hx, hy, og)
    return oracle.map_units_at(XY, kernel, Hx, Hy, ij) * oracle.density_scale(XY.shape[0], hx, hy)


def sample_pixels(gmap: np.ndarray, n_random: int, seed: int) -> np.ndarray:
    """Pixels to check at full size: the GPU map's peak and its 5x5 neighbourhood,
    the four corners, the peaks of each map quadrant, and n_random uniform ones.
    Returns ij[m, 2] = (i, j)."""
    ny, nx = gmap.shape
    rng = np.random.default_rng(seed)
    pts = set()
    jp, ip = np.unravel_index(np.argmax(gmap), gmap.shape)
    for dj in range(-2, 3):
        for di in range(-2, 3):
            pts.add((min(max(ip + di, 0), nx - 1), min(max(jp + dj, 0), ny - 1)))
    pts |= {(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)}
    for qj in (slice(0, ny // 2), slice(ny // 2, ny)):
        for qi in (slice(0, nx // 2), slice(nx // 2, nx)):
            sub = gmap[qj, qi]
            a, b = np.unravel_index(np.argmax(sub), sub.shape)
            pts.add((qi.start + b, qj.start + a))
    for _ in range(n_random):
        pts.add((int(rng.integers(0, nx)), int(rng.integers(0, ny))))
    return np.array(sorted(pts), dtype=np.int32)


def peak_error(y, r) -> float:
    """max |y - r| / max |r| over the compared outputs."""
    y = np.asarray(y, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.max(np.abs(y - r)) / np.max(np.abs(r)))


def mass_window(XY: np.ndarray, nx: int, ny: int, side: int = 256, stride: int = 64) -> tuple:
    """The side x side window, corners on multiples of stride, that holds the
    most points (the crop with the largest mass), as (i0, i1, j0, j1).  Chosen
    from the inputs alone, so every path is compared on the same window."""
    bx, by = nx // stride, ny // stride
    cnt, _, _ = np.histogram2d(XY[:, 1], XY[:, 0], bins=[by, bx], range=[[0, by * stride], [0, bx * stride]])
    w = side // stride
    best, arg = -1.0, (0, 0)
    for b in range(by - w + 1):
        for a in range(bx - w + 1):
            s = cnt[b:b + w, a:a + w].sum()
            if s > best:
                best, arg = s, (a, b)
    i0, j0 = arg[0] * stride, arg[1] * stride
    return (i0, i0 + side, j0, j0 + side)


_ORACLE_CACHE: dict = {}


def cached(key, compute):
    """Oracle results shared by several tests of one session (the large windows
    take tens of seconds on the host)."""
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = compute()
    return _ORACLE_CACHE[key]
