"""Seeded synthetic AIS-shaped vessel trajectories (the inputs of every test and
benchmark).

The paper's three AIS data sets (Sec. V-A, Table III) are not available, so these
generators stand in for them.  They reproduce the shapes the paper describes:
vessels moving along straight traffic lanes at 5-15 kn, reported every 10 s
(AIS intervals are 2-180 s, Sec. III-C), with a few lanes crossing and some
vessels anchored, all trajectories merged track-major into one buffer with a
per-track length array (Sec. IV-C, "Compression of Massive Trajectories").

This module holds no KDE arithmetic.  The Douglas-Peucker compressor and the
Mercator projection below are input preparation: they produce the compressed
point sets the heat map is evaluated on (Sec. III-A, III-B).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KNOT = 1852.0 / 3600.0  # m/s
DT = 10.0  # s between reports

# WGS84 ellipsoid (a, f): the paper leaves a and e of Eq. (1)-(2) unspecified.
WGS84_A = 6378137.0
WGS84_F = 1.0 / 298.257223563
WGS84_E2 = WGS84_F * (2.0 - WGS84_F)


@dataclass(frozen=True)
class Box:
    lon0: float
    lon1: float
    lat0: float
    lat1: float

    @property
    def center_lat(self) -> float:
        return 0.5 * (self.lat0 + self.lat1)


BOX_C1 = Box(121.40, 121.60, 31.20, 31.40)  # 0.2 x 0.2 degrees
BOX_C2 = Box(122.0, 123.0, 30.0, 31.0)  # 1 x 1 degree


def metres_per_degree(lat_deg: float) -> tuple[float, float]:
    """(metres per degree of longitude, metres per degree of latitude) on WGS84
    at latitude lat_deg: N cos(phi) pi/180 and M pi/180."""
    phi = math.radians(lat_deg)
    w = 1.0 - WGS84_E2 * math.sin(phi) ** 2
    n_rad = WGS84_A / math.sqrt(w)
    m_rad = WGS84_A * (1.0 - WGS84_E2) / w ** 1.5
    return n_rad * math.cos(phi) * math.pi / 180.0, m_rad * math.pi / 180.0


def mercator(lon_deg: np.ndarray, lat_deg: np.ndarray, lat_std_deg: float) -> tuple[np.ndarray, np.ndarray]:
    """Mercator projection of Eq. (1)-(4): x = lambda r0, y = q r0 with r0 the
    radius of the parallel at the standard latitude and q the isometric
    latitude; angles in radians, result in metres."""
    e = math.sqrt(WGS84_E2)
    phi0 = math.radians(lat_std_deg)
    r0 = WGS84_A / math.sqrt(1.0 - WGS84_E2 * math.sin(phi0) ** 2) * math.cos(phi0)
    lam = np.radians(lon_deg)
    phi = np.radians(lat_deg)
    es = e * np.sin(phi)
    q = np.log(np.tan(math.pi / 4.0 + phi / 2.0)) + (e / 2.0) * np.log((1.0 - es) / (1.0 + es))
    return lam * r0, q * r0


@dataclass
class Tracks:
    """Track-major merged buffer: xy[n, 2] = (lon, lat) degrees, FP64, and the
    per-track lengths (their sum is n)."""

    xy: np.ndarray
    lengths: np.ndarray
    box: Box

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])


def _chord(c: np.ndarray, u: np.ndarray, box_m: tuple[float, float, float, float]) -> tuple[float, float]:
    """Parameter range [t0, t1] of the line c + t u (metres) inside the box."""
    x0, x1, y0, y1 = box_m
    lo, hi = -math.inf, math.inf
    for ci, ui, a, b in ((c[0], u[0], x0, x1), (c[1], u[1], y0, y1)):
        if abs(ui) < 1e-12:
            continue
        ta, tb = (a - ci) / ui, (b - ci) / ui
        lo, hi = max(lo, min(ta, tb)), min(hi, max(ta, tb))
    return lo, hi


def _lane_track(rng, npts, lane, box_m, lat_sd_m):
    """One vessel along a straight lane: monotone random walk along the lane,
    i.i.d. lateral N(0, lat_sd_m) offsets.  Returns metres or None if the
    track does not fit the lane's chord inside the box."""
    c, u = lane
    v = rng.uniform(5.0, 15.0) * KNOT
    steps = v * DT * np.maximum(0.0, 1.0 + 0.1 * rng.standard_normal(npts - 1))
    along = np.concatenate(([0.0], np.cumsum(steps)))
    length = along[-1]
    t0, t1 = _chord(c, u, box_m)
    if t1 - t0 <= length:
        return None
    start = rng.uniform(t0, t1 - length)
    if rng.random() < 0.5:
        t = start + along
    else:
        t = (start + length) - along
    lat_off = rng.normal(0.0, lat_sd_m, npts)
    nrm = np.array([-u[1], u[0]])
    pts = c[None, :] + t[:, None] * u[None, :] + lat_off[:, None] * nrm[None, :]
    return pts


def _draw_lane(rng, box_m):
    x0, x1, y0, y1 = box_m
    cx = rng.uniform(x0 + 0.25 * (x1 - x0), x1 - 0.25 * (x1 - x0))
    cy = rng.uniform(y0 + 0.25 * (y1 - y0), y1 - 0.25 * (y1 - y0))
    th = rng.uniform(0.0, math.pi)
    return np.array([cx, cy]), np.array([math.cos(th), math.sin(th)])


def generate(seed: int, n_tracks: int, pts_per_track: int, box: Box, n_lanes: int | None = None,
             anchored_frac: float = 0.0, n_anchorages: int = 5, lateral_sd_m: float = 50.0,
             anchor_sd_m: float = 200.0) -> Tracks:
    """Tracks along n_lanes shared lanes (each through the central 50 % of the
    box, so they cross), a fraction anchored_frac of the tracks instead
    scattered i.i.d. N(centre, anchor_sd_m) around one of n_anchorages centres
    drawn in the inner 80 %.  Coordinates are planar metres about the box's
    south-west corner, converted to degrees at the box-centre latitude."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mlon, mlat = metres_per_degree(box.center_lat)
    box_m = (0.0, (box.lon1 - box.lon0) * mlon, 0.0, (box.lat1 - box.lat0) * mlat)
    if n_lanes is None:
        n_lanes = int(rng.integers(3, 7))
    lanes = [_draw_lane(rng, box_m) for _ in range(n_lanes)]
    n_anch = int(round(anchored_frac * n_tracks))
    anchors = np.stack([
        np.array([rng.uniform(0.1 * box_m[1], 0.9 * box_m[1]), rng.uniform(0.1 * box_m[3], 0.9 * box_m[3])])
        for _ in range(n_anchorages)]) if n_anch else None
    anchored = np.zeros(n_tracks, dtype=bool)
    if n_anch:
        anchored[rng.choice(n_tracks, size=n_anch, replace=False)] = True
    out = np.empty((n_tracks * pts_per_track, 2))
    for k in range(n_tracks):
        if anchored[k]:
            c = anchors[int(rng.integers(0, n_anchorages))]
            pts = c[None, :] + rng.normal(0.0, anchor_sd_m, (pts_per_track, 2))
        else:
            pts = None
            for _ in range(1000):
                lane = lanes[int(rng.integers(0, n_lanes))]
                pts = _lane_track(rng, pts_per_track, lane, box_m, lateral_sd_m)
                if pts is not None:
                    break
                if n_lanes == 1:
                    lanes[0] = _draw_lane(rng, box_m)
            if pts is None:
                raise RuntimeError("could not fit a track into the box")
        out[k * pts_per_track:(k + 1) * pts_per_track, 0] = box.lon0 + pts[:, 0] / mlon
        out[k * pts_per_track:(k + 1) * pts_per_track, 1] = box.lat0 + pts[:, 1] / mlat
    return Tracks(out, np.full(n_tracks, pts_per_track, dtype=np.int64), box)


# ---------------------------------------------------------------------------
# Workloads.  Seeds are 20041365 + the workload's index.
SEED0 = 20041365


def workload_small() -> Tracks:
    """20 tracks x 100 points on one lane in a 0.2 x 0.2 degree box."""
    return generate(SEED0 + 0, 20, 100, BOX_C1, n_lanes=1)


def workload_lanes(n_tracks: int = 2000, pts: int = 500, seed_index: int = 1) -> Tracks:
    """Crossing lanes (3-6) plus 10 % anchored tracks in a 1 x 1 degree box."""
    return generate(SEED0 + seed_index, n_tracks, pts, BOX_C2, n_lanes=None, anchored_frac=0.1)


# ---------------------------------------------------------------------------
# Douglas-Peucker compression (input preparation, Sec. III-B).

def _dp_keep(x: np.ndarray, y: np.ndarray, eps: float) -> np.ndarray:
    """Recursive Douglas-Peucker on one track in metres: keep both end points;
    in each segment keep the interior point whose distance to the line through
    the segment's end points (Eq. (9)) is largest if that distance exceeds eps
    (strictly), the lowest index winning ties; a segment whose end points
    coincide uses the distance to that point."""
    n = x.shape[0]
    keep = np.zeros(n, dtype=bool)
    keep[0] = keep[-1] = True
    stack = [(0, n - 1)]
    while stack:
        s, e = stack.pop()
        if e - s < 2:
            continue
        px, py = x[s + 1:e] - x[s], y[s + 1:e] - y[s]
        cx, cy = x[e] - x[s], y[e] - y[s]
        chord = math.hypot(cx, cy)
        if chord > 0.0:
            d = np.abs(px * cy - py * cx) / chord
        else:
            d = np.hypot(px, py)
        m = int(np.argmax(d))
        if d[m] > eps:
            k = s + 1 + m
            keep[k] = True
            stack.append((k, e))
            stack.append((s, k))
    return keep


def dp_compress(tracks: Tracks, eps_m: float) -> Tracks:
    """Compress every track at threshold eps_m metres (eps 0 keeps every point
    off the chord; collinear points at distance 0 are dropped)."""
    if eps_m < 0:
        raise ValueError("eps must be >= 0")
    mx, my = mercator(tracks.xy[:, 0], tracks.xy[:, 1], tracks.box.center_lat)
    keep_all = np.zeros(tracks.n, dtype=bool)
    off = 0
    lens = []
    for L in tracks.lengths:
        L = int(L)
        k = _dp_keep(mx[off:off + L], my[off:off + L], eps_m)
        keep_all[off:off + L] = k
        lens.append(int(k.sum()))
        off += L
    return Tracks(tracks.xy[keep_all].copy(), np.asarray(lens, dtype=np.int64), tracks.box)


def compression_ratio(original: Tracks, compressed: Tracks) -> float:
    """CR = (1 - N_c / N_o) x 100 % (Eq. (14))."""
    return (1.0 - compressed.n / original.n) * 100.0


# ---------------------------------------------------------------------------
# Batches of maps ("time windows" of one large pool of tracks).

@dataclass
class MapSpec:
    start: int      # first point of the contiguous slice of the pool
    count: int      # number of points
    side: int       # grid is side x side over the pool's box
    h_deg: float    # hx = hy
    kernel: int     # Table I kernel id
    eps_m: float = 0.0  # Douglas-Peucker threshold the window is compressed at (0: raw)


def batch_specs(n_maps: int, pool_points: int, seed: int = SEED0 + 4, min_points: int = 1000,
                max_points: int = 200_000, sides=(256, 512, 1024), h_range=(0.001, 0.008),
                eps_choices=(0.0, 10.0, 50.0, 100.0)) -> list[MapSpec]:
    """Per-map point counts log-uniform in [min_points, max_points], grid sides
    drawn uniformly from `sides`, bandwidth U(h_range), kernel uniform over the
    eight; each map is a contiguous slice (a time window) of the pool, to be
    Douglas-Peucker-compressed at a threshold drawn uniformly from eps_choices
    (a second generator, so the other draws do not depend on it)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rng_eps = np.random.Generator(np.random.PCG64(seed + 1))
    specs = []
    for _ in range(n_maps):
        count = int(round(math.exp(rng.uniform(math.log(min_points), math.log(max_points)))))
        count = min(count, pool_points)
        start = int(rng.integers(0, pool_points - count + 1))
        specs.append(MapSpec(start, count, int(rng.choice(sides)), float(rng.uniform(*h_range)),
                             int(rng.integers(0, 8)), float(rng_eps.choice(eps_choices))))
    return specs


def window_tracks(pool: Tracks, start: int, count: int) -> Tracks:
    """The points [start, start + count) of the pool's merged buffer as tracks:
    the pool's tracks cut at the window's two ends."""
    ends = np.cumsum(np.asarray(pool.lengths, dtype=np.int64))
    begins = ends - pool.lengths
    lo = np.maximum(begins, start)
    hi = np.minimum(ends, start + count)
    lens = (hi - lo)[hi > lo]
    return Tracks(pool.xy[start:start + count].copy(), lens.astype(np.int64), pool.box)
