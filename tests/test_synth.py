"""The seeded synthetic AIS generator and the Douglas-Peucker input preparation."""
import math

import numpy as np

import synth
from synth import ais


def test_small_workload_shape_and_determinism():
    a, b = synth.workload_small(), synth.workload_small()
    assert a.n == 2000 and a.xy.shape == (2000, 2) and a.xy.dtype == np.float64
    np.testing.assert_array_equal(a.xy, b.xy)
    assert list(a.lengths) == [100] * 20
    box = synth.BOX_C1
    assert (a.xy[:, 0] >= box.lon0).all() and (a.xy[:, 0] <= box.lon1).all()
    assert (a.xy[:, 1] >= box.lat0).all() and (a.xy[:, 1] <= box.lat1).all()


def test_lane_track_kinematics():
    """Speeds 5-15 kn at 10 s reports, lateral scatter N(0, 50 m) about the lane."""
    t = synth.generate(123, 40, 300, synth.BOX_C2, n_lanes=1)
    mlon, mlat = synth.metres_per_degree(synth.BOX_C2.center_lat)
    speeds = []
    for k in range(40):
        p = t.xy[k * 300:(k + 1) * 300]
        x = (p[:, 0] - synth.BOX_C2.lon0) * mlon
        y = (p[:, 1] - synth.BOX_C2.lat0) * mlat
        # end-to-end speed along the (single) lane direction
        d = math.hypot(x[-1] - x[0], y[-1] - y[0])
        speeds.append(d / (299 * ais.DT) / ais.KNOT)
        # residual about the least-squares line = lateral scatter
        A = np.column_stack([x, np.ones_like(x)])
        if np.ptp(x) > np.ptp(y):
            coef, *_ = np.linalg.lstsq(A, y, rcond=None)
            res = (y - A @ coef) / math.sqrt(1 + coef[0] ** 2)
        else:
            B = np.column_stack([y, np.ones_like(y)])
            coef, *_ = np.linalg.lstsq(B, x, rcond=None)
            res = (x - B @ coef) / math.sqrt(1 + coef[0] ** 2)
        assert 35.0 < res.std() < 65.0
    speeds = np.array(speeds)
    assert speeds.min() > 4.5 and speeds.max() < 15.5


def test_anchored_fraction():
    t = synth.generate(5, 100, 200, synth.BOX_C2, n_lanes=3, anchored_frac=0.1)
    assert t.n == 20000
    # anchored tracks have no along-track drift: first-to-last distance ~ scatter
    mlon, mlat = synth.metres_per_degree(synth.BOX_C2.center_lat)
    drift = []
    for k in range(100):
        p = t.xy[k * 200:(k + 1) * 200]
        drift.append(math.hypot((p[-1, 0] - p[0, 0]) * mlon, (p[-1, 1] - p[0, 1]) * mlat))
    assert sum(d < 2000.0 for d in drift) == 10


def test_mercator_textbook_values():
    """Eq. (1)-(4) on WGS84 at the equator: x = a * lambda, y(0) = 0, and the
    isometric latitude of 45 degrees."""
    x, y = synth.mercator(np.array([1.0, 0.0]), np.array([0.0, 45.0]), 0.0)
    assert x[0] == ais.WGS84_A * math.radians(1.0)
    assert abs(y[0]) < 1e-6
    e = math.sqrt(ais.WGS84_E2)
    phi = math.radians(45.0)
    q = math.atanh(math.sin(phi)) - e * math.atanh(e * math.sin(phi))
    assert abs(y[1] - ais.WGS84_A * q) < 1e-6


def _dp(x, y, eps):
    return np.flatnonzero(ais._dp_keep(np.asarray(x, float), np.asarray(y, float), eps))


def test_dp_textbook_cases():
    # collinear points: only the end points survive
    assert list(_dp(np.arange(10.0), 2 * np.arange(10.0), 0.0)) == [0, 9]
    # one spike of height 5: kept for eps < 5, dropped at eps = 5 (strictly larger)
    y = np.zeros(9)
    y[4] = 5.0
    assert list(_dp(np.arange(9.0), y, 4.999)) == [0, 4, 8]
    assert list(_dp(np.arange(9.0), y, 5.0)) == [0, 8]
    # equal maxima at indices 1 and 3 (then 2 and 3): the lower index wins each tie
    assert list(_dp([0.0, 1.0, 2.0, 3.0, 4.0], [0.0, 1.0, 0.0, 1.0, 0.0], 0.7)) == [0, 1, 4]
    # distance to the line, not the segment: a point beyond the chord's end
    assert list(_dp([0.0, 10.0, 5.0], [0.0, 0.0, 0.0], 0.0)) == [0, 2]
    # closed loop (coinciding end points): distance to that point
    assert list(_dp([0.0, 3.0, 0.0], [0.0, 4.0, 0.0], 4.9)) == [0, 1, 2]


def test_dp_compress_counts():
    t = synth.generate(9, 30, 200, synth.BOX_C2, n_lanes=2)
    c10 = synth.dp_compress(t, 10.0)
    c100 = synth.dp_compress(t, 100.0)
    assert c10.lengths.sum() == c10.n and c100.n < c10.n < t.n
    assert (c100.lengths >= 2).all()
    assert 0.0 < synth.compression_ratio(t, c10) < synth.compression_ratio(t, c100) < 100.0


def test_window_tracks_cuts_the_pool_at_both_ends():
    t = synth.workload_lanes(n_tracks=7, pts=10, seed_index=1)
    w = synth.window_tracks(t, 13, 25)
    np.testing.assert_array_equal(w.xy, t.xy[13:38])
    assert list(w.lengths) == [7, 10, 8]
    assert synth.window_tracks(t, 20, 10).lengths.tolist() == [10]
    assert synth.window_tracks(t, 0, 70).lengths.tolist() == [10] * 7


def test_batch_specs_thresholds_do_not_move_other_draws():
    a = synth.batch_specs(50, 10**6)
    b = synth.batch_specs(50, 10**6, eps_choices=(0.0,))
    assert [(s.start, s.count, s.side, s.h_deg, s.kernel) for s in a] == \
           [(s.start, s.count, s.side, s.h_deg, s.kernel) for s in b]
    assert {s.eps_m for s in a} == {0.0, 10.0, 50.0, 100.0}
    assert {s.eps_m for s in b} == {0.0}
