"""Pins of the FP64 oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every check is a printed value
(Table I), a closed form (unit mass, moments, roughness, single-point map), an
independent library routine (scipy.stats densities), a numerical integral, an
exact symmetry of the definition, or a finite difference of an already pinned
function.  A dropped term, a wrong sign, exponent or index, or transposed x/y
in the oracle fails at least one of them.
"""
import math
from fractions import Fraction
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import synth
from synth import ais
from oracle import GAUSSIAN, Grid

HERE = os.path.dirname(os.path.abspath(__file__))
K = list(range(8))
COMPACT = [0, 1, 2, 3, 4, 5, 7]


def _golden_table1():
    rows = {}
    env = {"__builtins__": {}, "pi": math.pi, "sqrt": math.sqrt, "exp": math.exp, "cos": math.cos}
    with open(os.path.join(HERE, "golden", "table1_kernel_constants.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, f00, fhalf = line.split()
            rows[name] = (eval(f00.replace("^", "**"), env), eval(fhalf.replace("^", "**"), env))
    return rows


# --------------------------------------------------------------------- 1-D factors
@pytest.mark.parametrize("kernel", K)
def test_table1_printed_values(kernel):
    """f(0,0) and f(1/2,1/2) of Table I equal k(0)^2 and k(1/2)^2."""
    f00, fhalf = _golden_table1()[oracle.KERNELS[kernel]]
    k0, kh = oracle.k(kernel, [0.0, 0.5])
    assert k0 * k0 == pytest.approx(f00, rel=1e-15)
    assert kh * kh == pytest.approx(fhalf, rel=1e-14)


# Closed forms: second moment mu2 = int u^2 k and roughness R = int k^2 of the
# textbook kernels with support [-1, 1] (Gaussian: whole line).
MU2 = [1 / 3, 1 / 6, 1 / 5, 1 / 7, 1 / 9, 35 / 243, 1.0, 1 - 8 / math.pi ** 2]
ROUGH = [1 / 2, 2 / 3, 3 / 5, 5 / 7, 350 / 429, 175 / 247, 1 / (2 * math.sqrt(math.pi)), math.pi ** 2 / 16]


def _quad(fn, kernel):
    lim = (-40.0, 40.0) if kernel == GAUSSIAN else (-1.0, 1.0)
    pts = None if kernel == GAUSSIAN else [0.0]
    v, _ = integrate.quad(fn, *lim, points=pts, epsabs=1e-14, epsrel=1e-13, limit=400)
    return v


@pytest.mark.parametrize("kernel", K)
def test_unit_mass(kernel):
    assert _quad(lambda u: oracle.k(kernel, [u])[0], kernel) == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("kernel", K)
def test_first_and_second_moment(kernel):
    assert abs(_quad(lambda u: u * oracle.k(kernel, [u])[0], kernel)) < 1e-13
    assert _quad(lambda u: u * u * oracle.k(kernel, [u])[0], kernel) == pytest.approx(MU2[kernel], rel=1e-11)


@pytest.mark.parametrize("kernel", K)
def test_roughness(kernel):
    assert _quad(lambda u: oracle.k(kernel, [u])[0] ** 2, kernel) == pytest.approx(ROUGH[kernel], rel=1e-11)


@pytest.mark.parametrize("kernel", COMPACT)
def test_support_edge(kernel):
    """Indicator of Eq. (8) read as |u| <= 1 inclusive: zero just outside, the
    boundary value at +-1 (1/2 for the uniform kernel, 0 otherwise)."""
    out = oracle.k(kernel, [-1.0 - 1e-12, 1.0 + 1e-12, 3.0, -7.5])
    assert np.all(out == 0.0)
    edge = oracle.k(kernel, [-1.0, 1.0])
    want = 0.5 if kernel == 0 else 0.0
    assert np.allclose(edge, want, atol=1e-15)


def test_library_densities():
    """Six of the eight factors are textbook densities in scipy.stats: uniform,
    symmetric triangular, Beta(a, a) on [-1, 1] for a = 2, 3, 4 (Epanechnikov,
    quartic, triweight) and the standard normal."""
    u = np.linspace(-1.3, 1.3, 1041)
    lib = {
        0: stats.uniform(loc=-1, scale=2).pdf(u),
        1: stats.triang(c=0.5, loc=-1, scale=2).pdf(u),
        2: stats.beta(2, 2, loc=-1, scale=2).pdf(u),
        3: stats.beta(3, 3, loc=-1, scale=2).pdf(u),
        4: stats.beta(4, 4, loc=-1, scale=2).pdf(u),
        6: stats.norm.pdf(u),
    }
    inside = np.abs(np.abs(u) - 1.0) > 1e-9  # the libraries differ on the closed/open end
    for kernel, ref in lib.items():
        np.testing.assert_allclose(oracle.k(kernel, u)[inside], ref[inside], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kernel", K)
def test_derivative_matches_difference(kernel):
    u = np.array([-0.93, -0.51, -0.2, 0.13, 0.47, 0.88, 1.7, -2.4])
    eps = 1e-6
    fd = (oracle.k(kernel, u + eps) - oracle.k(kernel, u - eps)) / (2 * eps)
    np.testing.assert_allclose(oracle.dk(kernel, u), fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("kernel", K)
def test_autoconvolution(kernel):
    """kbar(u) = int k(v) k(u - v) dv by adaptive quadrature (scipy) of the
    pinned factor; kbar(0) is the roughness; unit mass; derivative against a
    central difference."""
    for u in (0.0, 0.3, 0.9, 1.0, 1.5, 1.99, -0.7, 2.5):
        brk = sorted({x for x in (u - 1, u + 1, 0.0, u) if -1 < x < 1})
        conv = _quad(lambda v: oracle.k(kernel, [v])[0] * oracle.k(kernel, [u - v])[0], kernel) \
            if kernel == GAUSSIAN else integrate.quad(
                lambda v: oracle.k(kernel, [v])[0] * oracle.k(kernel, [u - v])[0], -1, 1,
                points=brk or None, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
        assert oracle.kbar(kernel, [u])[0] == pytest.approx(conv, rel=1e-10, abs=1e-14)
    assert oracle.kbar(kernel, [0.0])[0] == pytest.approx(ROUGH[kernel], rel=1e-14)
    lim = 40.0 if kernel == GAUSSIAN else 2.0
    mass = integrate.quad(lambda u: oracle.kbar(kernel, [u])[0], -lim, lim, points=[-1.0, 0.0, 1.0],
                          epsabs=1e-13, limit=200)[0]
    assert mass == pytest.approx(1.0, abs=1e-11)
    u = np.array([-1.7, -0.4, 0.25, 0.8, 1.1, 1.9])
    fd = (oracle.kbar(kernel, u + 1e-6) - oracle.kbar(kernel, u - 1e-6)) / 2e-6
    np.testing.assert_allclose(oracle.dkbar(kernel, u), fd, rtol=1e-7, atol=1e-9)


def test_autoconvolution_closed_forms():
    """Textbook autoconvolutions: two boxes give a triangle, (2 - |u|)/4; the
    triangle is the convolution of two unit boxes, so its autoconvolution is the
    centred cubic B-spline; the cosine factor's follows from the product-to-sum
    formula, (pi^2/32) ((2/pi) sin(pi a/2) + (2 - a) cos(pi a/2)), a = |u| <= 2."""
    u = np.array([-1.9, -1.2, -0.6, 0.0, 0.35, 0.999, 1.0, 1.4, 1.95, 2.0, 2.3])
    a = np.abs(u)
    np.testing.assert_allclose(oracle.kbar(0, u), np.where(a < 2, (2 - a) / 4, 0.0), rtol=1e-13, atol=1e-15)
    bs = np.where(a <= 1, (4 - 6 * a ** 2 + 3 * a ** 3) / 6, np.where(a < 2, (2 - a) ** 3 / 6, 0.0))
    np.testing.assert_allclose(oracle.kbar(1, u), bs, rtol=1e-13, atol=1e-15)
    cz = np.where(a < 2, math.pi ** 2 / 32 * ((2 / math.pi) * np.sin(math.pi * a / 2) + (2 - a) * np.cos(math.pi * a / 2)),
                  0.0)
    np.testing.assert_allclose(oracle.kbar(7, u), cz, rtol=1e-13, atol=1e-15)
    # uniform: the slope -1/4 comes only from the moving end of the overlap
    np.testing.assert_allclose(oracle.dkbar(0, np.array([-1.5, -0.2, 0.2, 1.5])), [0.25, 0.25, -0.25, -0.25],
                               rtol=1e-14)


# --------------------------------------------------------------------- maps
G_ASYM = Grid(10.0, 11.0, 20.0, 20.6, 21, 13)  # dx = 0.05, dy = 0.05


@pytest.mark.parametrize("kernel", K)
def test_single_point_at_node(kernel):
    """n = 1 at node (i, j) = (7, 4): the density is the outer product
    k((gy - y)/hy) k((gx - x)/hx) / (hx hy), peak k(0)^2/(hx hy) at row 4, col 7."""
    g = G_ASYM
    gx, gy = g.nodes()
    xy = np.array([[gx[7], gy[4]]])
    hx, hy = 0.17, 0.11
    m = oracle.map_world(xy, kernel, hx, hy, g)
    assert m.shape == (g.ny, g.nx)
    k0 = _golden_table1()[oracle.KERNELS[kernel]][0]
    assert m[4, 7] == pytest.approx(k0 / (hx * hy), rel=1e-13)
    assert m[4, 7] == m.max()
    if kernel != 0:  # the uniform kernel is flat on its support
        assert np.unravel_index(np.argmax(m), m.shape) == (4, 7)
    # row 4 is k((gx - x)/hx) k(0) / (hx hy): half-widths differ, so a transpose fails
    assert np.count_nonzero(m[4] > 1e-300) != np.count_nonzero(m[:, 7] > 1e-300) or kernel == GAUSSIAN


def _unit_mass_tol(kernel):
    return {0: 3e-2, 1: 2e-3, 7: 2e-3, 2: 2e-3}.get(kernel, 1e-4)


@pytest.mark.parametrize("kernel", K)
def test_map_unit_integral_and_moments(kernel):
    """The density integrates to 1 over the plane; its mean is the point mean
    and its per-axis variance the sample variance plus mu2 h^2 (Riemann sums on a
    fine grid whose box holds the whole support)."""
    rng = np.random.default_rng(7)
    g = Grid(0.0, 4.0, -1.0, 2.0, 401, 301)  # spacing 0.01
    xy = np.column_stack([rng.uniform(1.2, 2.8, 9), rng.uniform(0.0, 1.0, 9)])
    hx, hy = (0.15, 0.12) if kernel == GAUSSIAN else (0.31, 0.23)
    m = oracle.map_world(xy, kernel, hx, hy, g)
    gx, gy = g.nodes()
    w = g.dx * g.dy
    mass = m.sum() * w
    assert mass == pytest.approx(1.0, abs=_unit_mass_tol(kernel))
    mx = (m.sum(0) * gx).sum() * w / mass
    my = (m.sum(1) * gy).sum() * w / mass
    mtol = 3e-3 if kernel == 0 else 2e-4  # the uniform kernel's jumps: Riemann error O(spacing)
    assert mx == pytest.approx(xy[:, 0].mean(), abs=mtol)
    assert my == pytest.approx(xy[:, 1].mean(), abs=mtol)
    vx = (m.sum(0) * (gx - mx) ** 2).sum() * w / mass
    vy = (m.sum(1) * (gy - my) ** 2).sum() * w / mass
    tol = 2e-2 if kernel == 0 else 3e-3
    assert vx == pytest.approx(xy[:, 0].var() + MU2[kernel] * hx * hx, rel=tol)
    assert vy == pytest.approx(xy[:, 1].var() + MU2[kernel] * hy * hy, rel=tol)


def _pts(seed, n, g):
    rng = np.random.default_rng(seed)
    return np.column_stack([rng.uniform(g.xmin, g.xmax, n), rng.uniform(g.ymin, g.ymax, n)])


@pytest.mark.parametrize("kernel", K)
def test_reflection_transpose_translation_permutation(kernel):
    g = Grid(0.0, 3.0, 0.0, 2.0, 31, 21)  # spacing 0.1
    xy = _pts(3, 17, g)
    hx, hy = 0.37, 0.23
    m = oracle.map_world(xy, kernel, hx, hy, g)
    # reflection x -> xmin + xmax - x flips the columns
    r = xy.copy()
    r[:, 0] = g.xmin + g.xmax - r[:, 0]
    np.testing.assert_allclose(oracle.map_world(r, kernel, hx, hy, g)[:, ::-1], m, rtol=1e-9, atol=1e-12)
    # swapping the axes transposes the map
    gt = Grid(g.ymin, g.ymax, g.xmin, g.xmax, g.ny, g.nx)
    mt = oracle.map_world(xy[:, ::-1], kernel, hy, hx, gt)
    np.testing.assert_allclose(mt.T, m, rtol=1e-12, atol=1e-14)
    # shifting every point by 3 columns and 2 rows shifts the map
    s = xy + np.array([3 * g.dx, 2 * g.dy])
    ms = oracle.map_world(s, kernel, hx, hy, g)
    np.testing.assert_allclose(ms[2:, 3:], m[:-2, :-3], rtol=1e-9, atol=1e-12)
    # permutation invariance
    perm = np.random.default_rng(1).permutation(xy.shape[0])
    np.testing.assert_allclose(oracle.map_world(xy[perm], kernel, hx, hy, g), m, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kernel", K)
def test_raw_sum_linearity_and_scaling(kernel):
    g = Grid(0.0, 3.0, 0.0, 2.0, 31, 21)
    a, b = _pts(4, 11, g), _pts(5, 6, g)
    hx, hy = 0.4, 0.3
    ma = oracle.map_world(a, kernel, hx, hy, g, raw=True)
    mb = oracle.map_world(b, kernel, hx, hy, g, raw=True)
    mab = oracle.map_world(np.vstack([a, b]), kernel, hx, hy, g, raw=True)
    np.testing.assert_allclose(mab, ma + mb, rtol=1e-13, atol=1e-15)
    dens = oracle.map_world(a, kernel, hx, hy, g)
    np.testing.assert_allclose(dens, ma / (a.shape[0] * hx * hy), rtol=1e-14)
    # scaling coordinates, grid and h by c scales the density by 1/c^2
    c = 2.5
    gc = Grid(g.xmin * c, g.xmax * c, g.ymin * c, g.ymax * c, g.nx, g.ny)
    np.testing.assert_allclose(oracle.map_world(a * c, kernel, hx * c, hy * c, gc), dens / c ** 2, rtol=1e-9,
                               atol=1e-12)


def test_brute_force_against_library_densities():
    """Tiny map computed point by point from scipy.stats densities."""
    g = Grid(-1.0, 1.0, -0.5, 0.7, 7, 6)
    xy = _pts(11, 5, g)
    hx, hy = 0.45, 0.35
    gx, gy = g.nodes()
    dists = {
        0: lambda: stats.uniform(loc=-1, scale=2), 1: lambda: stats.triang(c=0.5, loc=-1, scale=2),
        2: lambda: stats.beta(2, 2, loc=-1, scale=2), 3: lambda: stats.beta(3, 3, loc=-1, scale=2),
        4: lambda: stats.beta(4, 4, loc=-1, scale=2), 6: lambda: stats.norm(),
    }
    for kernel, dist in dists.items():
        d = dist()
        ref = np.zeros((g.ny, g.nx))
        for (x, y) in xy:
            ref += np.outer(d.pdf((gy - y) / hy) / hy, d.pdf((gx - x) / hx) / hx)
        ref /= xy.shape[0]
        np.testing.assert_allclose(oracle.map_world(xy, kernel, hx, hy, g), ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("kernel", K)
def test_units_mode_equals_world_mode(kernel):
    """With a grid of spacing 1 from the origin and points on FP32-exact
    coordinates, grid units and world units coincide."""
    rng = np.random.default_rng(kernel)
    XY = (rng.integers(0, 40 * 256, (23, 2)) / 256.0).astype(np.float32)
    g = Grid(0.0, 39.0, 0.0, 29.0, 40, 30)
    H = (np.float32(2.75), np.float32(3.5))
    np.testing.assert_array_equal(oracle.to_units(XY.astype(np.float64), g), XY)
    w = oracle.map_world(XY.astype(np.float64), kernel, float(H[0]), float(H[1]), g, raw=True)
    u = oracle.map_units(XY, kernel, H[0], H[1], (0, 40, 0, 30))
    np.testing.assert_allclose(u, w, rtol=1e-14, atol=1e-15)
    ij = np.array([[0, 0], [39, 29], [17, 3], [5, 22]])
    np.testing.assert_allclose(oracle.map_units_at(XY, kernel, H[0], H[1], ij), w[ij[:, 1], ij[:, 0]], rtol=1e-14,
                               atol=1e-15)


def test_units_support_boundary_inclusive():
    """A point exactly Hx from a node contributes there (|i - X| <= Hx)."""
    XY = np.array([[5.0, 5.0]], dtype=np.float32)
    s = oracle.map_units(XY, 0, np.float32(2.0), np.float32(2.0), (0, 11, 0, 11))
    assert s[5, 3] == 0.25 and s[5, 7] == 0.25 and s[3, 3] == 0.25
    assert s[5, 2] == 0.0 and s[8, 5] == 0.0


@pytest.mark.parametrize("kernel", K)
def test_separable_form_equals_plain_loops(kernel):
    rng = np.random.default_rng(100 + kernel)
    XY = rng.uniform(-3, 35, (300, 2)).astype(np.float32)
    win = (2, 31, 5, 27)
    plain = oracle.map_units(XY, kernel, np.float32(2.3), np.float32(3.1), win)
    sep = oracle.map_units_separable(XY, kernel, np.float32(2.3), np.float32(3.1), win, chunk=77)
    np.testing.assert_allclose(sep, plain, rtol=1e-13, atol=1e-15 * plain.max())


def test_to_units_rounding():
    """FP64 subtract and divide, then one rounding to FP32 (nearest even)."""
    g = Grid(122.0, 123.0, 30.0, 31.0, 1024, 1024)
    xy = np.array([[122.5, 30.25], [122.0, 31.0], [123.0, 30.0]])
    XY = oracle.to_units(xy, g)
    assert XY.dtype == np.float32
    assert XY[0, 0] == np.float32(0.5 * 1023) and XY[0, 1] == np.float32(0.25 * 1023)
    assert XY[1, 0] == 0.0 and XY[1, 1] == np.float32(1023.0) and XY[2, 0] == np.float32(1023.0)


# --------------------------------------------------------------------- adjoint
def _map_units_f64(XY64, kernel, Hx, Hy, nx, ny):
    g = Grid(0.0, nx - 1.0, 0.0, ny - 1.0, nx, ny)
    return oracle.map_world(XY64, kernel, Hx, Hy, g, raw=True)


@pytest.mark.parametrize("kernel", [2, 3, 4, GAUSSIAN, 7])
def test_vjp_against_finite_differences(kernel):
    """dL/dX_p, dL/dY_p and dL/dHx, dL/dHy of L = <gbar, S> against central
    differences of the FP64 map (step 1e-6)."""
    rng = np.random.default_rng(20 + kernel)
    nx, ny = 24, 19
    XY = rng.uniform(3, 16, (6, 2)).astype(np.float32)
    Hx, Hy = np.float32(2.5), np.float32(3.25)
    gbar = rng.standard_normal((ny, nx))
    g, gh = oracle.vjp_units(XY, kernel, Hx, Hy, gbar)
    base = XY.astype(np.float64)
    eps = 1e-6

    def L(pts, hx=float(Hx), hy=float(Hy)):
        return float((gbar * _map_units_f64(pts, kernel, hx, hy, nx, ny)).sum())

    for p in range(XY.shape[0]):
        for c in range(2):
            a, b = base.copy(), base.copy()
            a[p, c] += eps
            b[p, c] -= eps
            fd = (L(a) - L(b)) / (2 * eps)
            assert g[p, c] == pytest.approx(fd, rel=2e-5, abs=2e-7)
    fdx = (L(base, hx=float(Hx) + eps) - L(base, hx=float(Hx) - eps)) / (2 * eps)
    fdy = (L(base, hy=float(Hy) + eps) - L(base, hy=float(Hy) - eps)) / (2 * eps)
    assert gh[:, 0].sum() == pytest.approx(fdx, rel=2e-5, abs=2e-7)
    assert gh[:, 1].sum() == pytest.approx(fdy, rel=2e-5, abs=2e-7)


@pytest.mark.parametrize("kernel", [2, GAUSSIAN])
def test_vjp_separable_equals_plain(kernel):
    rng = np.random.default_rng(40 + kernel)
    nx, ny = 33, 27
    XY = rng.uniform(-2, 34, (90, 2)).astype(np.float32)
    gbar = rng.standard_normal((ny, nx))
    g, gh = oracle.vjp_units(XY, kernel, np.float32(2.2), np.float32(1.7), gbar)
    g2, gh2 = oracle.vjp_units_separable(XY, kernel, np.float32(2.2), np.float32(1.7), gbar, chunk=31)
    scale = np.abs(g).max()
    np.testing.assert_allclose(g2, g, rtol=1e-11, atol=1e-13 * scale)
    np.testing.assert_allclose(gh2, gh, rtol=1e-11, atol=1e-13 * np.abs(gh).max())


# --------------------------------------------------------------------- LSCV
# Riemann-sum error of int f^2 on the 1001 x 801 grid: first order in the node
# spacing where f jumps (uniform), second order where its slope jumps
# (triangular, cosine, Epanechnikov at the support's edge), higher for the
# smoother factors.
LSCV_QUAD_TOL = {0: 1e-2, 1: 1e-3, 2: 2e-4, 3: 1e-5, 4: 1e-7, 5: 1e-6, 6: 1e-8, 7: 1e-3}


@pytest.mark.parametrize("kernel", K)
def test_lscv_against_its_definition(kernel):
    """LSCV(h) = int f^2 - (2/n) sum_p f_{-p}(x_p): the first term by quadrature
    of the pinned density on a fine grid, the second from leave-one-out maps
    evaluated at each point (a grid with a node on the point)."""
    rng = np.random.default_rng(60 + kernel)
    n = 7
    xy = np.column_stack([rng.uniform(0.4, 0.6, n), rng.uniform(0.3, 0.5, n)])
    hx, hy = 0.05, 0.04
    g = Grid(0.0, 1.0, 0.0, 0.8, 1001, 801)
    f = oracle.map_world(xy, kernel, hx, hy, g)
    int_f2 = (f * f).sum() * g.dx * g.dy
    loo = 0.0
    for p in range(n):
        others = np.delete(xy, p, axis=0)
        gp = Grid(xy[p, 0], xy[p, 0] + 1.0, xy[p, 1], xy[p, 1] + 1.0, 2, 2)
        loo += oracle.map_world(others, kernel, hx, hy, gp)[0, 0]
    ref = int_f2 - 2.0 / n * loo
    val, _ = oracle.lscv_world(xy, kernel, hx, hy)
    assert val == pytest.approx(ref, rel=LSCV_QUAD_TOL[kernel])


@pytest.mark.parametrize("kernel", K)
def test_lscv_gradient_against_finite_differences(kernel):
    rng = np.random.default_rng(80 + kernel)
    xy = np.column_stack([rng.uniform(0, 1, 40), rng.uniform(0, 1, 40)])
    hx, hy = 0.09, 0.13
    _, grad = oracle.lscv_world(xy, kernel, hx, hy)
    eps = 1e-6
    fx = (oracle.lscv_world(xy, kernel, hx + eps, hy)[0] - oracle.lscv_world(xy, kernel, hx - eps, hy)[0]) / (2 * eps)
    fy = (oracle.lscv_world(xy, kernel, hx, hy + eps)[0] - oracle.lscv_world(xy, kernel, hx, hy - eps)[0]) / (2 * eps)
    assert grad[0] == pytest.approx(fx, rel=1e-6)
    assert grad[1] == pytest.approx(fy, rel=1e-6)


@pytest.mark.parametrize("kernel", K)
def test_lscv_units_mode_equals_world_mode(kernel):
    """Grid-unit LSCV (the parity reference of the GPU) against world-unit LSCV
    (pinned above) on a grid with power-of-two spacings dx = 1/2, dy = 1/4 and
    points on a 1/256 lattice, so X = x/dx, Hx = hx/dx are exact: the value
    scales by 1/(dx dy) and the gradient by 1/(dx^2 dy), 1/(dx dy^2).  Hx != Hy
    and the point cloud is longer in x than in y, so swapped bandwidths or axes
    in the unit conversion change the result (checked)."""
    rng = np.random.default_rng(170 + kernel)
    dx, dy = 0.5, 0.25
    g = Grid(0.0, dx * 63, 0.0, dy * 47, 64, 48)
    xy = np.column_stack([rng.integers(0, 20 * 256, 30) / 256.0, rng.integers(0, 5 * 256, 30) / 256.0])
    hx, hy = 2.75, 0.625
    XY = oracle.to_units(xy, g)
    np.testing.assert_array_equal(XY.astype(np.float64), xy / np.array([dx, dy]))
    Hx, Hy = oracle.bandwidth_units(hx, hy, g)
    assert (float(Hx), float(Hy)) == (hx / dx, hy / dy)
    vw, gw = oracle.lscv_world(xy, kernel, hx, hy)
    vu, gu = oracle.lscv_units(XY, kernel, Hx, Hy)
    assert vu / (dx * dy) == pytest.approx(vw, rel=1e-13)
    assert gu[0] / (dx * dx * dy) == pytest.approx(gw[0], rel=1e-13)
    assert gu[1] / (dx * dy * dy) == pytest.approx(gw[1], rel=1e-13)
    vs, _ = oracle.lscv_units(XY, kernel, Hy, Hx)
    assert abs(vs / (dx * dy) - vw) > 1e-6 * abs(vw)


def test_lscv_two_points_gaussian_closed_form():
    """n = 2 Gaussian: int f^2 is a sum of N(0, 2h^2) densities and the
    leave-one-out density of each point is the other point's kernel."""
    xy = np.array([[0.0, 0.0], [0.3, -0.2]])
    hx, hy = 0.25, 0.5
    dx, dy = 0.3, -0.2
    phi2 = lambda d, h: math.exp(-d * d / (4 * h * h)) / math.sqrt(4 * math.pi * h * h)
    phi1 = lambda d, h: math.exp(-d * d / (2 * h * h)) / math.sqrt(2 * math.pi * h * h)
    int_f2 = 0.25 * (2 * phi2(0, hx) * phi2(0, hy) + 2 * phi2(dx, hx) * phi2(dy, hy))
    loo = phi1(dx, hx) * phi1(dy, hy)
    val, _ = oracle.lscv_world(xy, GAUSSIAN, hx, hy)
    assert val == pytest.approx(int_f2 - 2 * loo, rel=1e-13)


def test_errors_measure():
    r = np.array([0.0, 1.0, 2.0, 4.0])
    y = np.array([0.0, 1.0, 2.0, 4.4])
    e = oracle.errors(y, r)
    assert e["e_inf"] == pytest.approx(0.1)
    assert e["e_2"] == pytest.approx(0.4 / math.sqrt(21))
    assert e["e_rel"] == pytest.approx(0.1)


# ---------------------------------------------------------------------------
# The paper's binned visualisation: count matrix (Eq. (5)-(6), (12)-(13)) and
# the convolution of Eq. (7).

def _golden_binned():
    pts, rows, total, mode = [], [], None, None
    with open(os.path.join(HERE, "golden", "binned_counts_small.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("points"):
                mode = "p"
            elif line.startswith("counts"):
                mode = "c"
            elif line.startswith("total"):
                total = int(line.split()[1])
            elif mode == "p":
                x, y, lab = line.split()
                pts.append((float(x), float(y), int(lab)))
            else:
                rows.append([int(v) for v in line.split()])
    XY = np.array([(x, y) for x, y, _ in pts], dtype=np.float32)
    labels = np.array([lab for _, _, lab in pts], dtype=np.int32)
    return XY, labels, np.array(rows, dtype=np.uint32), total


def test_binned_counts_hand_worked_example():
    XY, labels, want, total = _golden_binned()
    counts, tot = oracle.bin_counts(XY, labels, 8, 6)
    np.testing.assert_array_equal(counts, want)
    assert tot == total == int(want.sum())
    # without labels: points only (9 of the 10 lie in the grid)
    counts0, tot0 = oracle.bin_counts(XY, None, 8, 6)
    assert tot0 == 9 and int(counts0.sum()) == 9
    assert counts0[3, 6] == 2 and counts0[2, 2] == 1 and counts0[0, 0] == 1


def _round_half_up(q: Fraction) -> int:
    return math.floor(q + Fraction(1, 2))


def test_binned_gap_cells_match_exact_rational_rounding():
    """Random segments inside a 40 x 30 grid: the filled cells equal Eq. (12)-(13)
    evaluated in exact rational arithmetic (1-based coordinates rounded half
    up), form an 8-connected monotone path, and number cmax - 1."""
    rng = np.random.default_rng(1213)
    for trial in range(300):
        a = rng.integers(0, [40, 30])
        b = rng.integers(0, [40, 30])
        XY = np.array([a, b], dtype=np.float32) - np.float32(0.25)  # ceil gives back a, b
        counts, tot = oracle.bin_counts(XY, np.zeros(2, np.int32), 40, 30)
        di, dj = int(b[0] - a[0]), int(b[1] - a[1])
        cmax = max(abs(di), abs(dj))
        want = np.zeros((30, 40), dtype=np.uint32)
        want[a[1], a[0]] += 1
        want[b[1], b[0]] += 1
        path = []
        for c in range(1, cmax):
            i1 = _round_half_up(Fraction(int(a[0]) + 1) + Fraction(c, cmax) * di) - 1
            j1 = _round_half_up(Fraction(int(a[1]) + 1) + Fraction(c, cmax) * dj) - 1
            want[j1, i1] += 1
            path.append((i1, j1))
        np.testing.assert_array_equal(counts, want)
        assert tot == 2 + max(cmax - 1, 0)
        full = [(int(a[0]), int(a[1]))] + path + [(int(b[0]), int(b[1]))]
        if cmax > 0:
            for (x0, y0), (x1, y1) in zip(full, full[1:]):
                assert abs(x1 - x0) <= 1 and abs(y1 - y0) <= 1


def test_binned_projection_edges():
    """ceil projection at the edges: X in (-1, 0] -> cell 0, X = nx-1 -> last cell,
    just above nx-1 or at -1 -> outside; NaN -> outside."""
    XY = np.array([[-0.999, 0.0], [0.0, -0.5], [4.0, 0.0], [np.nextafter(np.float32(4), np.float32(5)), 0.0],
                   [-1.0, 0.0], [np.nan, 1.0], [1.0, 3.0]], dtype=np.float32)
    counts, tot = oracle.bin_counts(XY, None, 5, 4)
    assert tot == 4
    assert counts[0, 0] == 2 and counts[0, 4] == 1 and counts[3, 1] == 1


def test_conv_impulse_response_closed_forms():
    """A single count: the map is the tap table itself (uniform: 1/4 on a 5 x 5
    square for H = 2; Epanechnikov H = 2: 0.75, 0.5625, 0 along an axis), cut
    at the grid edge."""
    counts = np.zeros((9, 11), dtype=np.uint32)
    counts[4, 5] = 1
    u = oracle.conv_counts(counts, 0, 2.0, 2.0, 3, 3)
    want = np.zeros((9, 11))
    want[2:7, 3:8] = 0.25
    np.testing.assert_allclose(u, want, rtol=0, atol=1e-15)
    e = oracle.conv_counts(counts, 2, 2.0, 2.0, 2, 2)
    ax = {0: 0.75, 1: 0.5625, 2: 0.0}
    for j in range(9):
        for i in range(11):
            di, dj = abs(i - 5), abs(j - 4)
            w = ax.get(di, 0.0) * ax.get(dj, 0.0) if di <= 2 and dj <= 2 else 0.0
            assert e[j, i] == pytest.approx(w, abs=1e-15)
    corner = np.zeros((9, 11), dtype=np.uint32)
    corner[0, 0] = 4
    c = oracle.conv_counts(corner, 0, 2.0, 2.0, 2, 2)
    assert c[0:3, 0:3].sum() == pytest.approx(4 * 9 * 0.25) and c.sum() == pytest.approx(4 * 9 * 0.25)


def test_conv_gaussian_tap_mass_poisson_summation():
    """Sum over a wide grid of the Gaussian taps of one count at H = 1 (sigma one
    cell, the paper's Gaussian): by Poisson summation sum_s phi(s) = 1 + 2
    sum_m exp(-2 pi^2 m^2), so the 2-D mass is (1 + 2 e^(-2 pi^2))^2 to 1e-15."""
    counts = np.zeros((41, 41), dtype=np.uint32)
    counts[20, 20] = 1
    g = oracle.conv_counts(counts, 6, 1.0, 1.0, 20, 20)
    one_d = 1.0 + 2.0 * sum(math.exp(-2.0 * math.pi ** 2 * m * m) for m in range(1, 4))
    assert g.sum() == pytest.approx(one_d ** 2, rel=1e-13)


def test_conv_shift_transpose_and_linearity():
    """Shifting the counts shifts the map; transposing counts with Hx, a and Hy,
    b swapped transposes it; the map is linear in the counts."""
    rng = np.random.default_rng(77)
    A = rng.integers(0, 5, (23, 31)).astype(np.uint32)
    A[:, -3:] = 0
    A[-2:, :] = 0
    B = rng.integers(0, 3, (23, 31)).astype(np.uint32)
    for kernel in (1, 5, 6, 7):
        m = oracle.conv_counts(A, kernel, 2.5, 1.5, 3, 2)
        sh = np.zeros_like(A)
        sh[2:, 3:] = A[:-2, :-3]
        ms = oracle.conv_counts(sh, kernel, 2.5, 1.5, 3, 2)
        np.testing.assert_allclose(ms[2 + 4:, 3 + 4:], m[4:-2, 4:-3], rtol=1e-13, atol=1e-13)
        mt = oracle.conv_counts(np.ascontiguousarray(A.T), kernel, 1.5, 2.5, 2, 3)
        np.testing.assert_allclose(mt, m.T, rtol=1e-13, atol=1e-13)
        mab = oracle.conv_counts(A + B, kernel, 2.5, 1.5, 3, 2)
        np.testing.assert_allclose(mab, m + oracle.conv_counts(B, kernel, 2.5, 1.5, 3, 2), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# The Gaussian truncated at |u| <= 8 (a banded variant of the Gaussian map).

def test_truncated_gaussian_factor_and_mass():
    """k_T(u) = phi(u) for |u| <= 8 (inclusive), 0 beyond; its mass is
    erf(8 / sqrt 2) = 1 - 1.2e-15."""
    u = np.array([0.0, 1.5, -7.999, 8.0, -8.0, 8.0001, 20.0])
    want = np.where(np.abs(u) <= 8.0, stats.norm.pdf(u), 0.0)
    np.testing.assert_array_equal(oracle.k(oracle.GAUSS_TRUNC, u) == 0.0, want == 0.0)
    np.testing.assert_allclose(oracle.k(oracle.GAUSS_TRUNC, u), want, rtol=1e-14, atol=0)
    m, _ = integrate.quad(lambda x: oracle.k(oracle.GAUSS_TRUNC, [x])[0], -8.0, 8.0, points=[0.0], limit=200)
    assert m == pytest.approx(math.erf(8.0 / math.sqrt(2.0)), abs=1e-13)


def test_truncated_gaussian_map_bound_and_boundary():
    """The truncated map never exceeds the full one and differs by at most the
    dropped tails: each pair loses less than phi(0)^2 e^-32.  On the grid, the
    support is |i - X| <= 8 H on the exact difference (inclusive)."""
    rng = np.random.default_rng(8)
    XY = np.column_stack([rng.uniform(-20, 60, 3000), rng.uniform(-20, 50, 3000)]).astype(np.float32)
    for H in (0.7, 2.0, 5.0):
        full = oracle.map_units(XY, oracle.GAUSSIAN, H, 0.8 * H, (0, 40, 0, 30))
        trunc = oracle.map_units(XY, oracle.GAUSS_TRUNC, H, 0.8 * H, (0, 40, 0, 30))
        assert np.all(trunc <= full + 1e-300)
        bound = XY.shape[0] * stats.norm.pdf(0.0) ** 2 * math.exp(-32.0)
        assert np.max(full - trunc) <= bound
        assert np.max(full - trunc) > 0.0 or H == 5.0
    one = np.array([[0.0, 0.0]], dtype=np.float32)
    m = oracle.map_units(one, oracle.GAUSS_TRUNC, 0.5, 0.5, (0, 6, 0, 1))[0]
    assert m[4] == pytest.approx(stats.norm.pdf(8.0) * stats.norm.pdf(0.0), rel=1e-13)  # d = 4 = 8 H: kept
    assert m[5] == 0.0                                                                   # d = 5 > 8 H


# ---------------------------------------------------------------------------
# Douglas-Peucker (Sec. III-B; Eq. (9)).

def _dp1(x, y, eps):
    xy = np.column_stack([np.asarray(x, float), np.asarray(y, float)])
    return list(np.flatnonzero(oracle.dp_keep(xy, [len(x)], eps)))


def test_dp_oracle_textbook_cases():
    assert _dp1(np.arange(10.0), 2 * np.arange(10.0), 0.0) == [0, 9]       # collinear
    y = np.zeros(9)
    y[4] = 5.0
    assert _dp1(np.arange(9.0), y, 4.999) == [0, 4, 8]                        # spike of height 5
    assert _dp1(np.arange(9.0), y, 5.0) == [0, 8]                             # strictly larger only
    assert _dp1([0.0, 1.0, 2.0, 3.0, 4.0], [0.0, 1.0, 0.0, 1.0, 0.0], 0.7) == [0, 1, 4]  # lowest index on ties
    assert _dp1([0.0, 10.0, 5.0], [0.0, 0.0, 0.0], 0.0) == [0, 2]            # distance to the line
    assert _dp1([0.0, 3.0, 0.0], [0.0, 4.0, 0.0], 4.9) == [0, 1, 2]          # zero chord: point distance 5
    assert _dp1([0.0, 3.0, 0.0], [0.0, 4.0, 0.0], 5.0) == [0, 2]


def test_dp_oracle_track_boundaries():
    """Tracks of 1, 2 and 3 points and a zig-zag: each track on its own."""
    xy = np.array([[0, 0], [5, 5], [6, 6], [0, 0], [1, 9], [2, 0],
                   [0, 0], [1, 1], [2, 0], [3, 1], [4, 0]], dtype=float)
    keep = oracle.dp_keep(xy, [1, 2, 3, 5], 0.5)
    assert list(keep) == [1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1]
    keep = oracle.dp_keep(xy, [1, 2, 3, 5], 100.0)
    assert list(keep) == [1, 1, 1, 1, 0, 1, 1, 0, 0, 0, 1]


def test_dp_oracle_matches_independent_python_dp():
    """The recursive Python compressor of the input generator (distance by
    hypot and division) gives the same mask on lane tracks at several eps: the
    two decision forms differ only at exact ties."""
    t = synth.generate(17, 40, 300, synth.BOX_C2, n_lanes=3)
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    for eps in (0.0, 10.0, 50.0, 200.0):
        keep = oracle.dp_keep(xy, t.lengths, eps)
        ref = np.concatenate([ais._dp_keep(mx[k * 300:(k + 1) * 300], my[k * 300:(k + 1) * 300], eps)
                              for k in range(40)])
        np.testing.assert_array_equal(keep.astype(bool), ref)


def test_dp_oracle_dropped_points_within_eps():
    """Brute force on random walks: every dropped point lies within eps of the
    line through the kept points that enclose it, and the end points are kept."""
    rng = np.random.default_rng(99)
    for trial in range(20):
        n = 60
        xy = np.cumsum(rng.normal(0, 1, (n, 2)), axis=0)
        eps = float(rng.uniform(0.2, 3.0))
        keep = oracle.dp_keep(xy, [n], eps).astype(bool)
        assert keep[0] and keep[-1]
        idx = np.flatnonzero(keep)
        for s, e in zip(idx, idx[1:]):
            c = xy[e] - xy[s]
            for i in range(s + 1, e):
                p = xy[i] - xy[s]
                d = abs(p[0] * c[1] - p[1] * c[0]) / max(np.hypot(*c), 1e-300) if np.hypot(*c) > 0 else np.hypot(*p)
                assert d <= eps * (1 + 1e-12)


# ------------------------------------------------------- compression quality (Sec. V-B)
def _golden_metrics():
    vals = {}
    with open(os.path.join(HERE, "golden", "compression_metrics_small.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, val = line.split()
            if key.startswith(("points", "lengths")):
                rows = [[float(v) for v in r.split(",")] for r in val.split(";")]
                vals[key] = np.array(rows) if key.startswith("points") else [int(v) for v in rows[0]]
            else:
                vals[key] = eval(val, {"__builtins__": {}, "sqrt": math.sqrt})
    return vals


def test_metrics_hand_worked_example():
    g = _golden_metrics()
    r = oracle.track_metrics(g["points_o"], g["lengths_o"], g["points_c"], g["lengths_c"])
    for m in (1, 2):
        assert r["dtw"][m - 1] == pytest.approx(g[f"dtw_{m}"], rel=1e-15)
        assert r["len_o"][m - 1] == pytest.approx(g[f"len_o_{m}"], rel=1e-15)
        assert r["len_c"][m - 1] == pytest.approx(g[f"len_c_{m}"], rel=1e-15, abs=0)
    for key in ("cr_percent", "rll", "dtw_mean", "dtw_std"):
        assert r[key] == pytest.approx(g[key], rel=1e-14), key
    assert (r["n_original"], r["n_compressed"]) == (6, 3)


def _dtw_brute(a, b):
    """Minimum over every warping path from (0, 0) to (na-1, nb-1) with steps
    (1, 0), (0, 1), (1, 1) of the summed squared distances, square-rooted."""
    na, nb = len(a), len(b)
    best = math.inf

    def walk(i, j, cost):
        nonlocal best
        cost += float(np.sum((a[i] - b[j]) ** 2))
        if (i, j) == (na - 1, nb - 1):
            best = min(best, cost)
            return
        if i + 1 < na:
            walk(i + 1, j, cost)
        if j + 1 < nb:
            walk(i, j + 1, cost)
        if i + 1 < na and j + 1 < nb:
            walk(i + 1, j + 1, cost)

    walk(0, 0, 0.0)
    return math.sqrt(best)


def test_dtw_matches_brute_force_over_warping_paths():
    rng = np.random.default_rng(5)
    for na in range(1, 6):
        for nb in range(1, 6):
            a = rng.normal(0, 3, (na, 2))
            b = rng.normal(0, 3, (nb, 2))
            assert oracle.dtw(a, b) == pytest.approx(_dtw_brute(a, b), rel=1e-13)


def test_dtw_closed_forms_and_symmetries():
    rng = np.random.default_rng(6)
    a = rng.normal(0, 10, (37, 2))
    p = rng.normal(0, 10, (1, 2))
    # one point on either side: every cell of the single row or column is on the path
    want = math.sqrt(float(np.sum((a - p) ** 2)))
    assert oracle.dtw(a, p) == pytest.approx(want, rel=1e-13)
    assert oracle.dtw(p, a) == pytest.approx(want, rel=1e-13)
    b = rng.normal(0, 10, (23, 2))
    assert oracle.dtw(a, a) == 0.0
    assert oracle.dtw(a, b) == oracle.dtw(b, a)  # the recurrence is symmetric under transposition
    assert oracle.dtw(a + 1000.0, b + 1000.0) == pytest.approx(oracle.dtw(a, b), rel=1e-9)  # translation
    assert oracle.dtw(2.0 * a, 2.0 * b) == pytest.approx(2.0 * oracle.dtw(a, b), rel=1e-13)  # degree-1 scaling
    assert oracle.dtw(a[:0], b[:0]) == 0.0
    assert oracle.dtw(a, b[:0]) == math.inf


def test_track_length_forms():
    rng = np.random.default_rng(7)
    xy = rng.normal(0, 50, (101, 2))
    assert oracle.track_length(xy) == pytest.approx(float(np.sum(np.hypot(*np.diff(xy, axis=0).T))), rel=1e-13)
    assert oracle.track_length(xy[::-1]) == pytest.approx(oracle.track_length(xy), rel=1e-13)
    line = np.column_stack([np.arange(11.0) * 3.0, np.arange(11.0) * 4.0])
    assert oracle.track_length(line) == 50.0
    assert oracle.track_length(xy[:1]) == 0.0 and oracle.track_length(xy[:0]) == 0.0


def _dp_pair(t, eps):
    mx, my = synth.mercator(t.xy[:, 0], t.xy[:, 1], t.box.center_lat)
    xy = np.column_stack([mx, my])
    keep = oracle.dp_keep(xy, t.lengths, eps).astype(bool)
    starts = np.concatenate([[0], np.cumsum(t.lengths)])
    lc = np.array([int(keep[a:b].sum()) for a, b in zip(starts[:-1], starts[1:])])
    return xy, xy[keep], lc


def test_metrics_threshold_zero_row_and_nesting():
    """Eps 0 keeps every point off its chord, which on noisy tracks is all of
    them: CR, RLL and DTW are 0 (the first row of Table IV).  Larger eps keeps a
    subset of the points of smaller eps, so CR grows; a kept subsequence with
    the end points is never longer (triangle inequality), so 0 <= RLL < 1."""
    t = synth.generate(23, 30, 200, synth.BOX_C2, n_lanes=2)
    xy, xc, lc = _dp_pair(t, 0.0)
    r = oracle.track_metrics(xy, t.lengths, xc, lc)
    assert r["cr_percent"] == 0.0 and r["rll"] == 0.0 and r["dtw_mean"] == 0.0 and r["dtw_std"] == 0.0
    prev = None
    for eps in (1.0, 10.0, 50.0):
        xy, xc, lc = _dp_pair(t, eps)
        r = oracle.track_metrics(xy, t.lengths, xc, lc)
        assert 0.0 <= r["rll"] < 1.0
        assert np.all(r["len_c"] <= r["len_o"] * (1 + 1e-12))
        assert np.all(r["dtw"] >= 0.0)
        if prev is not None:
            assert r["cr_percent"] >= prev["cr_percent"]
        prev = r


def test_metrics_population_std_and_empty_tracks():
    # DTW values 1 and 3 from one-column tracks: mu 2, population delta 1
    xo = np.array([[0.0, 0.0], [0.0, 1.0], [5.0, 5.0], [5.0, 8.0]])
    xc = np.array([[0.0, 0.0], [5.0, 5.0]])
    r = oracle.track_metrics(xo, [2, 2], xc, [1, 1])
    assert list(r["dtw"]) == [1.0, 3.0]
    assert r["dtw_mean"] == 2.0 and r["dtw_std"] == 1.0
    # an empty pair is at distance 0 and counts in M
    r = oracle.track_metrics(xo, [2, 0, 2], xc, [1, 0, 1])
    assert list(r["dtw"]) == [1.0, 0.0, 3.0]
    assert r["dtw_mean"] == pytest.approx(4.0 / 3.0, rel=1e-15)
