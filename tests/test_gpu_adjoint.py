"""Parity of the adjoints (kde_backward, kde_lscv) with the FP64 oracle.

Gates: point gradients relative L2 <= 1e-4, bandwidth gradients and LSCV
relative error <= 1e-4.  The oracle's gradients are themselves pinned against
central finite differences in tests/test_oracle_pins.py."""
import numpy as np
import pytest

import oracle
import paper_2004_13653_amd as kde
import synth
from tests import kdetest as kt

pytestmark = pytest.mark.gpu

GRAD_GATE = 1e-4


def _rel_l2(y, r):
    """||y - r|| / ||r||; for an all-zero reference, ||y|| itself."""
    y = np.asarray(y, np.float64)
    nr = np.linalg.norm(r)
    return float(np.linalg.norm(y - r) / nr) if nr > 0 else float(np.linalg.norm(y))


def _rel(y, r):
    y, r = np.asarray(y, np.float64), np.asarray(r, np.float64)
    return np.where(r != 0, np.abs(y - r) / np.where(r != 0, np.abs(r), 1.0), np.abs(y))


def _expected_vjp(XY, kernel, hx, hy, og, gbar, raw):
    """World-unit dL/dx_p, dL/dy_p and dL/dhx, dL/dhy of L = <gbar, out> from the
    oracle's raw-sum VJP (k includes its constant)."""
    Hx, Hy = oracle.bandwidth_units(hx, hy, og)
    g, gh = oracle.vjp_units_separable(XY, kernel, Hx, Hy, gbar)
    n = XY.shape[0]
    sigma = 1.0 if raw else oracle.density_scale(n, hx, hy)
    gp = np.column_stack([g[:, 0] * sigma / og.dx, g[:, 1] * sigma / og.dy])
    dhx = sigma * gh[:, 0].sum() / og.dx
    dhy = sigma * gh[:, 1].sum() / og.dy
    if not raw:
        S = oracle.map_units_separable(XY, kernel, Hx, Hy, (0, og.nx, 0, og.ny))
        q = float((gbar * S).sum())
        dhx -= sigma * q / hx
        dhy -= sigma * q / hy
    return gp, np.array([dhx, dhy])


def _gpu_vjp(XY, kernel, hx, hy, g, gbar, raw=False, grid_units=False, fp32=False):
    import torch
    pts = kt.to_device(XY)
    go = torch.from_numpy(np.ascontiguousarray(gbar, dtype=np.float32)).to(kt.device())
    gp, gh = kde.backward(pts, kernel, hx, hy, g, go, raw=raw, grid_units=grid_units, fp32=fp32)
    torch.cuda.synchronize()
    return gp.cpu().numpy().astype(np.float64), np.array(gh)


@pytest.mark.parametrize("kernel", list(range(8)))
@pytest.mark.parametrize("raw", [False, True])
@pytest.mark.parametrize("shape", [(150, 97), (180, 530)])
def test_vjp_all_kernels(kernel, raw, shape):
    """2,000 lane points, random cotangent, on a 150 x 97 grid (ragged strips) and
    on a 180 x 530 grid, whose row sweep crosses the 256-row chunks twice (rows
    0-255, 256-511, 512-529)."""
    nx, ny = shape
    t = kt.lanes(20, 100)
    g, og = kt.grids(synth.BOX_C2, nx, ny)
    XY = kde.to_grid_units(t.xy, g)
    rng = np.random.default_rng(kernel)
    gbar = rng.standard_normal((ny, nx))
    h = 0.02
    gp, gh = _gpu_vjp(XY, kernel, h, 0.7 * h, g, gbar, raw=raw)
    rp, rh = _expected_vjp(XY, kernel, h, 0.7 * h, og, gbar, raw)
    e_p = _rel_l2(gp, rp)
    e_h = _rel(gh, rh)
    kt.log(f"kernel={kernel} raw={raw} {nx}x{ny}: points rel-L2 {e_p:.2e}, h rel {e_h}")
    assert e_p <= GRAD_GATE
    assert np.all(e_h <= GRAD_GATE)


@pytest.mark.parametrize("kernel", [0, 2, 5, 7])
@pytest.mark.parametrize("raw", [False, True])
def test_vjp_wide_compact_supports(kernel, raw):
    """Compact supports wider than the per-point windows take (more than 1,024
    nodes: Hx = 30, Hy = 13 px here) take the workgroup sweep of row strips;
    2,000 lane points, random cotangent, 150 x 97 grid, against the oracle."""
    nx, ny = 150, 97
    t = kt.lanes(20, 100)
    g, og = kt.grids(synth.BOX_C2, nx, ny)
    XY = kde.to_grid_units(t.xy, g)
    Hx, Hy = kde.bandwidth_units(0.2, 0.14, g)
    assert (np.floor(2 * Hx) + 3) * (np.floor(2 * Hy) + 3) > 1024
    rng = np.random.default_rng(100 + kernel)
    gbar = rng.standard_normal((ny, nx))
    gp, gh = _gpu_vjp(XY, kernel, 0.2, 0.14, g, gbar, raw=raw)
    rp, rh = _expected_vjp(XY, kernel, 0.2, 0.14, og, gbar, raw)
    e_p = _rel_l2(gp, rp)
    e_h = _rel(gh, rh)
    kt.log(f"kernel={kernel} raw={raw} wide: points rel-L2 {e_p:.2e}, h rel {e_h}")
    assert e_p <= GRAD_GATE
    assert np.all(e_h <= GRAD_GATE)


@pytest.mark.parametrize("shape,n", [((96, 80), 1), ((96, 80), 255), ((300, 257), 257), ((513, 33), 2000),
                                     ((40, 700), 700)])
@pytest.mark.parametrize("raw", [False, True])
def test_gaussian_vjp_matrix_cores(shape, n, raw):
    """The Gaussian VJP on matrix cores (the default) and per pair in FP32
    (KDE_VJP_FP32), both against the oracle, on ragged shapes: point counts
    around the 256-point blocks, grids with 1-3 tiles of 256 nodes along either
    axis and contraction lengths that are not multiples of the 32-node chunks,
    some points outside the grid.  Matrix-core results are bitwise reproducible."""
    nx, ny = shape
    rng = np.random.default_rng(n + nx)
    XY = np.column_stack([rng.uniform(-3, nx + 3, n), rng.uniform(-3, ny + 3, n)]).astype(np.float32)
    g, og = kt.grids(synth.BOX_C2, nx, ny)
    gbar = rng.standard_normal((ny, nx))
    hx, hy = 3.1 * og.dx, 1.7 * og.dy
    rp, rh = _expected_vjp(XY.astype(np.float64), 6, hx, hy, og, gbar, raw)
    gp, gh = _gpu_vjp(XY, 6, hx, hy, g, gbar, raw=raw)
    gp2, gh2 = _gpu_vjp(XY, 6, hx, hy, g, gbar, raw=raw)
    fp, fh = _gpu_vjp(XY, 6, hx, hy, g, gbar, raw=raw, fp32=True)
    e_m, e_f = _rel_l2(gp, rp), _rel_l2(fp, rp)
    kt.log(f"{nx}x{ny} n={n} raw={raw}: matrix cores rel-L2 {e_m:.2e}, h {_rel(gh, rh)}; "
           f"FP32 rel-L2 {e_f:.2e}, h {_rel(fh, rh)}")
    assert np.array_equal(gp, gp2) and np.array_equal(gh, gh2)
    assert e_m <= GRAD_GATE and e_f <= GRAD_GATE
    assert np.all(_rel(gh, rh) <= GRAD_GATE) and np.all(_rel(fh, rh) <= GRAD_GATE)


def _sample_points(XY, ny, nx, seed):
    """Indices of >= 256 points for full-size gradient checks: points in the rows
    around the 256-row chunk edge, past it, below it, near the grid's edges, and
    uniform ones."""
    rng = np.random.default_rng(seed)
    X, Y = XY[:, 0], XY[:, 1]
    pick = []
    for mask, m in (((Y >= 240) & (Y <= 272), 64), ((Y > 300) & (Y < ny), 64), ((Y >= 0) & (Y < 200), 32),
                    ((X < 6) | (X > nx - 7) | (Y < 6) | (Y > ny - 7), 32)):
        idx = np.flatnonzero(mask)
        if idx.size:
            pick.append(rng.choice(idx, size=min(m, idx.size), replace=False))
    pick.append(rng.choice(XY.shape[0], size=96, replace=False))
    return np.unique(np.concatenate(pick))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kernel", [6, 2])
def test_vjp_full_size_against_oracle(kernel):
    """250,000 points on 512 x 512 at h = 0.004 deg, L2 loss against the map of
    the same tracks Douglas-Peucker-compressed at 50 m: gbar = 2 (f - T), f and T
    from the oracle.  dL/d(x_p, y_p) of >= 256 sampled points (rows around and
    past the 256-row chunk edge, the grid's edges, uniform) against the oracle's
    plain loops, and both bandwidth gradients (sums over every point) against
    its factored form; gate relative L2 / relative error <= 1e-4."""
    t = kt.lanes(500, 500)
    tc = kt.lanes_dp(500, 500, 50.0)
    g, og = kt.grids(synth.BOX_C2, 512, 512)
    XY = kde.to_grid_units(t.xy, g)
    XYc = kde.to_grid_units(tc.xy, g)
    h = 0.004
    Hx, Hy = oracle.bandwidth_units(h, h, og)
    full = (0, 512, 0, 512)
    S = oracle.map_units_separable(XY, kernel, Hx, Hy, full)
    sigma = oracle.density_scale(XY.shape[0], h, h)
    T = oracle.map_units_separable(XYc, kernel, Hx, Hy, full) * oracle.density_scale(XYc.shape[0], h, h)
    gbar = (2.0 * (S * sigma - T)).astype(np.float32).astype(np.float64)
    kt.log(f"kernel={kernel}: n={XY.shape[0]}, compressed {XYc.shape[0]}, |gbar|max={np.abs(gbar).max():.3e}")
    gp, gh = _gpu_vjp(XY, kernel, h, h, g, gbar)
    sel = _sample_points(XY, 512, 512, seed=kernel)
    rp, _ = oracle.vjp_units(XY, kernel, Hx, Hy, gbar, sel=sel)
    rp = np.column_stack([rp[:, 0] * sigma / og.dx, rp[:, 1] * sigma / og.dy])
    e_p = _rel_l2(gp[sel], rp)
    kt.log(f"  {sel.size} sampled points ({int((XY[sel, 1] >= 256).sum())} in rows >= 256): rel-L2 {e_p:.2e}")
    assert sel.size >= 256
    assert e_p <= GRAD_GATE
    _, ghs = oracle.vjp_units_separable(XY, kernel, Hx, Hy, gbar)
    q = float((gbar * S).sum())
    rh = np.array([sigma * ghs[:, 0].sum() / og.dx - sigma * q / h, sigma * ghs[:, 1].sum() / og.dy - sigma * q / h])
    e_h = _rel(gh, rh)
    kt.log(f"  bandwidth gradient {gh} ref {rh}: rel {e_h}")
    assert np.all(e_h <= GRAD_GATE)


def test_vjp_grid_units_and_l2_loss():
    """L2 loss against a target map: gbar = 2 (f - T), T the map of the
    Douglas-Peucker-compressed points, gradients for the raw points."""
    import torch
    t = kt.lanes(40, 200)
    tc = synth.dp_compress(t, 50.0)
    g, og = kt.grids(synth.BOX_C2, 256, 256)
    XY = kde.to_grid_units(t.xy, g)
    XYc = kde.to_grid_units(tc.xy, g)
    h = 0.006
    f = kt.gpu_map(XY, 6, h, h, g)
    T = kt.gpu_map(XYc, 6, h, h, g)
    gbar = 2.0 * (f - T)
    gp, gh = _gpu_vjp(XY, 6, h, h, g, gbar, grid_units=True)
    rp, rh = _expected_vjp(XY, 6, h, h, og, gbar, False)
    rp_units = rp * np.array([og.dx, og.dy])
    assert _rel_l2(gp, rp_units) <= GRAD_GATE
    assert np.all(np.abs(gh - rh) / np.abs(rh) <= GRAD_GATE)


def test_autograd_function_matches_backward():
    import torch
    t = kt.lanes(20, 100)
    g, og = kt.grids(synth.BOX_C2, 96, 80)
    XY = kde.to_grid_units(t.xy, g)
    pts = kt.to_device(XY).requires_grad_(True)
    hx = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    hy = torch.tensor(0.015, dtype=torch.float64, requires_grad=True)
    out = kde.kde_map(pts, hx, hy, "epanechnikov", g)
    w = torch.linspace(-1, 1, out.numel(), device=out.device).reshape(out.shape)
    (out * w).sum().backward()
    rp, rh = _expected_vjp(XY, 2, 0.02, 0.015, og, w.cpu().numpy().astype(np.float64), False)
    assert _rel_l2(pts.grad.cpu().numpy(), rp * np.array([og.dx, og.dy])) <= GRAD_GATE
    assert abs(hx.grad.item() - rh[0]) <= GRAD_GATE * abs(rh[0])
    assert abs(hy.grad.item() - rh[1]) <= GRAD_GATE * abs(rh[1])


def _lscv_against_oracle(XY, kernel, hx, hy, g, og):
    """kde_lscv against the oracle in parity mode (FP32 grid-unit inputs, FP64
    arithmetic), converted to world units: value relative error and both
    gradient components' relative errors <= 1e-4."""
    import torch
    Hx, Hy = oracle.bandwidth_units(hx, hy, og)
    vu, gu = oracle.lscv_units(XY, kernel, Hx, Hy)
    ref_v = vu * float(Hx) * float(Hy) / (hx * hy)
    ref_g = np.array([gu[0] * float(Hx) ** 2 * float(Hy) / (hx * hx * hy),
                      gu[1] * float(Hx) * float(Hy) ** 2 / (hx * hy * hy)])
    v, gh = kde.lscv(kt.to_device(XY), kernel, hx, hy, g)
    torch.cuda.synchronize()
    kt.log(f"lscv kernel={kernel} n={XY.shape[0]} h=({hx}, {hy}): value {v:.6e} ref {ref_v:.6e}; "
           f"grad {gh} ref {ref_g}")
    assert abs(v - ref_v) <= GRAD_GATE * abs(ref_v)
    assert np.all(np.abs(np.array(gh) - ref_g) <= GRAD_GATE * np.abs(ref_g))


@pytest.mark.parametrize("kernel", [6, 2])
@pytest.mark.parametrize("hdeg", [0.001, 0.004, 0.01])
def test_lscv_value_and_gradient(kernel, hdeg):
    """20,000 lane points, LSCV over all ordered pairs against the oracle."""
    t = kt.lanes(100, 200)
    g, og = kt.grids(synth.BOX_C2, 512, 512)
    _lscv_against_oracle(kde.to_grid_units(t.xy, g), kernel, hdeg, 1.3 * hdeg, g, og)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kernel", [6, 2, 5, 0])
def test_lscv_50k_points(kernel):
    """50,000 lane points (100 tracks x 500) at h = (0.004, 0.0052) deg on the
    512 x 512 grid's units: 2.5*10^9 ordered pairs against the oracle (the
    Gaussian over all pairs, the compact kernels over the support-culled tiles
    of the spatially sorted points)."""
    t = kt.lanes(100, 500)
    g, og = kt.grids(synth.BOX_C2, 512, 512)
    _lscv_against_oracle(kde.to_grid_units(t.xy, g), kernel, 0.004, 1.3 * 0.004, g, og)


@pytest.mark.parametrize("kernel", [0, 1, 3, 4, 5, 7])
@pytest.mark.parametrize("hdeg", [0.002, 0.01])
def test_lscv_other_kernels(kernel, hdeg):
    """The six other Table I kernels (autoconvolutions as piecewise polynomials
    or, for the cosine, a closed form) on 4,000 lane points, against the oracle's
    quadrature of the defining integral."""
    import torch
    t = kt.lanes(40, 100)
    g, og = kt.grids(synth.BOX_C2, 512, 512)
    XY = kde.to_grid_units(t.xy, g)
    Hx, Hy = oracle.bandwidth_units(hdeg, 1.3 * hdeg, og)
    vu, gu = oracle.lscv_units(XY, kernel, Hx, Hy)
    hx, hy = hdeg, 1.3 * hdeg
    ref_v = vu * float(Hx) * float(Hy) / (hx * hy)
    ref_g = np.array([gu[0] * float(Hx) ** 2 * float(Hy) / (hx * hx * hy),
                      gu[1] * float(Hx) * float(Hy) ** 2 / (hx * hy * hy)])
    v, gh = kde.lscv(kt.to_device(XY), kernel, hx, hy, g)
    torch.cuda.synchronize()
    kt.log(f"lscv kernel={kernel} h={hdeg}: value {v:.6e} ref {ref_v:.6e}; grad {gh} ref {ref_g}")
    assert abs(v - ref_v) <= GRAD_GATE * abs(ref_v)
    assert np.all(np.abs(np.array(gh) - ref_g) <= GRAD_GATE * np.abs(ref_g))


@pytest.mark.parametrize("n", [3, 255, 256, 257, 513, 1000, 2049])
def test_lscv_ragged_point_counts(n):
    """Point counts around the 256-point tiles (one to nine p-blocks, odd and
    even, so the paired rows of tiles, the lone middle row and the diagonal
    tiles all occur), Gaussian and tricube, against the oracle."""
    import torch
    rng = np.random.default_rng(n)
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 128, 128)
    og = oracle.Grid(0.0, 1.0, 0.0, 1.0, 128, 128)
    XY = rng.uniform(20.0, 60.0, (n, 2)).astype(np.float32)
    for kernel, h in ((6, 0.03), (5, 0.05)):
        Hx, Hy = oracle.bandwidth_units(h, 1.2 * h, og)
        vu, gu = oracle.lscv_units(XY, kernel, Hx, Hy)
        ref_v = vu * float(Hx) * float(Hy) / (h * 1.2 * h)
        v, gh = kde.lscv(kt.to_device(XY), kernel, h, 1.2 * h, g)
        torch.cuda.synchronize()
        assert abs(v - ref_v) <= GRAD_GATE * abs(ref_v), (kernel, v, ref_v)
        ref_g = np.array([gu[0] * float(Hx) ** 2 * float(Hy) / (h * h * 1.2 * h),
                          gu[1] * float(Hx) * float(Hy) ** 2 / (h * 1.2 * h * 1.2 * h)])
        assert np.all(np.abs(np.array(gh) - ref_g) <= GRAD_GATE * np.abs(ref_g)), (kernel, gh, ref_g)


@pytest.mark.parametrize("kernel", [5, 2, 7])
def test_lscv_culled_points_off_grid_and_coincident(kernel):
    """Support culling with points far outside the grid (their sort cells are
    clamped to the border cells), with all points coincident (every tile in
    support) and with two distant clusters (most tiles skipped), against the
    oracle."""
    rng = np.random.default_rng(40 + kernel)
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 128, 128)
    og = oracle.Grid(0.0, 1.0, 0.0, 1.0, 128, 128)
    spread = rng.uniform(-300.0, 450.0, (3000, 2)).astype(np.float32)
    same = np.full((700, 2), 17.25, dtype=np.float32)
    two = np.concatenate([rng.normal(10.0, 1.0, (900, 2)), rng.normal(100.0, 1.0, (1100, 2))]).astype(np.float32)
    for XY, h in ((spread, 0.2), (same, 0.02), (two, 0.03)):
        _lscv_against_oracle(XY, kernel, h, 1.3 * h, g, og)


def test_lscv_autograd_and_edge_cases():
    import torch
    g = kde.Grid(0.0, 1.0, 0.0, 1.0, 64, 64)
    og = oracle.Grid(0.0, 1.0, 0.0, 1.0, 64, 64)
    XY = np.array([[10.0, 12.0], [13.5, 11.25]], dtype=np.float32)  # n = 2
    hx = torch.tensor(0.05, dtype=torch.float64, requires_grad=True)
    hy = torch.tensor(0.04, dtype=torch.float64, requires_grad=True)
    val = kde.kde_lscv(kt.to_device(XY), hx, hy, "gaussian", g)
    val.backward()
    Hx, Hy = oracle.bandwidth_units(0.05, 0.04, og)
    vu, gu = oracle.lscv_units(XY, 6, Hx, Hy)
    assert val.item() == pytest.approx(vu * float(Hx) * float(Hy) / (0.05 * 0.04), rel=1e-5)
    assert hx.grad.item() == pytest.approx(gu[0] * float(Hx) ** 2 * float(Hy) / (0.05 ** 2 * 0.04), rel=1e-4)
    with pytest.raises(kde.KDEError):
        kde.lscv(kt.to_device(XY[:1]), "gaussian", 0.05, 0.04, g)
    with pytest.raises(kde.KDEError):
        kde.lscv(kt.to_device(XY), 9, 0.05, 0.04, g)  # no such kernel


def test_full_size_adjoint_runs_and_is_deterministic():
    """250,000 points on 512 x 512 (Gaussian and Epanechnikov): VJP and LSCV are
    bitwise reproducible and finite; for the Gaussian, L = sum(out) does not
    change when one interior point moves (a lattice sum of a smooth Gaussian is
    translation invariant to far below FP32), so its point gradients vanish next
    to those of a random cotangent."""
    import torch
    t = kt.lanes(500, 500)
    g, og = kt.grids(synth.BOX_C2, 512, 512)
    XY = kde.to_grid_units(t.xy, g)
    pts = kt.to_device(XY)
    ones = torch.ones((512, 512), device=kt.device())
    for kernel, h in ((6, 0.004), (2, 0.004)):
        a, ha = kde.backward(pts, kernel, h, h, g, ones, raw=True, grid_units=True)
        b, hb = kde.backward(pts, kernel, h, h, g, ones, raw=True, grid_units=True)
        torch.cuda.synchronize()
        assert torch.equal(a, b) and ha == hb
        assert torch.isfinite(a).all()
        va, ga = kde.lscv(pts, kernel, h, h, g)
        vb, gb = kde.lscv(pts, kernel, h, h, g)
        assert va == vb and ga == gb and np.isfinite(va)
        if kernel == 6:
            inside = (XY[:, 0] > 20) & (XY[:, 0] < 490) & (XY[:, 1] > 20) & (XY[:, 1] < 490)
            rnd = torch.randn((512, 512), device=kt.device(), generator=torch.Generator(kt.device()).manual_seed(3))
            c, _ = kde.backward(pts, kernel, h, h, g, rnd, raw=True, grid_units=True, want_h=False)
            torch.cuda.synchronize()
            assert np.abs(a.cpu().numpy()[inside]).max() < 1e-4 * np.abs(c.cpu().numpy()).max()


def test_backward_serves_and_consumes_the_timing_request():
    """kde_backward records an armed main-kernel timing request (the VJP kernel,
    on both paths) and consumes it: events released afterwards are never
    touched by later calls."""
    import gc

    import torch
    rng = np.random.default_rng(5)
    XY = rng.uniform(0, 64, (3000, 2)).astype(np.float32)
    g, og = kt.grids(synth.BOX_C2, 64, 64)
    pts = kt.to_device(XY)
    go = torch.from_numpy(rng.standard_normal((64, 64)).astype(np.float32)).to(kt.device())
    for fp32 in (False, True):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kde.time_next_main_kernel(a, b)
        kde.backward(pts, "gaussian", 2 * og.dx, 2 * og.dy, g, go, fp32=fp32)
        torch.cuda.synchronize()
        assert a.elapsed_time(b) > 0.0
        del a, b
        gc.collect()
        gp, gh = kde.backward(pts, "gaussian", 2 * og.dx, 2 * og.dy, g, go, fp32=fp32)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(gp.cpu().numpy()))
