"""Pins of the oracle's lateral transport step (MUSCL + superbee, CN with frozen slopes; section 3.4).

* first-order limit: where every limited slope vanishes the step is CN with
  the textbook first-order upwind operator -- checked against a dense solve;
* linear data: away from the inflow boundary the step is an exact shift
  (second-order reconstruction: superbee(1) = 1);
* reflection x -> -x with c -> -c and the transpose x <-> y (the mirrored
  upwind ratio for negative velocity);
* conservation for data away from the boundaries;
* smooth translation converges at close to second order.
"""
import numpy as np
import pytest
from scipy import stats


def _orc(oracle_mod, inputs):
    c = inputs.small()
    return oracle_mod.Oracle(c["grid"], c["phys"])


def _upwind_matrix(nx, ny, dx, dy, cx, cy):
    """Textbook first-order upwind divergence with zero inflow, as a dense matrix."""
    n = nx * ny
    U = np.zeros((n, n))
    for p in range(nx):
        for q in range(ny):
            k = p * ny + q
            U[k, k] += abs(cx) / dx + abs(cy) / dy
            if cx > 0 and p > 0:
                U[k, k - ny] -= cx / dx
            if cx < 0 and p < nx - 1:
                U[k, k + ny] -= -cx / dx
            if cy > 0 and q > 0:
                U[k, k - 1] -= cy / dy
            if cy < 0 and q < ny - 1:
                U[k, k + 1] -= -cy / dy
    return U


@pytest.mark.parametrize("cx,cy", [(0.3, 0.2), (-0.25, 0.1), (0.15, -0.35), (-0.2, -0.3), (0.0, 0.4)])
def test_checkerboard_reduces_to_first_order_cn(oracle_mod, inputs, cx, cy):
    o = _orc(oracle_mod, inputs)
    nx, ny, dx, dy, h = 7, 6, 0.2, 0.25, 0.3
    p, q = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    pl = 1.0 + 0.5 * ((p + q) % 2)          # every interior difference alternates sign -> delta = 0
    pl[0, :] = pl[:, 0] = 0.0               # keep the boundary rows oscillating too
    pl = np.where((p + q) % 2 == 0, 0.0, pl)
    got = o.transport_plane(pl, cx, cy, h, dx, dy)
    U = _upwind_matrix(nx, ny, dx, dy, cx, cy)
    ref = np.linalg.solve(np.eye(nx * ny) + 0.5 * h * U, (np.eye(nx * ny) - 0.5 * h * U) @ pl.reshape(-1))
    assert np.allclose(got.reshape(-1), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("cx,cy", [(0.3, 0.2), (-0.3, 0.2), (0.2, -0.1), (-0.15, -0.25)])
def test_linear_data_shifts_exactly_in_interior(oracle_mod, inputs, cx, cy):
    o = _orc(oracle_mod, inputs)
    nx = ny = 40
    dx = dy = 0.1
    h = 0.04
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y, indexing="ij")
    sx, sy = 0.7, -0.4
    pl = 10.0 + sx * X + sy * Y
    got = o.transport_plane(pl, cx, cy, h, dx, dy)
    ref = pl - h * (cx * sx + cy * sy)
    inner = np.s_[12:28, 12:28]   # the inflow error decays like (h|c|/2dx)^k; 12 cells -> below rounding
    assert np.allclose(got[inner], ref[inner], rtol=1e-13, atol=1e-13)


def test_reflection_and_transpose_symmetry(oracle_mod, inputs):
    o = _orc(oracle_mod, inputs)
    rng = np.random.default_rng(4)
    pl = rng.uniform(0, 1, (9, 9)) ** 3
    a = o.transport_plane(pl, 0.31, -0.17, 0.2, 0.1, 0.1)
    b = o.transport_plane(pl[::-1, :], -0.31, -0.17, 0.2, 0.1, 0.1)[::-1, :]
    c = o.transport_plane(pl[:, ::-1], 0.31, 0.17, 0.2, 0.1, 0.1)[:, ::-1]
    d = o.transport_plane(pl.T, -0.17, 0.31, 0.2, 0.1, 0.1).T
    assert np.allclose(a, b, rtol=1e-14, atol=1e-15)
    assert np.allclose(a, c, rtol=1e-14, atol=1e-15)
    assert np.allclose(a, d, rtol=1e-14, atol=1e-15)


def test_conservation_away_from_boundaries(oracle_mod, inputs):
    o = _orc(oracle_mod, inputs)
    nx = ny = 30
    x = np.arange(nx) - 14.5
    X, Y = np.meshgrid(x, x, indexing="ij")
    pl = np.exp(-(X ** 2 + Y ** 2) / 4.0)
    pl[np.abs(pl) < 1e-30] = 0
    got = o.transport_plane(pl, 0.2, -0.13, 0.1, 0.1, 0.1)
    assert abs(got.sum() - pl.sum()) < 1e-12 * pl.sum()
    # scaling (the limiter is homogeneous of degree one)
    got3 = o.transport_plane(3.0 * pl, 0.2, -0.13, 0.1, 0.1, 0.1)
    assert np.allclose(got3, 3.0 * got, rtol=1e-13, atol=1e-14 * abs(got).max())


def test_smooth_translation_converges(oracle_mod, inputs):
    """Gaussian bump translated by c*z; cell-average error falls ~2nd order (limiter clips the peak)."""
    o = _orc(oracle_mod, inputs)
    cx, cy, L, z, s = 0.5, 0.3, 4.0, 1.0, 0.35
    errs = []
    for n in (40, 80, 160):
        dx = L / n
        h = 0.5 * dx          # CFL fixed
        steps = int(round(z / h))
        e = np.linspace(-L / 2, L / 2, n + 1)
        cdf = lambda mu: np.diff(stats.norm.cdf(e, mu, s)) / dx
        pl = np.outer(cdf(-0.5), cdf(-0.3))
        for _ in range(steps):
            pl = o.transport_plane(pl, cx, cy, h, dx, dx)
        ref = np.outer(cdf(-0.5 + cx * z), cdf(-0.3 + cy * z))
        errs.append(np.abs(pl - ref).sum() * dx * dx)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 2.8 and r2 > 2.8, (errs, r1, r2)
