"""Pins of the oracle's geometry and extrapolation stencils (Sec. 2.1-2.2, App. A)."""
import numpy as np
import pytest

import workloads as wl
from oracle import geometry as G


@pytest.mark.parametrize("kind,deg", [(G.KIND_4B, 3), (G.KIND_3B, 2), (G.KIND_3N, 2)])
def test_extrapolation_weights_reproduce_polynomials(kind, deg):
    rng = np.random.default_rng(7)
    for theta in (1e-3, 0.17, 0.5, 0.93, 1.0):
        wb, wn = G.extrapolation_weights(kind, theta)
        pos = [-1.0, -2.0, -3.0][:len(wn)] if kind != G.KIND_3N else [0.0, -1.0, -2.0]
        for _ in range(5):
            c = rng.standard_normal(deg + 1)
            p = lambda x: np.polyval(c, x)
            val = wb * p(theta) + sum(w * p(x) for w, x in zip(wn, pos))
            assert abs(val - p(1.0)) < 1e-11 * (1 + np.abs(c).sum())
        assert abs(wb + np.sum(wn) - 1.0) < 1e-13


def test_extrapolation_weight_limits():
    wb, wn = G.extrapolation_weights(G.KIND_4B, 1.0)
    assert abs(wb - 1.0) < 1e-15 and np.max(np.abs(wn)) < 1e-15
    wb, wn = G.extrapolation_weights(G.KIND_3B, 1.0)
    assert abs(wb - 1.0) < 1e-15 and np.max(np.abs(wn)) < 1e-15
    # theta -> 0: the boundary value sits at the fluid node x_i
    wb, wn = G.extrapolation_weights(G.KIND_4B, 1e-12)
    assert np.allclose([wb, *wn], [4, -6, 4, -1], atol=1e-9)
    wb, wn = G.extrapolation_weights(G.KIND_3B, 1e-12)
    assert np.allclose([wb, *wn], [3, -3, 1], atol=1e-9)
    _, wn = G.extrapolation_weights(G.KIND_3N, 0.3)
    assert np.allclose(wn, [3, -3, 1], atol=1e-15)


def test_lagrange_derivative_weights():
    rng = np.random.default_rng(3)
    nodes = [-1.0, 0.0, 1.0]
    for x in (-0.7, 0.2, 0.99):
        c = rng.standard_normal(3)
        w = G.lagrange_deriv_weights(nodes, x)
        val = sum(wk * np.polyval(c, xk) for wk, xk in zip(w, nodes))
        assert abs(val - np.polyval(np.polyder(c), x)) < 1e-13


def test_spline_interpolates_and_circle_crossings():
    w = wl.taylor_couette(128)
    geo = G.Geometry(w.grid, w.bodies)
    # control points lie on their circle to the spline accuracy
    for k, r in ((0, 0.25), (1, 0.75)):
        m = geo.c_body == k
        rad = np.hypot(geo.c_x[m], geo.c_y[m])
        assert np.max(np.abs(rad - r)) < 1e-8
        # normals point into the fluid: outward for the obstacle, inward for the wall
        dot = (geo.c_x[m] * geo.c_nx[m] + geo.c_y[m] * geo.c_ny[m]) / rad
        assert np.all(dot > 0.999) if k == 0 else np.all(dot < -0.999)
    # classification agrees with the analytic circles
    X, Y = wl.node_coords(w.grid)
    R = np.hypot(X, Y)
    assert np.array_equal(geo.solid, (R < 0.25) | (R > 0.75))
    # control points sit on their grid edge, fluid side at distance theta h
    ax0 = geo.c_axis == 0
    xf = geo.x[geo.c_if]
    yf = geo.y[geo.c_jf]
    assert np.allclose(np.abs(geo.c_x[ax0] - xf[ax0]), geo.c_theta[ax0] * geo.h, atol=1e-13)
    assert np.allclose(geo.c_y[ax0], yf[ax0])
    assert np.allclose(np.abs(geo.c_y[~ax0] - yf[~ax0]), geo.c_theta[~ax0] * geo.h, atol=1e-13)
    # every fluid-solid edge has exactly one control point
    edges = (geo.solid[:, 1:] != geo.solid[:, :-1]).sum() + (geo.solid[1:, :] != geo.solid[:-1, :]).sum()
    assert edges == geo.nc


def _poly_field(c, x, y):
    # generic cubic in (x, y)
    return (c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
            + c[6] * x ** 3 + c[7] * x * x * y + c[8] * x * y * y + c[9] * y ** 3)


@pytest.mark.parametrize("make", [lambda: wl.taylor_couette(64), lambda: wl.two_c_shapes_lamb_oseen(128)])
def test_ghost_extensions_exact_on_polynomials(make):
    w = make()
    geo = G.Geometry(w.grid, w.bodies)
    rng = np.random.default_rng(11)
    X, Y = wl.node_coords(w.grid)
    gx, gy = geo.x[geo.g_i], geo.y[geo.g_j]
    c = rng.standard_normal(10)
    f = _poly_field(c, X, Y).ravel()
    bc = _poly_field(c, geo.c_x, geo.c_y)
    ghost = geo.E4b_f @ f + geo.E4b_b @ bc
    assert np.max(np.abs(ghost - _poly_field(c, gx, gy))) < 1e-9
    c[6:] = 0.0          # quadratic
    f = _poly_field(c, X, Y).ravel()
    bc = _poly_field(c, geo.c_x, geo.c_y)
    for Ef, Eb in ((geo.E3b_f, geo.E3b_b), (geo.E3n_f, None)):
        ghost = Ef @ f + (Eb @ bc if Eb is not None else 0.0)
        assert np.max(np.abs(ghost - _poly_field(c, gx, gy))) < 1e-10


def test_poisson_correction_rows():
    """gamma restores the 5-point stencil on both sides of the boundary:
    with psi zero in the solid, -lap_h psi + gamma equals -lap_h of the exact
    field at A+ (ghost values replace solid neighbours) and vanishes at A-."""
    w = wl.taylor_couette(64)
    geo = G.Geometry(w.grid, w.bodies)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(10)
    X, Y = wl.node_coords(w.grid)
    h = geo.h
    exact = _poly_field(c, X, Y)
    psi = np.where(geo.fluid, exact, 0.0)
    bc = _poly_field(c, geo.c_x, geo.c_y)
    gam = geo.Aop @ psi.ravel() + geo.Bop @ bc
    pad = lambda a: np.pad(a, 1)
    lap = lambda a: (pad(a)[1:-1, 2:] + pad(a)[1:-1, :-2] + pad(a)[2:, 1:-1] + pad(a)[:-2, 1:-1] - 4 * a) / h ** 2
    lhs = (-lap(psi)).ravel()[geo.a_lin] + gam
    want = np.where(geo.a_is_ghost, 0.0, (-lap(exact)).ravel()[geo.a_lin])
    assert np.max(np.abs(lhs - want)) < 1e-7 * np.max(np.abs(exact)) / h ** 2


def test_geometry_errors():
    w = wl.taylor_couette(64)
    bad = [wl.BodyDesc(points=w.bodies[0].points[::-1].copy())]
    with pytest.raises(G.GeometryError):
        G.Geometry(w.grid, bad)
    edge = [wl.BodyDesc(points=wl.circle_points((0.9, 0.0), 0.2, 64))]
    with pytest.raises(G.GeometryError):
        G.Geometry(w.grid, edge)
    # two obstacles too close for disjoint bounding regions
    two = [wl.BodyDesc(points=wl.circle_points((-0.2, 0.01), 0.15, 128)),
           wl.BodyDesc(points=wl.circle_points((0.13, 0.013), 0.15, 128))]
    grid = wl.GridDesc(nx=64, ny=64, x0=-1 + 1 / 64, y0=-1 + 1 / 64, h=2 / 64, exterior="free")
    with pytest.raises(G.GeometryError):
        G.Geometry(grid, two)
