"""Pins of the oracle's transport step, boundary vorticity and Kelvin rates
(Sec. 3, Sec. 5.1, Sec. 5.3)."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import geometry as G, transport
from oracle.reconstruct import Reconstructor

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_upwind_weights_match_paper():
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))["upwind_stencils"]
    assert np.allclose(transport.W_LEFT, c["left_biased"], atol=1e-16)
    assert np.allclose(transport.W_RIGHT, c["right_biased"], atol=1e-16)


def _quad(c, x, y):
    return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y


@pytest.mark.parametrize("make", [lambda: wl.taylor_couette(64), lambda: wl.two_c_shapes_lamb_oseen(128)])
def test_boundary_vorticity_exact_for_quadratic_velocity(make):
    rng = np.random.default_rng(4)
    cu, cv = rng.standard_normal(6), rng.standard_normal(6)
    w = make()
    geo = G.Geometry(w.grid, w.bodies, bc_override=(lambda x, y: 0 * x,
                                                    lambda x, y: (_quad(cu, x, y), _quad(cv, x, y))))
    X, Y = wl.node_coords(w.grid)
    U = np.zeros((geo.ny + 2, geo.nx + 2))
    V = np.zeros_like(U)
    has = geo.cls != G.SOLID
    U[1:-1, 1:-1] = np.where(has, _quad(cu, X, Y), 0.0)
    V[1:-1, 1:-1] = np.where(has, _quad(cv, X, Y), 0.0)
    wb = transport.boundary_vorticity(geo, U, V)
    x, y = geo.c_x, geo.c_y
    dvdx = cv[1] + 2 * cv[3] * x + cv[4] * y
    dudy = cu[2] + cu[4] * x + 2 * cu[5] * y
    assert np.max(np.abs(wb - (dvdx - dudy))) < 1e-9


def test_velocity_extension_feeds_exact_boundary_vorticity():
    """Third-order velocity extension + the boundary stencil: exact for quadratic fields."""
    rng = np.random.default_rng(8)
    cu, cv = rng.standard_normal(6), rng.standard_normal(6)
    w = wl.taylor_couette(64)
    geo = G.Geometry(w.grid, w.bodies, bc_override=(lambda x, y: 0 * x,
                                                    lambda x, y: (_quad(cu, x, y), _quad(cv, x, y))))
    X, Y = wl.node_coords(w.grid)
    U = np.zeros((geo.ny + 2, geo.nx + 2))
    V = np.zeros_like(U)
    U[1:-1, 1:-1] = np.where(geo.fluid, _quad(cu, X, Y), 0.0)
    V[1:-1, 1:-1] = np.where(geo.fluid, _quad(cv, X, Y), 0.0)
    U[geo.g_j + 1, geo.g_i + 1] = geo.E3b_f @ U[1:-1, 1:-1].ravel() + geo.E3b_b @ geo.c_ub[:, 0]
    V[geo.g_j + 1, geo.g_i + 1] = geo.E3b_f @ V[1:-1, 1:-1].ravel() + geo.E3b_b @ geo.c_ub[:, 1]
    wb = transport.boundary_vorticity(geo, U, V)
    x, y = geo.c_x, geo.c_y
    want = (cv[1] + 2 * cv[3] * x + cv[4] * y) - (cu[2] + cu[4] * x + 2 * cu[5] * y)
    assert np.max(np.abs(wb - want)) < 1e-9


def _state(make, seed):
    w = make()
    geo = G.Geometry(w.grid, w.bodies)
    R = Reconstructor(geo)
    rng = np.random.default_rng(seed)
    omega = np.where(geo.fluid, wl.seeded_vortices(w.grid, seed, count=5), 0.0)
    Gam = rng.uniform(-0.3, 0.3, geo.nbc)
    rec = R.reconstruct(omega, Gam)
    return w, geo, omega, rec


@pytest.mark.parametrize("make", [wl.cylinder_small, lambda: wl.taylor_couette(64)])
def test_conservation_telescopes(make):
    """h^2 sum_R domega/dt = -h sum_dR (F+Q).n on fluid rectangles, and the
    Kelvin rate equals the net flux through dR_k."""
    w, geo, omega, rec = _state(make, 2)
    dw, dG, wb, (Fx, Qx, Fy, Qy, *_) = transport.rhs(geo, omega, rec.U, rec.V, w.grid.nu)
    h = geo.h
    Tx, Ty = Fx + Qx, Fy + Qy
    rng = np.random.default_rng(0)
    done = 0
    for _ in range(200):
        i0, j0 = rng.integers(2, geo.nx - 12), rng.integers(2, geo.ny - 12)
        i1, j1 = i0 + rng.integers(1, 10), j0 + rng.integers(1, 10)
        if not geo.fluid[j0 - 2:j1 + 3, i0 - 2:i1 + 3].all():
            continue
        lhs = h * h * dw[j0:j1 + 1, i0:i1 + 1].sum()
        rhs = -h * (Tx[j0:j1 + 1, i1 + 1].sum() - Tx[j0:j1 + 1, i0].sum()
                    + Ty[j1 + 1, i0:i1 + 1].sum() - Ty[j0, i0:i1 + 1].sum())
        assert abs(lhs - rhs) < 1e-12 * (np.abs(Tx).max() + np.abs(Ty).max()) * h * 40
        done += 1
    assert done > 10
    # Kelvin rate of R_k = -h * outward flux; the same through R_k grown by one node
    i0, i1, j0, j1 = geo.rects[0]
    ring = dw[j0 - 1:j1 + 2, i0 - 1:i1 + 2].sum() - dw[j0:j1 + 1, i0:i1 + 1].sum()
    rhs = -h * (Tx[j0 - 1:j1 + 2, i1 + 2].sum() - Tx[j0 - 1:j1 + 2, i0 - 1].sum()
                + Ty[j1 + 2, i0 - 1:i1 + 2].sum() - Ty[j0 - 1, i0 - 1:i1 + 2].sum())
    assert abs(dG[0] + h * h * ring - rhs) < 1e-11 * (abs(rhs) + abs(dG[0]) + 1e-3)


def test_uniform_free_stream_is_steady():
    """omega = 0 and a uniform stream past nothing: no vorticity flux."""
    grid = wl.GridDesc(nx=24, ny=20, x0=0.0, y0=0.0, h=0.1, exterior="free", u_inf=(1.0, 0.5))
    body = wl.BodyDesc(points=wl.circle_points((1.23, 1.017), 0.35, 64))
    geo = G.Geometry(grid, [body])
    U = np.zeros((geo.ny + 2, geo.nx + 2))
    V = np.zeros_like(U)
    U[:] = 1.0
    V[:] = 0.5
    omega = np.zeros((geo.ny, geo.nx))
    far = np.ones_like(geo.fluid)
    dw, *_ = transport.rhs(geo, omega, U, V, 0.01, wb=np.zeros(geo.nc))
    assert np.max(np.abs(dw)) == 0.0
