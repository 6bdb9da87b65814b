"""Surface loads of the oracle (Sec. 5.4) pinned to what the mathematics fixes:

* the vorticity gradient at a control point is exact on every quadratic
  field (quadratic along the grid line, one-sided three-point derivative of
  values interpolated quadratically along the rows);
* the surface integration: a tangential pressure gradient d p/ds = s_x gives
  p = x - x_0, and its pressure force is -(area, 0) (divergence theorem),
  converging at second order; a constant wall vorticity W on a circle of
  radius R gives zero force and the torque 2 pi nu W R^2, at second order;
* the ordering follows the curve: consecutive control points are close."""
import numpy as np

import workloads as wl
from oracle import geometry as OG
from oracle import loads as OL


def _circle(h):
    n = int(round(4 / h))
    w = wl.cylinder(nx=n, ny=n, h=h, points=256, center=(2.0, 0.0))
    return OG.Geometry(w.grid, w.bodies)


def test_gradient_exact_on_quadratics():
    g = OG.Geometry(wl.cylinder_small().grid, wl.cylinder_small().bodies)
    X, Y = np.meshgrid(g.x, g.y)
    q = lambda x, y: 0.3 + 1.1 * x - 0.7 * y + 0.5 * x * x - 0.9 * x * y + 0.4 * y * y
    grad = OL.vorticity_gradient(g, q(X, Y), q(g.c_x, g.c_y))
    assert np.max(np.abs(grad[:, 0] - (1.1 + 1.0 * g.c_x - 0.9 * g.c_y))) < 1e-12
    assert np.max(np.abs(grad[:, 1] - (-0.7 - 0.9 * g.c_x + 0.8 * g.c_y))) < 1e-12


def test_integration_converges_to_the_analytic_loads():
    R, W = 0.5, 1.7
    ep, ef, et = [], [], []
    for h in (1 / 32, 1 / 64, 1 / 128):
        g = _circle(h)
        nu = g.grid.nu
        o = OL.surface_order(g, 0)
        # d p/ds = s_x = -n_y  ->  p = x - x_0, pressure force -(pi R^2, 0)
        p, F = OL.integrate_surface(g, np.zeros(g.nc), -g.c_ny / nu)
        ep.append(np.max(np.abs(p[o] - (g.c_x[o] - g.c_x[o[0]]))))
        ef.append(np.hypot(F[0, 0] + np.pi * R * R, F[0, 1]))
        # constant wall vorticity: no force, torque 2 pi nu W R^2
        _, F2 = OL.integrate_surface(g, np.full(g.nc, W), np.zeros(g.nc))
        assert np.hypot(F2[0, 0], F2[0, 1]) < 1e-14
        et.append(abs(F2[0, 2] - 2 * np.pi * nu * W * R * R))
        # consecutive control points lie close along the curve
        xy = np.stack([g.c_x[o], g.c_y[o]], 1)
        assert np.max(np.linalg.norm(np.roll(xy, -1, 0) - xy, axis=1)) < 1.5 * h
    for e in (ep, ef, et):
        assert e[1] < e[0] / 3.0 and e[2] < e[1] / 3.0, e


def test_solid_body_rotation_carries_no_shear():
    """A body rotating at Omega with the wall vorticity of solid-body rotation
    (2 Omega) and no vorticity flux: no viscous traction, so the torque comes
    only from the pressure, which on a circle the rotation leaves uniform."""
    import dataclasses
    w = wl.cylinder_small()
    b = dataclasses.replace(w.bodies[0], omega_rigid=1.3)
    g = OG.Geometry(w.grid, [b])
    p, F = OL.integrate_surface(g, np.full(g.nc, 2.6), np.zeros(g.nc))
    assert np.max(np.abs(F[0])) < 1e-12, F


def test_loads_of_a_symmetric_flow():
    """A cylinder on a grid symmetric about its axis, started from rest: the
    flow stays mirror-symmetric, so the lift and the torque vanish to
    rounding while the drag is positive."""
    from oracle import ns as ONS
    from oracle.reconstruct import Reconstructor
    w = wl.cylinder_small()
    g = OG.Geometry(w.grid, w.bodies)
    st = ONS.Stepper(g)
    om, G = np.zeros((w.grid.ny, w.grid.nx)), np.zeros(g.nbc)
    for _ in range(4):
        om, G = st.step(om, G, w.dt)
    r = Reconstructor(g).reconstruct(om, G)
    L = OL.surface_loads(g, om, r.U, r.V)
    Fx, Fy, T = L["forces"][0]
    assert Fx > 0.0
    assert abs(Fy) < 1e-10 * Fx and abs(T) < 1e-10 * Fx
