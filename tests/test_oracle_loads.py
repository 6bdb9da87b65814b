"""Surface loads of the oracle (Sec. 5.4) pinned to what the mathematics fixes:

* the vorticity gradient at a control point is exact on every quadratic
  field (quadratic along the grid line, one-sided three-point derivative of
  values interpolated quadratically along the rows);
* the surface integration: a tangential pressure gradient d p/ds = s_x gives
  p = x - x_0, and its pressure force is -(area, 0) (divergence theorem),
  converging at second order; a constant wall vorticity W on a circle of
  radius R gives zero force and the torque 2 pi nu W R^2, at second order;
* the ordering follows the curve: consecutive control points are close."""
import dataclasses

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


def test_pressure_loads_equal_the_vorticity_flux_identities():
    """Sec. 5.4 writes the pressure force and moment directly in terms of the
    tangential pressure gradient d p/ds = nu d omega/dn.  On a closed curve,
    with n into the fluid and s = k x n, integration by parts gives
    F_p = int (y, -x) dp/ds ds and M_p = -(1/2) int |x - c|^2 dp/ds ds.  (The
    paper prints the moment with a plus sign; the traction -p n fixes the
    minus, reading 25.)  An ellipse with a smooth surface pressure
    P = sin(2x) cos(y) + x y^2: the oracle's route (p integrated along the
    curve, then -p n summed) and both identities converge at second order to
    the boundary integrals of -P n evaluated on the exact ellipse."""
    from workloads import ellipse_points
    ctr, a, b, ang = (2.0, 0.05), 0.8, 0.45, 0.35
    P = lambda x, y: np.sin(2 * x) * np.cos(y) + x * y * y
    dP = lambda x, y: (2 * np.cos(2 * x) * np.cos(y) + y * y, -np.sin(2 * x) * np.sin(y) + 2 * x * y)
    # exact loads: the trapezoid rule in the ellipse's angle (spectrally accurate)
    t = 2 * np.pi * np.arange(4096) / 4096
    ca, sa = np.cos(ang), np.sin(ang)
    x = ctr[0] + ca * a * np.cos(t) - sa * b * np.sin(t)
    y = ctr[1] + sa * a * np.cos(t) + ca * b * np.sin(t)
    xp = -ca * a * np.sin(t) - sa * b * np.cos(t)
    yp = -sa * a * np.sin(t) + ca * b * np.cos(t)
    dt = 2 * np.pi / t.size
    Pv = P(x, y)
    F_ex = np.array([-np.sum(Pv * yp), np.sum(Pv * xp)]) * dt              # -P n ds, n ds = (y', -x') dt
    M_ex = np.sum(Pv * ((x - ctr[0]) * xp + (y - ctr[1]) * yp)) * dt        # (x - c) x (-P n ds)
    errs = {"route": [], "F_id": [], "M_id": []}
    M_printed = []
    for h in (1 / 32, 1 / 64, 1 / 128):
        n = int(round(4 / h))
        w = wl.cylinder(nx=n, ny=n, h=h, points=256, center=ctr)
        body = dataclasses.replace(w.bodies[0], points=ellipse_points(ctr, a, b, ang, 256))
        g = OG.Geometry(w.grid, [body])
        nu = g.grid.nu
        gx, gy = dP(g.c_x, g.c_y)
        dpds = gx * (-g.c_ny) + gy * g.c_nx
        p, F = OL.integrate_surface(g, np.zeros(g.nc), dpds / nu)
        errs["route"].append(max(np.hypot(*(F[0, :2] - F_ex)), abs(F[0, 2] - M_ex)))
        o = OL.surface_order(g, 0)
        xy = np.stack([g.c_x[o], g.c_y[o]], axis=1)
        ds = np.linalg.norm(np.roll(xy, -1, axis=0) - xy, axis=1)
        wgt = 0.5 * (ds + np.roll(ds, 1))
        F_id = np.array([np.sum(xy[:, 1] * dpds[o] * wgt), np.sum(-xy[:, 0] * dpds[o] * wgt)])
        r2 = np.sum((xy - np.asarray(ctr)) ** 2, axis=1)
        M_id = -0.5 * np.sum(r2 * dpds[o] * wgt)
        errs["F_id"].append(np.hypot(*(F_id - F_ex)))
        errs["M_id"].append(abs(M_id - M_ex))
        M_printed.append(-M_id)
    # second order: about 16x over two halvings of h (each halving at least 2x:
    # the control points' positions along the curve change with h)
    for k, e in errs.items():
        assert e[1] < e[0] / 2.0 and e[2] < e[1] / 2.0 and e[2] < e[0] / 10.0, (k, e)
        assert e[2] < 2e-3 * (np.hypot(*F_ex) + abs(M_ex)), (k, e)
    assert abs(M_ex) > 1e-2 and abs(M_printed[-1] - M_ex) > abs(M_ex)
