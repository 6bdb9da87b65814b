"""The oracle's control-volume force (Noca's momentum formulation, Sec. 5.4)
pinned to what the mathematics fixes:

* steady inviscid flow past a cylinder with circulation G in a stream U
  (complex potential U (z + R^2/z) + G log(z) / (2 pi i)): the box integrals
  give the Kutta-Joukowski force (0, -U G) (no drag), for any box around the
  body and any origin of x, converging as h -> 0;
* a Lamb-Oseen vortex carried by a uniform stream (an exact, viscous,
  unsteady Navier-Stokes solution whose vorticity crosses the box) with no
  body inside the box: the force vanishes, at second order in h, whatever
  the origin, while the separate terms stay of order one.  A dropped term,
  a wrong sign or factor in gamma or in the time-derivative part fails it.

The control-volume moment (M = d I/dt + S_lambda) likewise:

* the cut-cell quadrature of I: the fluid area of a box around a disk equals
  the box minus the polygon's area, and the polar moment |x - c|^2/2 over it
  converges at second order to the exact value;
* the same inviscid flow: moment (c_x - x_x) (-U G) about any origin x (zero
  about the centre: the pressure on a circle acts through its centre);
* the body-free Lamb-Oseen vortex: zero moment at second order.
"""
import numpy as np

import workloads as wl
from oracle import geometry as OG
from oracle import loads as OL


def _ring_fields(grid, f):
    xs = grid.x0 + grid.h * np.arange(-1, grid.nx + 1)
    ys = grid.y0 + grid.h * np.arange(-1, grid.ny + 1)
    X, Y = np.meshgrid(xs, ys)
    u, v, w = f(X, Y)
    return u, v, w[1:-1, 1:-1]


def _box(grid, x0, x1, y0, y1):
    h = grid.h
    return (int(round((x0 - grid.x0) / h)), int(round((x1 - grid.x0) / h)),
            int(round((y0 - grid.y0) / h)), int(round((y1 - grid.y0) / h)))


def test_kutta_joukowski():
    U0, R, G, c = 1.0, 0.5, 1.3, (0.013, -0.021)

    def f(X, Y):
        z = (X - c[0]) + 1j * (Y - c[1])
        dw = U0 * (1 - R * R / z ** 2) + G / (2j * np.pi * z)
        return dw.real, -dw.imag, np.zeros_like(X)

    for box, origin in [((-1, 1, -1, 1), (0.0, 0.0)), ((-1.5, 2.2, -0.9, 1.7), (0.3, -0.4))]:
        err = []
        for h in (1 / 16, 1 / 32, 1 / 64):
            n = int(round(6 / h))
            g = wl.GridDesc(nx=n, ny=n, x0=-3 + 0.5 * h, y0=-3 + 0.5 * h, h=h, nu=0.0)
            U, V, w = _ring_fields(g, f)
            _, Sg = OL.control_volume_terms(g, w, U, V, _box(g, *box), origin)
            err.append(np.hypot(Sg[0], Sg[1] + U0 * G))
        assert err[-1] < 1e-4 * U0 * G and err[-1] < err[0], err


def test_body_free_viscous_vortex_feels_no_force():
    G, nu, Uinf = 1.1, 0.02, (0.7, 0.2)

    def at(grid, t):
        xc, yc = -0.3 + Uinf[0] * t, 0.1 + Uinf[1] * t
        a = 4 * nu * t

        def f(X, Y):
            dx, dy = X - xc, Y - yc
            r2 = dx * dx + dy * dy
            q = G / (2 * np.pi * r2) * (-np.expm1(-r2 / a))      # u_theta / r
            return Uinf[0] - dy * q, Uinf[1] + dx * q, G / (np.pi * a) * np.exp(-r2 / a)
        return _ring_fields(grid, f)

    t1, dt = 1.5, 1e-4
    for origin in [(0.0, 0.0), (0.5, -0.7)]:
        F, size = [], []
        for h in (1 / 32, 1 / 64, 1 / 128):
            n = int(round(4 / h))
            g = wl.GridDesc(nx=n, ny=n, x0=-2 + 0.5 * h, y0=-2 + 0.5 * h, h=h, nu=nu)
            box = _box(g, -0.8, 0.48, -0.6, 0.64)
            Sp = OL.control_volume_terms(g, at(g, t1 + dt)[2], *at(g, t1 + dt)[:2], box, origin)[0]
            Sm = OL.control_volume_terms(g, at(g, t1 - dt)[2], *at(g, t1 - dt)[:2], box, origin)[0]
            U, V, w = at(g, t1)
            _, Sg = OL.control_volume_terms(g, w, U, V, box, origin)
            F.append(np.hypot(*(Sg - (Sp - Sm) / (2 * dt))))
            size.append(np.hypot(*Sg))
        assert F[1] < F[0] / 3 and F[2] < F[1] / 3, F
        assert F[2] < 1e-4 * size[2], (F, size)


def test_cut_cell_quadrature():
    R, c = 0.3, (0.013, -0.021)
    err = []
    for h in (1 / 32, 1 / 64, 1 / 128):
        n = int(round(2 / h))
        g = wl.GridDesc(nx=n, ny=n, x0=-1 + 0.5 * h, y0=-1 + 0.5 * h, h=h, nu=0.01)
        b = wl.BodyDesc(points=wl.circle_points(c, R, 512), center=c)
        geo = OG.Geometry(g, [b])
        W = OL.fluid_weights(geo)
        i0, i1, j0, j1 = box = _box(g, -0.7, 0.8, -0.6, 0.75)
        xa, xb, ya, yb = g.x0 + i0 * h, g.x0 + i1 * h, g.y0 + j0 * h, g.y0 + j1 * h
        P = b.points
        polygon = 0.5 * abs(np.sum(P[:, 0] * np.roll(P[:, 1], -1) - np.roll(P[:, 0], -1) * P[:, 1]))
        fac = np.ones((j1 - j0 + 1, i1 - i0 + 1))
        fac[[0, -1], :] *= 0.5
        fac[:, [0, -1]] *= 0.5
        area = np.sum(W[j0:j1 + 1, i0:i1 + 1] * fac)
        assert abs(area - ((xb - xa) * (yb - ya) - polygon)) < 1e-7
        polar = OL.cv_moment_volume(geo, np.ones((n, n)), W, box, c)
        exact = 0.5 * (((xb - c[0]) ** 3 - (xa - c[0]) ** 3) / 3 * (yb - ya)
                       + ((yb - c[1]) ** 3 - (ya - c[1]) ** 3) / 3 * (xb - xa)) - np.pi * R ** 4 / 4
        err.append(abs(polar - exact))
    assert err[1] < err[0] / 3 and err[2] < err[1] / 3, err


def test_moment_of_inviscid_flow_with_circulation():
    U0, R, G, c = 1.0, 0.5, 1.3, (0.013, -0.021)

    def f(X, Y):
        z = (X - c[0]) + 1j * (Y - c[1])
        dw = U0 * (1 - R * R / z ** 2) + G / (2j * np.pi * z)
        return dw.real, -dw.imag, np.zeros_like(X)

    for box, origin in [((-1, 1, -1, 1), c), ((-1.5, 2.2, -0.9, 1.7), (0.3, -0.4))]:
        expect = -(c[0] - origin[0]) * U0 * G
        err = []
        for h in (1 / 16, 1 / 32, 1 / 64):
            n = int(round(6 / h))
            g = wl.GridDesc(nx=n, ny=n, x0=-3 + 0.5 * h, y0=-3 + 0.5 * h, h=h, nu=0.0)
            U, V, w = _ring_fields(g, f)
            err.append(abs(OL.cv_moment_surface(g, w, U, V, _box(g, *box), origin) - expect))
        assert err[-1] < 1e-5 and err[-1] < err[0], err


def test_body_free_viscous_vortex_feels_no_moment():
    G, nu, Uinf = 1.1, 0.02, (0.7, 0.2)

    def at(grid, t):
        xc, yc = -0.3 + Uinf[0] * t, 0.1 + Uinf[1] * t
        a = 4 * nu * t

        def f(X, Y):
            dx, dy = X - xc, Y - yc
            r2 = dx * dx + dy * dy
            q = G / (2 * np.pi * r2) * (-np.expm1(-r2 / a))
            return Uinf[0] - dy * q, Uinf[1] + dx * q, G / (np.pi * a) * np.exp(-r2 / a)
        return _ring_fields(grid, f)

    t1, dt = 1.5, 1e-4
    for origin in [(0.0, 0.0), (0.5, -0.7)]:
        M, size = [], []
        for h in (1 / 32, 1 / 64, 1 / 128):
            n = int(round(4 / h))
            g = wl.GridDesc(nx=n, ny=n, x0=-2 + 0.5 * h, y0=-2 + 0.5 * h, h=h, nu=nu)
            geo = OG.Geometry(g, [])
            W = OL.fluid_weights(geo)
            box = _box(g, -0.8, 0.48, -0.6, 0.64)
            Ip = OL.cv_moment_volume(geo, at(g, t1 + dt)[2], W, box, origin)
            Im = OL.cv_moment_volume(geo, at(g, t1 - dt)[2], W, box, origin)
            U, V, w = at(g, t1)
            S = OL.cv_moment_surface(g, w, U, V, box, origin)
            M.append(abs((Ip - Im) / (2 * dt) + S))
            size.append(abs(S))
        # against terms of about 0.07 (origin at 0) and 0.3: second order about
        # the origin; about the other point not monotone, but below 3e-4 of
        # the terms
        assert M[2] < 3e-4 * size[2] and M[2] < M[0], (M, size)
        if origin == (0.0, 0.0):
            assert M[1] < M[0] / 3 and M[2] < M[1] / 3, M

