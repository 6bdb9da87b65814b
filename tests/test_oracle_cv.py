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
  a wrong sign or factor in gamma or in the time-derivative part fails it."""
import numpy as np

import workloads as wl
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
