"""The full Navier-Stokes convergence case of Sec. 6 (its parameter table):
a Lamb-Oseen vortex (circulation pi, nu = 0.001) centred on a cylinder
(centre (0.507, 0.507), radius 0.15) that rotates with the vortex's own
velocity at its radius, so that the vortex is an exact solution outside the
cylinder for all time; grid x_ij = (i/N, j/N), free space, RK3 with
C_stab = 0.7 from t = 1.  Shared by the oracle and GPU tests: the exact
fields and the case set-up, no arithmetic of the method."""
import numpy as np

import workloads as wl

G0, NU, XC, R = np.pi, 0.001, (0.507, 0.507), 0.15


def exact(X, Y, t):
    """Vorticity and velocity of the vortex at time t."""
    dx, dy = X - XC[0], Y - XC[1]
    r2 = dx * dx + dy * dy
    a = 4 * NU * t
    q = G0 / (2 * np.pi * r2) * (-np.expm1(-r2 / a))      # u_theta / r
    return G0 / (np.pi * a) * np.exp(-r2 / a), -q * dy, q * dx


def rotation(t):
    """Angular velocity of the cylinder: the vortex's u_theta(R) / R."""
    return G0 / (2 * np.pi * R * R) * (-np.expm1(-R * R / (4 * NU * t)))


def case(n, t0):
    h = 1.0 / n
    grid = wl.GridDesc(nx=n, ny=n, x0=0.0, y0=0.0, h=h, exterior="free", u_inf=(0.0, 0.0), nu=NU)
    body = wl.BodyDesc(points=wl.circle_points(XC, R, max(256, int(8 * np.pi * R / h))), center=XC,
                       omega_rigid=rotation(t0))
    return grid, body


def a_max(t0):
    """Bound on |u_x| + |u_y| of the flow: the wall speed at t0, both
    components at once."""
    return np.sqrt(2.0) * rotation(t0) * R


def time_step(dt_max, t0, t1, c_stab=0.7):
    """Number of steps and dt over [t0, t1] with dt <= C_stab dt_max (dt_max
    from the caller's stability bound for a_max(t0))."""
    n = int(np.ceil((t1 - t0) / (c_stab * dt_max)))
    return n, (t1 - t0) / n


def initial(grid, fluid, rect, t0):
    """omega at t0 on the fluid nodes and the circulation around the bounding
    region (h^2 times the vortex's vorticity summed over it)."""
    X, Y = wl.node_coords(grid)
    w0, _, _ = exact(X, Y, t0)
    i0, i1, j0, j1 = rect
    return np.where(fluid, w0, 0.0), np.array([grid.h ** 2 * w0[j0:j1 + 1, i0:i1 + 1].sum()])


def errors(grid, fluid, om, U, V, t):
    """(L2, Linf) of the vorticity and of the velocity over the fluid nodes."""
    X, Y = wl.node_coords(grid)
    we, ue, ve = exact(X, Y, t)
    ew = np.abs(om - we)[fluid]
    eu = np.hypot(U[1:-1, 1:-1] - ue, V[1:-1, 1:-1] - ve)[fluid]
    return np.sqrt(np.mean(ew ** 2)), ew.max(), np.sqrt(np.mean(eu ** 2)), eu.max()
