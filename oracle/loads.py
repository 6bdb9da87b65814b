"""Surface loads on the immersed bodies (Sec. 5.4), FP64 reference.

Test infrastructure: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg use the oracle; the library shares none of this code.

* Shear stress: tau(s) = nu omega_b(s) at every control point.
* Vorticity gradient at a control point: the derivatives of the vorticity
  field extended past the boundary with omega_b (E3b at the ghosts), taken
  with the stencil points of the vorticity boundary condition (Sec. 5.3) --
  along the grid line the derivative of the quadratic through the three line
  nodes, across it the one-sided three-point derivative from omega_b and two
  values interpolated along the neighbouring rows -- projected on the unit
  normal into the fluid.
* Surface pressure relative to the first control point of each body: the
  tangential pressure gradient equals nu d omega / dn on a stationary no-slip
  wall, integrated along the control points in the order of the boundary
  curve's parameter (trapezoid rule on the chords).
* Force and torque on each body (about its centre): the surface integral of
  -p n + nu omega s (n: unit normal into the fluid, s = k x n), the
  trapezoid rule over the same closed polygon; a constant added to p
  integrates to zero around the body, so the relative pressure suffices.
* A body in steady rigid motion (constant translation, rotation Omega about
  its centre): the rigid motion carries vorticity 2 Omega and no strain, so
  the viscous traction is nu (omega - 2 Omega) s; the wall's centripetal
  acceleration -Omega^2 (x - c) adds Omega^2 (x - c).s to the tangential
  pressure gradient (momentum balance at the no-slip wall).  Bodies with
  sampled boundary data are treated as stationary walls.
"""
import numpy as np

from .transport import boundary_vorticity, vorticity_extensions


def vorticity_gradient(geom, omega_ext, wb):
    """(d_x omega, d_y omega) at every control point.  omega_ext: [ny][nx]
    vorticity with the ghost values of the extended field; wb: omega_b."""
    g = np.zeros((geom.nc, 2))
    for c in range(geom.nc):
        terms, bc = geom.wb_stencils[c]
        # the boundary-vorticity stencil computes d_x u_y (its component-1
        # terms) minus d_y u_x (its component-0 terms); applied to one scalar
        # field the two parts are d_x and -d_y of that field
        dx = dy = 0.0
        for (i, j, comp, w) in terms:
            if comp == 1:
                dx += w * omega_ext[j, i]
            else:
                dy -= w * omega_ext[j, i]
        for (comp, w) in bc:
            if comp == 1:
                dx += w * wb[c]
            else:
                dy -= w * wb[c]
        g[c] = dx, dy
    return g


def extended_vorticity(geom, omega, wb):
    """Vorticity with the ghost values E3b (third order, with omega_b)."""
    _, e3b, _ = vorticity_extensions(geom, omega, wb)
    ext = np.array(omega, dtype=np.float64, copy=True)
    ext[geom.g_j, geom.g_i] = e3b
    return ext


def surface_order(geom, k):
    """Control points of body k in the order of the curve's parameter."""
    idx = np.nonzero(geom.c_body == k)[0]
    return idx[np.argsort(geom.c_seg[idx] + geom.c_s[idx], kind="stable")]


def integrate_surface(geom, wb, dwdn):
    """Relative surface pressure (nu d omega/dn integrated along each body's
    control points from the first one) and (F_x, F_y, torque) per body."""
    nu = geom.grid.nu
    nrm = np.stack([geom.c_nx, geom.c_ny], axis=1)
    p = np.zeros(geom.nc)
    forces = np.zeros((len(geom.bodies), 3))
    for k, b in enumerate(geom.bodies):
        order = surface_order(geom, k)
        if order.size == 0:
            continue
        xy = np.stack([geom.c_x[order], geom.c_y[order]], axis=1)
        ds = np.linalg.norm(np.roll(xy, -1, axis=0) - xy, axis=1)   # chord to the next point (closed)
        Om = 0.0 if getattr(b, "bc_samples", None) is not None else float(b.omega_rigid)
        rel = xy - np.asarray(b.center, dtype=np.float64)
        nn = nrm[order]
        # tangential pressure gradient: viscous part plus the rigid rotation's
        # centripetal part Omega^2 (x - c).s
        dpds = nu * dwdn[order] + Om * Om * (rel[:, 0] * (-nn[:, 1]) + rel[:, 1] * nn[:, 0])
        pk = np.zeros(order.size)
        for q in range(1, order.size):
            pk[q] = pk[q - 1] + 0.5 * (dpds[q - 1] + dpds[q]) * ds[q - 1]
        p[order] = pk
        n = nrm[order]
        s = np.stack([-n[:, 1], n[:, 0]], axis=1)
        f = -pk[:, None] * n + nu * (wb[order] - 2.0 * Om)[:, None] * s
        wgt = 0.5 * (ds + np.roll(ds, 1))                            # trapezoid weight of each point
        F = np.sum(f * wgt[:, None], axis=0)
        r = xy - np.asarray(b.center, dtype=np.float64)
        T = np.sum((r[:, 0] * f[:, 1] - r[:, 1] * f[:, 0]) * wgt)
        forces[k] = F[0], F[1], T
    return p, forces


def surface_loads(geom, omega, U, V):
    """Per control point: omega_b, tau = nu omega_b, d omega/dn and the
    relative surface pressure; per body: (F_x, F_y, torque)."""
    wb = boundary_vorticity(geom, U, V)
    grad = vorticity_gradient(geom, extended_vorticity(geom, omega, wb), wb)
    dwdn = grad[:, 0] * geom.c_nx + grad[:, 1] * geom.c_ny
    p, forces = integrate_surface(geom, wb, dwdn)
    return {"omega_b": wb, "tau": geom.grid.nu * wb, "dwdn": dwdn, "p": p, "forces": forces}
