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
* Control-volume force (Noca's momentum formulation for a stationary
  obstacle with no-slip walls and a stationary control volume, Sec. 5.4):
  F = -d/dt int_V u dV - d/dt oint_S x x (n x u) dS + oint_S n . gamma dS,
  gamma = |u|^2/2 I - u u - u (x x omega k) + x.(div T) I - x (div T) + T,
  T = nu (grad u + grad u^T).  V is the box minus the body; with div u = 0
  and u = 0 on the wall, int_V u dV = oint_S x (u.n) dS, so every term is an
  integral over the box surface S.  The box is a rectangle of grid lines
  through nodes, integrated by the trapezoid rule along its edges; the
  derivatives are centred differences of the node values, and
  div T = nu lap u = nu (-d_y omega, d_x omega).  control_volume_terms returns
  the two instantaneous parts, S_t = oint_S [x (u.n) + x x (n x u)] dS and
  S_gamma = oint_S n . gamma dS, so that F = S_gamma - d S_t / dt.
* Control-volume moment (the paper's analogue of Noca's formulation for the
  moment, Sec. 5.4 and its appendix): M = -d/dt int_V x x u dV
  + d/dt oint_S |x|^2/2 n x u dS + oint_S lambda(n) dS, with
  lambda(n) = |u|^2/2 (x x n) - (x x u)(u.n) - |x|^2/2 n x (u x omega k)
  + |x|^2/2 (div T) x n + x x (T.n).  Since div(|x|^2/2 (u_y, -u_x)) =
  x x u + |x|^2/2 omega and u = 0 on the walls, the two time-derivative terms
  together are d/dt int_V |x|^2/2 omega dV over the box minus the body, so
  M = d I / dt + S_lambda with I = int_V |x|^2/2 omega dV.  I is a sum over
  the box's nodes of omega times the fluid area of each node's dual cell
  (h x h about the node; half or a quarter of it on the box's edges and
  corners), omega extended to the ghost nodes by E3b; the fluid area of a
  cell cut by a body is the cell minus its intersection with the polygon of
  the body's boundary points (the boundary points of an enclosure bound the
  fluid instead).
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


def control_volume_terms(grid, omega, U, V, box, origin=(0.0, 0.0)):
    """(S_t, S_gamma) of the control-volume force on the box of nodes
    i0..i1 x j0..j1 (box = (i0, i1, j0, j1)); U, V: velocity with the one-node
    ring, [ny+2][nx+2]; omega: [ny][nx]; x measured from `origin`."""
    i0, i1, j0, j1 = box
    h, nu = grid.h, grid.nu
    St = np.zeros(2)
    Sg = np.zeros(2)

    def node_terms(i, j, n, wgt):
        x = grid.x0 + i * h - origin[0]
        y = grid.y0 + j * h - origin[1]
        u, v = U[j + 1, i + 1], V[j + 1, i + 1]
        w = omega[j, i]
        ux_x = (U[j + 1, i + 2] - U[j + 1, i]) / (2 * h)
        ux_y = (U[j + 2, i + 1] - U[j, i + 1]) / (2 * h)
        uy_x = (V[j + 1, i + 2] - V[j + 1, i]) / (2 * h)
        uy_y = (V[j + 2, i + 1] - V[j, i + 1]) / (2 * h)
        w_x = (omega[j, i + 1] - omega[j, i - 1]) / (2 * h)
        w_y = (omega[j + 1, i] - omega[j - 1, i]) / (2 * h)
        T = nu * np.array([[2 * ux_x, ux_y + uy_x], [ux_y + uy_x, 2 * uy_y]])
        divT = nu * np.array([-w_y, w_x])
        xv = np.array([x, y])
        uv = np.array([u, v])
        un = uv @ n
        nxu = n[0] * v - n[1] * u                      # k-component of n x u
        St[:] += wgt * (xv * un + nxu * np.array([y, -x]))
        g = (0.5 * (u * u + v * v) * n - un * uv - un * w * np.array([y, -x])
             + (xv @ divT) * n - (n @ xv) * divT + T @ n)
        Sg[:] += wgt * g

    edges = [((i0, j0), (1, 0), i1 - i0, np.array([0.0, -1.0])),   # bottom
             ((i1, j0), (0, 1), j1 - j0, np.array([1.0, 0.0])),    # right
             ((i0, j1), (1, 0), i1 - i0, np.array([0.0, 1.0])),    # top
             ((i0, j0), (0, 1), j1 - j0, np.array([-1.0, 0.0]))]   # left
    for (a, b), (di, dj), m, n in edges:
        for k in range(m + 1):
            wgt = h * (0.5 if k in (0, m) else 1.0)
            node_terms(a + k * di, b + k * dj, n, wgt)
    return St, Sg


def cv_moment_surface(grid, omega, U, V, box, origin=(0.0, 0.0)):
    """S_lambda = oint_S lambda(n) dS on the box (the same box, nodes, weights
    and differences as control_volume_terms)."""
    i0, i1, j0, j1 = box
    h, nu = grid.h, grid.nu
    total = 0.0
    edges = [((i0, j0), (1, 0), i1 - i0, (0.0, -1.0)), ((i1, j0), (0, 1), j1 - j0, (1.0, 0.0)),
             ((i0, j1), (1, 0), i1 - i0, (0.0, 1.0)), ((i0, j0), (0, 1), j1 - j0, (-1.0, 0.0))]
    for (a, b), (di, dj), m, (nx, ny) in edges:
        for k in range(m + 1):
            i, j = a + k * di, b + k * dj
            wgt = h * (0.5 if k in (0, m) else 1.0)
            x = grid.x0 + i * h - origin[0]
            y = grid.y0 + j * h - origin[1]
            u, v = U[j + 1, i + 1], V[j + 1, i + 1]
            w = omega[j, i]
            ux_x = (U[j + 1, i + 2] - U[j + 1, i]) / (2 * h)
            ux_y = (U[j + 2, i + 1] - U[j, i + 1]) / (2 * h)
            uy_x = (V[j + 1, i + 2] - V[j + 1, i]) / (2 * h)
            uy_y = (V[j + 2, i + 1] - V[j, i + 1]) / (2 * h)
            w_x = (omega[j, i + 1] - omega[j, i - 1]) / (2 * h)
            w_y = (omega[j + 1, i] - omega[j - 1, i]) / (2 * h)
            Tn = (nu * (2 * ux_x * nx + (ux_y + uy_x) * ny), nu * ((ux_y + uy_x) * nx + 2 * uy_y * ny))
            divT = (-nu * w_y, nu * w_x)
            r2 = 0.5 * (x * x + y * y)
            un = u * nx + v * ny
            lam = (0.5 * (u * u + v * v) * (x * ny - y * nx)      # |u|^2/2 (x x n)
                   - (x * v - y * u) * un                         # -(x x u)(u.n)
                   + r2 * w * un                                  # -|x|^2/2 n x (u x omega k)
                   + r2 * (divT[0] * ny - divT[1] * nx)           # |x|^2/2 (div T) x n
                   + (x * Tn[1] - y * Tn[0]))                     # x x (T.n)
            total += wgt * lam
    return total


def _clip_area(poly, x0, x1, y0, y1):
    """Area of the polygon (closed, either orientation) inside the rectangle
    [x0, x1] x [y0, y1]: clipped against the four half-planes in turn."""
    pts = [tuple(p) for p in poly]
    for axis, bound, keep_below in ((0, x0, False), (0, x1, True), (1, y0, False), (1, y1, True)):
        out = []
        n = len(pts)
        for q in range(n):
            a, b = pts[q - 1], pts[q]
            ina = (a[axis] <= bound) if keep_below else (a[axis] >= bound)
            inb = (b[axis] <= bound) if keep_below else (b[axis] >= bound)
            if inb:
                if not ina:
                    out.append(_cut(a, b, axis, bound))
                out.append(b)
            elif ina:
                out.append(_cut(a, b, axis, bound))
        pts = out
        if not pts:
            return 0.0
    xs = np.array([p[0] for p in pts])
    ys = np.array([p[1] for p in pts])
    return abs(0.5 * np.sum(xs * np.roll(ys, -1) - np.roll(xs, -1) * ys))


def _cut(a, b, axis, bound):
    t = (bound - a[axis]) / (b[axis] - a[axis])
    return (a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1]))


def fluid_weights(geom):
    """[ny][nx] fluid area of each node's dual cell (h x h about the node)."""
    g = geom.grid
    h = g.h
    W = np.where(geom.fluid, h * h, 0.0)
    for b in geom.bodies:
        P = np.asarray(b.points, dtype=np.float64)
        # the dual cells the boundary passes through: those holding points
        # sampled along every edge of the polygon (edges are shorter than h)
        cells = set()
        for q in range(len(P)):
            a, c = P[q - 1], P[q]
            for s in np.linspace(0.0, 1.0, 5):
                x, y = a + s * (c - a)
                cells.add((int(np.floor((x - g.x0) / h + 0.5)), int(np.floor((y - g.y0) / h + 0.5))))
        for (i, j) in cells:
            if not (0 <= i < g.nx and 0 <= j < g.ny):
                continue
            xc, yc = g.x0 + i * h, g.y0 + j * h
            inside = _clip_area(P, xc - 0.5 * h, xc + 0.5 * h, yc - 0.5 * h, yc + 0.5 * h)
            W[j, i] = inside if b.is_enclosure else h * h - inside
    return W


def cv_moment_volume(geom, omega_ext, W, box, origin=(0.0, 0.0)):
    """I = int |x|^2/2 omega over the box minus the bodies: node values times
    the fluid area of their dual cells, halved on the box's edges."""
    i0, i1, j0, j1 = box
    g = geom.grid
    total = 0.0
    for j in range(j0, j1 + 1):
        for i in range(i0, i1 + 1):
            f = (0.5 if i in (i0, i1) else 1.0) * (0.5 if j in (j0, j1) else 1.0)
            x = g.x0 + i * g.h - origin[0]
            y = g.y0 + j * g.h - origin[1]
            total += f * W[j, i] * 0.5 * (x * x + y * y) * omega_ext[j, i]
    return total


def cv_moment_terms(geom, omega, U, V, box, origin=(0.0, 0.0), W=None):
    """(I, S_lambda) of the control-volume moment, with omega extended by E3b
    (with omega_b) at the ghost nodes and zero at the other solid nodes."""
    wb = boundary_vorticity(geom, U, V)
    ext = np.where(geom.fluid, np.asarray(omega, dtype=np.float64), 0.0)
    _, e3b, _ = vorticity_extensions(geom, omega, wb)
    ext[geom.g_j, geom.g_i] = e3b
    if W is None:
        W = fluid_weights(geom)
    return (cv_moment_volume(geom, ext, W, box, origin),
            cv_moment_surface(geom.grid, omega, U, V, box, origin))
