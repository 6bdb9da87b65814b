"""Immersed geometry: from boundary point sets to the IIM sets and stencils.

Follows Sec. 2.1 (extrapolation form of the explicit-jump IIM: a ghost value
is the Lagrange interpolating polynomial through a boundary value and the
fluid nodes behind it, evaluated one node past the boundary; the node next
to the boundary is left out of stencils that use the boundary value),
Sec. 2.2 (control points C = grid-line / boundary intersections, affected
points A+ (fluid) and A- (solid) adjacent to a control point, averaging of
the one-dimensional extrapolations over directions, control points without
enough fluid neighbours ignored) and App. A (intersections and normals).

Readings taken where the paper is silent (the boundary is given as points
rather than a level set):
  * each body is the closed periodic cubic spline through its points with a
    uniform parameter (knot k at t = k);
  * crossings of a grid line are the real roots of the spline cubic on each
    segment, found by bisection on monotone pieces;
  * a node is inside a body when an odd number of that body's crossings lie
    before it on its grid line (checked along both axes);
  * solid = inside an obstacle or outside an enclosing wall;
  * on a fluid-solid edge the control point is the crossing nearest the
    fluid node; theta = distance(fluid node, control point) / h in (0, 1];
  * "fourth order" extrapolation = cubic through 4 points, "third order" =
    quadratic through 3 points (error O(h^(n+1)) for degree n);
  * a direction is valid when the needed nodes behind the fluid node are all
    fluid; the ghost value is the unweighted mean over valid directions.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class GeometryError(ValueError):
    pass


FLUID, GHOST, SOLID = 0, 1, 2


# ----------------------------------------------------------------------------
# spline
# ----------------------------------------------------------------------------

def periodic_spline(points):
    """Per-segment power-basis coefficients (a, b, c, d), each shaped (P, 2), of
    the periodic cubic spline X(k + s) = a + b s + c s^2 + d s^3, s in [0, 1]."""
    Q = np.asarray(points, dtype=np.float64)
    P = Q.shape[0]
    if P < 4:
        raise GeometryError("a body needs at least 4 boundary points")
    col = np.zeros(P)
    col[0], col[1], col[-1] = 4.0, 1.0, 1.0
    rhs = 6.0 * (np.roll(Q, -1, axis=0) - 2.0 * Q + np.roll(Q, 1, axis=0))
    M = np.stack([sla.solve_circulant(col, rhs[:, 0]), sla.solve_circulant(col, rhs[:, 1])], axis=1)
    M1 = np.roll(M, -1, axis=0)
    Q1 = np.roll(Q, -1, axis=0)
    a = Q.copy()
    b = (Q1 - Q) - (2.0 * M + M1) / 6.0
    c = 0.5 * M
    d = (M1 - M) / 6.0
    return a, b, c, d


def _cubic(coef, s):
    a, b, c, d = coef
    return a + s * (b + s * (c + s * d))


def _cubic_d(coef, s):
    _, b, c, d = coef
    return b + s * (2.0 * c + 3.0 * s * d)


def line_crossings(a, b, c, d, axis, levels):
    """Crossings of the spline with the lines {coordinate[axis] = level}.

    Returns (seg, s, line) arrays: segment index, parameter s in (0, 1) and the
    index into `levels` of each crossing."""
    P = a.shape[0]
    A, B, C, D = a[:, axis], b[:, axis], c[:, axis], d[:, axis]
    # critical points of the cubic on (0, 1): B + 2 C s + 3 D s^2 = 0
    crit = np.full((P, 2), np.nan)
    for k in range(P):
        r = np.roots([3.0 * D[k], 2.0 * C[k], B[k]]) if (abs(D[k]) + abs(C[k])) > 0 else []
        rr = [x.real for x in np.atleast_1d(r) if abs(x.imag) < 1e-14 and 0.0 < x.real < 1.0]
        for q, x in enumerate(sorted(rr)[:2]):
            crit[k, q] = x
    segs, sa, sb = [], [], []
    for k in range(P):
        pts = [0.0] + [x for x in crit[k] if not np.isnan(x)] + [1.0]
        for q in range(len(pts) - 1):
            segs.append(k)
            sa.append(pts[q])
            sb.append(pts[q + 1])
    segs = np.array(segs)
    sa = np.array(sa)
    sb = np.array(sb)
    ya = A[segs] + sa * (B[segs] + sa * (C[segs] + sa * D[segs]))
    yb = A[segs] + sb * (B[segs] + sb * (C[segs] + sb * D[segs]))
    lo = np.minimum(ya, yb)
    hi = np.maximum(ya, yb)
    levels = np.asarray(levels)
    out_seg, out_lo, out_hi, out_line, out_inc = [], [], [], [], []
    i0 = np.searchsorted(levels, lo, side="left")
    i1 = np.searchsorted(levels, hi, side="right")
    for p in range(segs.size):
        for L in range(i0[p], i1[p]):
            Y = levels[L]
            fa, fb = ya[p] - Y, yb[p] - Y
            if fa == 0.0 or fb == 0.0:
                raise GeometryError("a boundary curve touches grid line %d exactly" % L)
            if (fa < 0) != (fb < 0):
                out_seg.append(segs[p])
                out_lo.append(sa[p])
                out_hi.append(sb[p])
                out_line.append(L)
                out_inc.append(fb > fa)
    if not out_seg:
        return np.zeros(0, int), np.zeros(0), np.zeros(0, int)
    seg = np.array(out_seg)
    lo = np.array(out_lo)
    hi = np.array(out_hi)
    line = np.array(out_line)
    inc = np.array(out_inc)
    Y = levels[line]
    for _ in range(80):                      # bisection to full precision
        mid = 0.5 * (lo + hi)
        f = A[seg] + mid * (B[seg] + mid * (C[seg] + mid * D[seg])) - Y
        up = (f > 0) == inc                  # root lies below mid
        hi = np.where(up, mid, hi)
        lo = np.where(up, lo, mid)
    s = 0.5 * (lo + hi)
    if np.any(s < 1e-12) or np.any(s > 1.0 - 1e-12):
        raise GeometryError("a spline knot lies on a grid line")
    for k in range(P):                       # tangency: root at a critical point
        for q in range(2):
            if not np.isnan(crit[k, q]):
                m = seg == k
                if np.any(np.abs(s[m] - crit[k, q]) < 1e-9):
                    raise GeometryError("a boundary curve is tangent to a grid line")
    return seg, s, line


# ----------------------------------------------------------------------------
# Lagrange weights
# ----------------------------------------------------------------------------

def lagrange_weights(nodes, x):
    """Weights w_k with p(x) = sum_k w_k f(nodes_k) for the interpolating polynomial."""
    nodes = np.asarray(nodes, dtype=np.float64)
    w = np.ones(nodes.size)
    for k in range(nodes.size):
        for l in range(nodes.size):
            if l != k:
                w[k] *= (x - nodes[l]) / (nodes[k] - nodes[l])
    return w


def lagrange_deriv_weights(nodes, x):
    """Weights of p'(x) for the interpolating polynomial through `nodes`."""
    nodes = np.asarray(nodes, dtype=np.float64)
    n = nodes.size
    w = np.zeros(n)
    for k in range(n):
        denom = 1.0
        for l in range(n):
            if l != k:
                denom *= nodes[k] - nodes[l]
        tot = 0.0
        for m in range(n):
            if m == k:
                continue
            prod = 1.0
            for l in range(n):
                if l != k and l != m:
                    prod *= x - nodes[l]
            tot += prod
        w[k] = tot / denom
    return w


# stencil kinds: (number of fluid nodes behind, uses the boundary value)
KIND_4B = "4b"     # cubic through {c, x_i-1, x_i-2, x_i-3}
KIND_3B = "3b"     # quadratic through {c, x_i-1, x_i-2}
KIND_3N = "3n"     # quadratic through {x_i, x_i-1, x_i-2}  (no boundary value)


def extrapolation_weights(kind, theta):
    """(w_bc, w_nodes) for extrapolation to the ghost at +1; fluid node x_i at 0,
    x_{i-m} at -m, control point at theta."""
    if kind == KIND_4B:
        w = lagrange_weights([theta, -1.0, -2.0, -3.0], 1.0)
        return w[0], w[1:]
    if kind == KIND_3B:
        w = lagrange_weights([theta, -1.0, -2.0], 1.0)
        return w[0], w[1:]
    if kind == KIND_3N:
        w = lagrange_weights([0.0, -1.0, -2.0], 1.0)
        return 0.0, w
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

class Geometry:
    """All static IIM data for one grid and one set of bodies."""

    def __init__(self, grid, bodies, rect_margin=3, bc_override=None):
        """bc_override: optional (psi_fn, u_fn) giving the boundary stream
        function and velocity at arbitrary points (replaces rigid motion)."""
        self.grid = grid
        self._bc_override = bc_override
        self.bodies = bodies
        nx, ny, h = grid.nx, grid.ny, grid.h
        self.nx, self.ny, self.h = nx, ny, h
        self.x = grid.x0 + h * np.arange(nx)
        self.y = grid.y0 + h * np.arange(ny)
        nb = len(bodies)
        if sum(1 for b in bodies if b.is_enclosure) > 1:
            raise GeometryError("at most one enclosing wall")
        self.splines = []
        inside = np.zeros((nb, ny, nx), dtype=bool)
        # crossings per body: dict axis -> (seg, s, line, pos, normal)
        self.crossings = []
        for k, b in enumerate(bodies):
            pts = np.asarray(b.points, dtype=np.float64)
            area = 0.5 * np.sum(pts[:, 0] * np.roll(pts[:, 1], -1) - np.roll(pts[:, 0], -1) * pts[:, 1])
            if b.is_enclosure and area >= 0:
                raise GeometryError("body %d: an enclosing wall must be ordered clockwise" % k)
            if (not b.is_enclosure) and area <= 0:
                raise GeometryError("body %d: an obstacle must be ordered counter-clockwise" % k)
            margin = 3 * h
            if (pts[:, 0].min() < self.x[0] + margin or pts[:, 0].max() > self.x[-1] - margin
                    or pts[:, 1].min() < self.y[0] + margin or pts[:, 1].max() > self.y[-1] - margin):
                raise GeometryError("body %d is too close to the grid edge" % k)
            coef = periodic_spline(pts)
            self.splines.append(coef)
            rec = {}
            for axis, levels, other in ((1, self.y, self.x), (0, self.x, self.y)):
                # axis=1: horizontal lines y = y_j (crossing position is x)
                seg, s, line = line_crossings(*coef, axis=axis, levels=levels)
                pos = _cubic(tuple(cc[seg] for cc in coef), s[:, None])
                tan = _cubic_d(tuple(cc[seg] for cc in coef), s[:, None])
                nrm = np.stack([tan[:, 1], -tan[:, 0]], axis=1)
                nrm /= np.linalg.norm(nrm, axis=1)[:, None]
                along = pos[:, 1 - axis]          # coordinate along the line
                rec[axis] = (seg, s, line, along, nrm, pos)
                # parity classification along these lines
                for L in np.unique(line):
                    xs = np.sort(along[line == L])
                    cnt = np.searchsorted(xs, other, side="left")
                    if np.any(np.isin(other, xs)):
                        raise GeometryError("a node lies exactly on a boundary")
                    odd = (cnt % 2) == 1
                    if axis == 1:
                        if "h" not in rec:
                            rec["h"] = np.zeros((ny, nx), dtype=bool)
                        rec["h"][L, :] = odd
                    else:
                        if "v" not in rec:
                            rec["v"] = np.zeros((ny, nx), dtype=bool)
                        rec["v"][:, L] = odd
            hmask = rec.get("h", np.zeros((ny, nx), dtype=bool))
            vmask = rec.get("v", np.zeros((ny, nx), dtype=bool))
            if np.any(hmask != vmask):
                raise GeometryError("body %d: horizontal and vertical classification disagree" % k)
            inside[k] = hmask
            self.crossings.append(rec)
        solid = np.zeros((ny, nx), dtype=bool)
        owner = np.full((ny, nx), -1, dtype=int)
        for k, b in enumerate(bodies):
            region = ~inside[k] if b.is_enclosure else inside[k]
            if np.any(solid & region):
                raise GeometryError("bodies %d overlap another body" % k)
            solid |= region
            owner[region] = k
        self.solid = solid
        self.fluid = ~solid
        self.solid_owner = owner
        self._build_control_points()
        self._build_sets()
        self._build_ghost_operators()
        self._build_poisson_operators()
        self._build_rects(rect_margin)
        self._check_vorticity_bc_stencils()

    # ------------------------------------------------------------------
    def _build_control_points(self):
        nx, ny, h = self.nx, self.ny, self.h
        solid = self.solid
        recs = []  # (axis, i_f, j_f, sigma, theta, body, xc, yc, nx_, ny_, seg, s)
        # gather all crossings per (axis, line) over bodies
        for axis in (1, 0):
            allc = []
            for k, rec in enumerate(self.crossings):
                seg, s, line, along, nrm, pos = rec[axis]
                for q in range(line.size):
                    allc.append((line[q], along[q], k, nrm[q, 0], nrm[q, 1], pos[q, 0], pos[q, 1], seg[q], s[q]))
            if not allc:
                continue
            arr = np.array(allc, dtype=np.float64)
            lines = arr[:, 0].astype(int)
            for L in np.unique(lines):
                sel = arr[lines == L]
                order = np.argsort(sel[:, 1])
                sel = sel[order]
                pos_along = sel[:, 1]
                if axis == 1:      # horizontal line j = L, nodes along x
                    nodes = self.x
                    cls = solid[L, :]
                else:
                    nodes = self.y
                    cls = solid[:, L]
                n_along = nodes.size
                for a in range(n_along - 1):
                    if cls[a] == cls[a + 1]:
                        continue
                    lo, hi = nodes[a], nodes[a + 1]
                    m = (pos_along > lo) & (pos_along < hi)
                    cand = sel[m]
                    if cand.shape[0] % 2 == 0:
                        raise GeometryError("inconsistent crossings on a fluid-solid edge")
                    if np.unique(cand[:, 2]).size != 1:
                        raise GeometryError("two bodies cross the same grid edge")
                    if not cls[a]:           # fluid at a, ghost at a+1
                        f_idx, sigma = a, +1
                        q = np.argmin(cand[:, 1] - lo)
                        theta = (cand[q, 1] - lo) / h
                    else:                    # fluid at a+1, ghost at a
                        f_idx, sigma = a + 1, -1
                        q = np.argmin(hi - cand[:, 1])
                        theta = (hi - cand[q, 1]) / h
                    c = cand[q]
                    if axis == 1:
                        i_f, j_f, ax = f_idx, L, 0
                    else:
                        i_f, j_f, ax = L, f_idx, 1
                    recs.append((ax, i_f, j_f, sigma, theta, int(c[2]), c[5], c[6], c[3], c[4], c[7], c[8]))
        # canonical order: by ghost node linear index, then axis, then sigma
        def ghost_lin(r):
            ax, i_f, j_f, sigma = r[0], r[1], r[2], r[3]
            gi, gj = (i_f + sigma, j_f) if ax == 0 else (i_f, j_f + sigma)
            return (gj * nx + gi, ax, sigma)
        recs.sort(key=ghost_lin)
        R = np.array(recs, dtype=np.float64).reshape(-1, 12)
        self.nc = R.shape[0]
        self.c_axis = R[:, 0].astype(int)        # 0: along x (horizontal line), 1: along y
        self.c_if = R[:, 1].astype(int)
        self.c_jf = R[:, 2].astype(int)
        self.c_sigma = R[:, 3].astype(int)
        self.c_theta = R[:, 4]
        self.c_body = R[:, 5].astype(int)
        self.c_x = R[:, 6]
        self.c_y = R[:, 7]
        self.c_nx = R[:, 8]
        self.c_ny = R[:, 9]
        self.c_seg = R[:, 10].astype(int)      # spline segment and parameter of the crossing
        self.c_s = R[:, 11]
        self.c_ig = np.where(self.c_axis == 0, self.c_if + self.c_sigma, self.c_if)
        self.c_jg = np.where(self.c_axis == 1, self.c_jf + self.c_sigma, self.c_jf)
        if np.any(self.c_theta <= 0) or np.any(self.c_theta > 1):
            raise GeometryError("control point outside its grid edge")
        # boundary data at the control points: rigid motion, or prescribed
        # samples (u_x, u_y, psi_b) at the boundary points interpolated by
        # periodic cubic splines in the curve's parameter (the same
        # construction as the curve itself), evaluated at each crossing
        ub = np.zeros((self.nc, 2))
        psib = np.zeros(self.nc)
        for k, b in enumerate(self.bodies):
            m = self.c_body == k
            smp = getattr(b, "bc_samples", None)
            if smp is not None:
                smp = np.asarray(smp, dtype=np.float64)
                cu = periodic_spline(smp[:, 0:2])
                cp = periodic_spline(np.stack([smp[:, 2], np.zeros(smp.shape[0])], axis=1))
                seg, s = self.c_seg[m], self.c_s[m][:, None]
                ub[m] = _cubic(tuple(cc[seg] for cc in cu), s)
                psib[m] = _cubic(tuple(cc[seg] for cc in cp), s)[:, 0]
                continue
            ub[m], psib[m] = self._rigid_data(m, b.center, b.u_rigid, b.omega_rigid)
        if self._bc_override is not None:
            psi_fn, u_fn = self._bc_override
            psib = np.asarray(psi_fn(self.c_x, self.c_y), dtype=np.float64)
            ub = np.stack(u_fn(self.c_x, self.c_y), axis=1).astype(np.float64)
        self.c_ub = ub
        self.c_psib = psib

    def _rigid_data(self, m, center, u_rigid, omega):
        """u_b and psi_b of the rigid motion u_rigid + omega k x (x - center)
        at the control points selected by m."""
        U = np.asarray(u_rigid, dtype=np.float64)
        Om = float(omega)
        dx, dy = self.c_x[m] - center[0], self.c_y[m] - center[1]
        ub = np.stack([U[0] - Om * dy, U[1] + Om * dx], axis=1)
        # stream function of the rigid motion (u = d_y psi, v = -d_x psi)
        psib = U[0] * self.c_y[m] - U[1] * self.c_x[m] - 0.5 * Om * (dx * dx + dy * dy)
        return ub, psib

    def set_rigid_motion(self, motions):
        """Boundary data of a time-dependent rigid motion: motions[k] =
        (u_x, u_y, omega) of body k at the current time (bodies with boundary
        samples are not allowed)."""
        for k, b in enumerate(self.bodies):
            if getattr(b, "bc_samples", None) is not None:
                raise ValueError("body %d has prescribed boundary samples" % k)
            m = self.c_body == k
            ux, uy, om = motions[k]
            self.c_ub[m], self.c_psib[m] = self._rigid_data(m, b.center, (ux, uy), om)

    # ------------------------------------------------------------------
    def _build_sets(self):
        nx, ny = self.nx, self.ny
        solid = self.solid
        pad = np.zeros((ny + 2, nx + 2), dtype=bool)
        pad[1:-1, 1:-1] = self.fluid
        fluid_nb = pad[1:-1, 2:] | pad[1:-1, :-2] | pad[2:, 1:-1] | pad[:-2, 1:-1]
        pad[:] = False
        pad[1:-1, 1:-1] = solid
        solid_nb = pad[1:-1, 2:] | pad[1:-1, :-2] | pad[2:, 1:-1] | pad[:-2, 1:-1]
        self.ghost_mask = solid & fluid_nb          # A-
        self.aplus_mask = self.fluid & solid_nb     # A+
        cls = np.full((ny, nx), SOLID, dtype=int)
        cls[self.fluid] = FLUID
        cls[self.ghost_mask] = GHOST
        self.cls = cls
        # ghost numbering (row-major)
        gj, gi = np.nonzero(self.ghost_mask)
        self.ng = gi.size
        self.g_i, self.g_j = gi, gj
        self.ghost_id = np.full((ny, nx), -1, dtype=int)
        self.ghost_id[gj, gi] = np.arange(self.ng)
        # incident control points of each ghost
        self.g_ctrl = [[] for _ in range(self.ng)]
        for c in range(self.nc):
            g = self.ghost_id[self.c_jg[c], self.c_ig[c]]
            if g < 0:
                raise GeometryError("control point without a ghost")
            self.g_ctrl[g].append(c)
        # affected points A = A+ U A-, row-major order
        aj, ai = np.nonzero(self.ghost_mask | self.aplus_mask)
        self.na = ai.size
        self.a_i, self.a_j = ai, aj
        self.a_lin = aj * nx + ai
        self.a_is_ghost = self.ghost_mask[aj, ai]
        self.a_id = np.full((ny, nx), -1, dtype=int)
        self.a_id[aj, ai] = np.arange(self.na)
        # body of every affected point
        body = np.full(self.na, -1, dtype=int)
        for c in range(self.nc):
            for (i, j) in ((self.c_if[c], self.c_jf[c]), (self.c_ig[c], self.c_jg[c])):
                a = self.a_id[j, i]
                if body[a] >= 0 and body[a] != self.c_body[c]:
                    raise GeometryError("an affected point is adjacent to two bodies")
                body[a] = self.c_body[c]
        if np.any(body < 0):
            raise GeometryError("affected point without a control point")
        self.a_body = body

    # ------------------------------------------------------------------
    def _in_grid(self, i, j):
        return 0 <= i < self.nx and 0 <= j < self.ny

    def _direction_nodes(self, c, count):
        """Fluid-side nodes x_i, x_{i-1}, ..., x_{i-count+1} of control point c."""
        ax, s = self.c_axis[c], self.c_sigma[c]
        out = []
        for m in range(count):
            if ax == 0:
                out.append((self.c_if[c] - m * s, self.c_jf[c]))
            else:
                out.append((self.c_if[c], self.c_jf[c] - m * s))
        return out

    def _valid(self, c, count):
        for (i, j) in self._direction_nodes(c, count):
            if not self._in_grid(i, j) or not self.fluid[j, i]:
                return False
        return True

    def _ghost_operator(self, kind):
        """Sparse (ng x N) node weights and (ng x nc) boundary weights."""
        N = self.nx * self.ny
        count = 4 if kind == KIND_4B else 3
        rows_f, cols_f, vals_f = [], [], []
        rows_b, cols_b, vals_b = [], [], []
        nvalid = np.zeros(self.ng, dtype=int)
        for g in range(self.ng):
            valid = [c for c in self.g_ctrl[g] if self._valid(c, count)]
            nvalid[g] = len(valid)
            if not valid:
                raise GeometryError("ghost node (%d, %d) has no valid %s stencil"
                                    % (self.g_i[g], self.g_j[g], kind))
            inv = 1.0 / len(valid)
            for c in valid:
                wb, wn = extrapolation_weights(kind, self.c_theta[c])
                nodes = self._direction_nodes(c, count)
                if kind == KIND_3N:
                    use = nodes[:3]            # x_i, x_{i-1}, x_{i-2}
                else:
                    use = nodes[1:count]       # x_{i-1}, ... (x_i excluded)
                    rows_b.append(g)
                    cols_b.append(c)
                    vals_b.append(inv * wb)
                for (i, j), w in zip(use, wn):
                    rows_f.append(g)
                    cols_f.append(j * self.nx + i)
                    vals_f.append(inv * w)
        Ef = sp.csr_matrix((vals_f, (rows_f, cols_f)), shape=(self.ng, N))
        Eb = sp.csr_matrix((vals_b, (rows_b, cols_b)), shape=(self.ng, self.nc))
        return Ef, Eb, nvalid

    def _build_ghost_operators(self):
        self.E4b_f, self.E4b_b, self.n4 = self._ghost_operator(KIND_4B)
        self.E3b_f, self.E3b_b, self.n3 = self._ghost_operator(KIND_3B)
        self.E3n_f, _, _ = self._ghost_operator(KIND_3N)

    # ------------------------------------------------------------------
    def _build_poisson_operators(self):
        """gamma = A psi + B psi_b (Sec. 4.2, corrections of the 5-point stencil).

        p in A+ : gamma_p = -h^-2 * sum over solid neighbours q of ghost_q(psi, psi_b)
        q in A- : gamma_q = +h^-2 * sum over fluid neighbours r of psi_r
        """
        nx, ny, h = self.nx, self.ny, self.h
        N = nx * ny
        inv_h2 = 1.0 / (h * h)
        Arows = []
        Brows = []
        for a in range(self.na):
            i, j = self.a_i[a], self.a_j[a]
            ra = sp.csr_matrix((1, N))
            rb = sp.csr_matrix((1, self.nc))
            if self.a_is_ghost[a]:
                cols = [(i + di, j + dj) for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1))
                        if self._in_grid(i + di, j + dj) and self.fluid[j + dj, i + di]]
                ra = sp.csr_matrix((np.full(len(cols), inv_h2),
                                    (np.zeros(len(cols), int), [jj * nx + ii for ii, jj in cols])),
                                   shape=(1, N))
            else:
                for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    ii, jj = i + di, j + dj
                    if self._in_grid(ii, jj) and self.solid[jj, ii]:
                        g = self.ghost_id[jj, ii]
                        ra = ra - inv_h2 * self.E4b_f[g]
                        rb = rb - inv_h2 * self.E4b_b[g]
            Arows.append(ra)
            Brows.append(rb)
        # (no affected points: no bodies; empty operators)
        self.Aop = sp.vstack(Arows).tocsr() if Arows else sp.csr_matrix((0, N))
        self.Bop = sp.vstack(Brows).tocsr() if Brows else sp.csr_matrix((0, self.nc))
        # E_a: V_A -> V_G inclusion
        self.Ea = sp.csr_matrix((np.ones(self.na), (self.a_lin, np.arange(self.na))),
                                shape=(N, self.na))

    # ------------------------------------------------------------------
    def _build_rects(self, margin):
        """Bounding regions R_k (Sec. 4.2 / 5.1): default = bounding box of the
        body's affected points grown by `margin` nodes."""
        nx, ny = self.nx, self.ny
        self.circ_bodies = [k for k, b in enumerate(self.bodies) if not b.is_enclosure]
        self.rects = []
        for k in self.circ_bodies:
            b = self.bodies[k]
            m = self.a_body == k
            if b.rect is not None:
                i0, i1, j0, j1 = b.rect
            else:
                i0, i1 = self.a_i[m].min() - margin, self.a_i[m].max() + margin
                j0, j1 = self.a_j[m].min() - margin, self.a_j[m].max() + margin
            if i0 < 2 or j0 < 2 or i1 > nx - 3 or j1 > ny - 3:
                raise GeometryError("R_%d leaves the grid" % k)
            if np.any((self.a_i[m] < i0) | (self.a_i[m] > i1) | (self.a_j[m] < j0) | (self.a_j[m] > j1)):
                raise GeometryError("R_%d does not contain its body" % k)
            inr = (self.a_i >= i0) & (self.a_i <= i1) & (self.a_j >= j0) & (self.a_j <= j1)
            if np.any(inr & ~m):
                raise GeometryError("R_%d contains another body" % k)
            # frame of width 2 on both sides of dR_k must be plain fluid
            fr = np.zeros((ny, nx), dtype=bool)
            fr[j0 - 2:j1 + 3, i0 - 2:i1 + 3] = True
            fr[j0 + 2:j1 - 1, i0 + 2:i1 - 1] = False
            if np.any(fr & ~self.fluid) or np.any(fr & self.aplus_mask):
                raise GeometryError("the faces of R_%d are too close to a boundary" % k)
            self.rects.append((int(i0), int(i1), int(j0), int(j1)))
        self.nbc = len(self.circ_bodies)

    # ------------------------------------------------------------------
    def _has_value(self, i, j):
        """A node carries a (possibly extended) velocity: fluid or A-."""
        return self._in_grid(i, j) and self.cls[j, i] != SOLID

    def vorticity_bc_stencil(self, c):
        """Second-order stencil of the boundary vorticity at control point c
        (Sec. 5.3): omega_b = d_x u_y - d_y u_x of the extended velocity.

        Reading of the stencil figure (only its caption survives): for a control
        point on a horizontal grid line between fluid node x_i and ghost
        x_{i+s}, d_x u_y is the derivative at x_c of the quadratic through u_y
        at x_{i-s}, x_i, x_{i+s}.  d_y u_x is the one-sided three-point
        derivative tau(-3 u_x^b + 4 U_1 - U_2)/(2h) into the fluid
        (tau = sign n_y), where U_r is u_x at (x_c, y_j + r tau h) interpolated
        by a quadratic along that row through x_{i-s}, x_i, x_{i+s}, or, when
        one of those carries no value, through x_{i-2s}, x_{i-s}, x_i.
        Vertical lines: swap the axes.

        Returns (terms, bc_terms): terms = [(i, j, comp, weight)] with comp 0 =
        u_x, 1 = u_y; bc_terms = [(comp, weight)] on u_b(c)."""
        h = self.h
        i, j, s = int(self.c_if[c]), int(self.c_jf[c]), int(self.c_sigma[c])
        xi_c = s * self.c_theta[c]               # control point, fluid node at 0
        terms, bc = [], []
        along_nodes = [-s, 0, s]
        dw = lagrange_deriv_weights(along_nodes, xi_c) / h
        if self.c_axis[c] == 0:
            tau = 1 if self.c_ny[c] >= 0 else -1
            for off, w in zip(along_nodes, dw):            # + d_x u_y
                terms.append((i + off, j, 1, w))
            lin_comp, line_sign = 0, -1.0                   # - d_y u_x
        else:
            tau = 1 if self.c_nx[c] >= 0 else -1
            for off, w in zip(along_nodes, dw):            # - d_y u_x
                terms.append((i, j + off, 0, -w))
            lin_comp, line_sign = 1, 1.0                    # + d_x u_y
        coef = {0: -3.0, 1: 4.0, 2: -1.0}
        scale = line_sign * tau / (2.0 * h)
        bc.append((lin_comp, scale * coef[0]))
        for r in (1, 2):
            chosen = None
            for offs in ([-s, 0, s], [-2 * s, -s, 0]):
                if self.c_axis[c] == 0:
                    pts = [(i + o, j + r * tau) for o in offs]
                else:
                    pts = [(i + r * tau, j + o) for o in offs]
                if all(self._has_value(a, b) for a, b in pts):
                    chosen = (offs, pts)
                    break
            if chosen is None:
                raise GeometryError("control point %d: no vorticity boundary stencil" % c)
            offs, pts = chosen
            wi = lagrange_weights(offs, xi_c)
            for (a, b), w in zip(pts, wi):
                terms.append((a, b, lin_comp, scale * coef[r] * w))
        return terms, bc

    def _check_vorticity_bc_stencils(self):
        self.wb_stencils = [self.vorticity_bc_stencil(c) for c in range(self.nc)]

    # ------------------------------------------------------------------
    def psi_tilde_b(self):
        """Boundary data of the perturbation stream function at the control
        points: psi_b(c) - psi_inf(c), psi_inf = u_inf,x y - u_inf,y x."""
        ux, uy = self.grid.u_inf
        return self.c_psib - (ux * self.c_y - uy * self.c_x)
