"""Vorticity transport with IIM boundary treatment and the Kelvin circulation
ODE (Sec. 3.1-3.2, Sec. 5.1, Sec. 5.3).

Conservative form (eq. of the 2D flux differencing):
    d omega_ij/dt = -[F_{i+1/2,j} - F_{i-1/2,j} + Q_{i+1/2,j} - Q_{i-1/2,j}
                      + F_{i,j+1/2} - F_{i,j-1/2} + Q_{i,j+1/2} - Q_{i,j-1/2}] / h

Advective flux: third-order upwind reconstruction of f = u omega with the
stencils [-1/6, 5/6, 1/3] (left-biased) and [1/3, 5/6, -1/6] (right-biased);
the side is chosen by the sign of the face velocity u_{i+1/2} = (u_i+u_{i+1})/2
(our reading of the printed flux: the bracket of f values, selected by the
sign of the face velocity).  Diffusive flux: Q = -nu (omega_{i+1}-omega_i)/h.

Boundary treatment (Sec. 3.2):
  * diffusion uses omega extended to A- at fourth order with omega_b (E4b);
  * velocity is extended to A- at third order with u_b;
  * omega is extended to A- twice at third order, with omega_b (E3b) and
    without a boundary value (E3n);
  * a face between a fluid node and a ghost always uses the stencil that
    reaches only one node past the boundary (downwind stencil on inflow faces,
    upwind stencil on outflow faces);
  * in any stencil, a ghost on the upwind side of the face takes E3b and a
    ghost on the downwind side takes E3n.

Domain edges in free space (our reading): nodes outside the grid carry
omega = 0 and count as fluid for the choice of stencil; the face velocity
at the outermost face uses the exact ring velocity.  With an outflow plane
at the face x_{nx-1/2} (Sec. 5.2) the two nodes past it carry the mirrored
vorticity and x-velocity instead.  With the periodic exterior (Sec. 4.1)
node i + nx is node i: the two nodes past every edge carry the values,
classes and extensions of the nodes they repeat.

Boundary vorticity omega_b at each control point: the stencil of
Geometry.vorticity_bc_stencil applied to the extended velocity.

Kelvin (Sec. 5.1): dGamma_k/dt = -h sum over the faces of dR_k of (F+Q).n_out.
"""
from __future__ import annotations

import numpy as np

from .geometry import FLUID, GHOST, SOLID

OUTSIDE = 3
W_LEFT = (-1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0)
W_RIGHT = (1.0 / 3.0, 5.0 / 6.0, -1.0 / 6.0)


def boundary_vorticity(geom, U, V):
    """omega_b at every control point from the extended velocity ring arrays."""
    wb = np.zeros(geom.nc)
    for c in range(geom.nc):
        terms, bc = geom.wb_stencils[c]
        tot = 0.0
        for (i, j, comp, w) in terms:
            tot += w * (U[j + 1, i + 1] if comp == 0 else V[j + 1, i + 1])
        for (comp, w) in bc:
            tot += w * geom.c_ub[c, comp]
        wb[c] = tot
    return wb


def vorticity_extensions(geom, omega, wb):
    w = omega.ravel()
    e4b = geom.E4b_f @ w + geom.E4b_b @ wb
    e3b = geom.E3b_f @ w + geom.E3b_b @ wb
    e3n = geom.E3n_f @ w
    return e4b, e3b, e3n


def _padded(geom, omega, U, V, e4b, e3b, e3n):
    nx, ny = geom.nx, geom.ny
    if geom.grid.exterior == "periodic":
        wrap = lambda a: np.pad(a, 2, mode="wrap")
        w = np.where(geom.fluid, omega, 0.0)
        w4, w3b, w3n = np.zeros((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))
        w4[geom.g_j, geom.g_i] = e4b
        w3b[geom.g_j, geom.g_i] = e3b
        w3n[geom.g_j, geom.g_i] = e3n
        return (wrap(geom.cls), wrap(w), wrap(w4), wrap(w3b), wrap(w3n), wrap(U[1:-1, 1:-1]),
                wrap(V[1:-1, 1:-1]))
    P = lambda fill: np.full((ny + 4, nx + 4), fill, dtype=np.float64)
    cls = np.full((ny + 4, nx + 4), OUTSIDE, dtype=int)
    cls[2:-2, 2:-2] = geom.cls
    w = P(0.0)
    w[2:-2, 2:-2] = np.where(geom.fluid, omega, 0.0)
    w4, w3b, w3n = P(0.0), P(0.0), P(0.0)
    gj, gi = geom.g_j + 2, geom.g_i + 2
    w4[gj, gi] = e4b
    w3b[gj, gi] = e3b
    w3n[gj, gi] = e3n
    u, v = P(0.0), P(0.0)
    u[1:-1, 1:-1] = U
    v[1:-1, 1:-1] = V
    if geom.grid.exterior == "outflow":
        # even mirror of the vorticity and of u_x across the face x_{nx-1/2} (Sec. 5.2):
        # node nx+m carries the values of node nx-1-m; the outflow faces use them
        w[2:-2, nx + 2] = w[2:-2, nx + 1]
        w[2:-2, nx + 3] = w[2:-2, nx]
        u[2:-2, nx + 3] = u[2:-2, nx]
    return cls, w, w4, w3b, w3n, u, v


def _face_fluxes(cls, w, w4, w3b, w3n, vel, nu, h):
    """Fluxes on the faces between columns I and I+1 of the padded arrays for
    I = 1 .. ncol-3 (i.e. grid faces i+1/2, i = -1 .. n-1).  Arrays are
    [rows, cols]; the flux direction is along the columns."""
    ncol = cls.shape[1]
    I = np.arange(1, ncol - 2)
    cl, cr = cls[:, I], cls[:, I + 1]
    fl_like = lambda c: (c == FLUID) | (c == OUTSIDE)
    active = (cl == FLUID) | (cr == FLUID)
    uf = 0.5 * (vel[:, I] + vel[:, I + 1])
    up_left = uf >= 0.0
    both = fl_like(cl) & fl_like(cr)
    use_left = np.where(both, up_left, fl_like(cl))
    F = np.zeros(cl.shape)
    for k in range(3):
        # left-biased: columns I-1+k ; right-biased: columns I+k
        col_l = I - 1 + k
        col_r = I + k
        for use, col, wt in ((use_left, col_l, W_LEFT[k]), (~use_left, col_r, W_RIGHT[k])):
            c = cls[:, col]
            on_left = (col <= I)[None, :]
            upwind = np.where(on_left, up_left, ~up_left)
            om = np.where(fl_like(c), w[:, col], np.where(upwind, w3b[:, col], w3n[:, col]))
            if np.any(active & use & (c == SOLID)):
                raise AssertionError("flux stencil reaches a solid interior node")
            F += np.where(use, wt * vel[:, col] * om, 0.0)
    om4 = lambda c, col: np.where(fl_like(c), w[:, col], w4[:, col])
    Q = -nu * (om4(cr, I + 1) - om4(cl, I)) / h
    F = np.where(active, F, 0.0)
    Q = np.where(active, Q, 0.0)
    return F, Q


def rhs(geom, omega, U, V, nu, wb=None):
    """Returns (domega_dt [ny][nx], dGamma_dt [nbc], omega_b [nc], fluxes)."""
    h = geom.h
    if wb is None:
        wb = boundary_vorticity(geom, U, V)
    e4b, e3b, e3n = vorticity_extensions(geom, np.where(geom.fluid, omega, 0.0), wb)
    cls, w, w4, w3b, w3n, u, v = _padded(geom, omega, U, V, e4b, e3b, e3n)
    r = slice(2, -2)
    Fx, Qx = _face_fluxes(cls[r, :], w[r, :], w4[r, :], w3b[r, :], w3n[r, :], u[r, :], nu, h)
    Fy, Qy = _face_fluxes(cls[:, r].T, w[:, r].T, w4[:, r].T, w3b[:, r].T, w3n[:, r].T,
                          v[:, r].T, nu, h)
    Fy, Qy = Fy.T, Qy.T
    # Fx[j, i+1] is the flux on face i+1/2 (i = -1..nx-1); Fy[j+1, i] on face j+1/2
    Tx = Fx + Qx
    Ty = Fy + Qy
    div = (Tx[:, 1:] - Tx[:, :-1]) + (Ty[1:, :] - Ty[:-1, :])
    dw = np.where(geom.fluid, -div / h, 0.0)
    dG = np.zeros(geom.nbc)
    for col, (i0, i1, j0, j1) in enumerate(geom.rects):
        out = (Tx[j0:j1 + 1, i1 + 1].sum() - Tx[j0:j1 + 1, i0].sum()
               + Ty[j1 + 1, i0:i1 + 1].sum() - Ty[j0, i0:i1 + 1].sum())
        dG[col] = -h * out
    return dw, dG, wb, (Fx, Qx, Fy, Qy, e4b, e3b, e3n)
