"""IIM velocity reconstruction (Sec. 4.1-4.2).

Discrete problem (two-sided corrections, zero extension inside solids):

    -lap_h psi + E_a gamma = omega                     on every grid node
    gamma = A psi + B (psi_b_tilde + sum_k psibar_k 1_k)   on the affected points
    sum_{B_k} gamma = sum_{R_k} omega - Gamma_k / h^2   for every non-enclosing body

Eliminating psi = G (omega - E_a gamma), G = (-lap_h)^-1 with the exterior
condition, gives the Schur system solved here (our reading of the Schur
equation: the sign follows from substituting the psi recovery into the
correction equation),

    (I + A G E_a) gamma - sum_k psibar_k B 1_k = A G omega + B psi_b_tilde,
    sum_{B_k} gamma = sum_{R_k} omega - Gamma_k / h^2.

The circulation row follows from summing the 5-point equation over R_k
(discrete Gauss theorem) with the circulation h^-2 scaling kept.

psi is the perturbation stream function; in free space the total stream
function is psi + psi_inf, psi_inf = u_inf,x y - u_inf,y x, and
psi_b_tilde = psi_b - psi_inf at the control points.  With the periodic
exterior (Sec. 4.1) u_inf is the prescribed mean velocity, psi is periodic
with zero mean, and the system is solvable when the circulations satisfy
the discrete form of the paper's solvability condition,
h^2 sum_{outside every R_k} omega = -sum_k Gamma_k (summing the 5-point
equation over the periodic lattice gives sum omega = sum_A gamma, and the
circulation rows give sum_A gamma); G drops the mean of its source.

Velocity (Sec. 4.2, last paragraph): psi is extrapolated to A- at fourth
order with the boundary value psi_b_tilde + psibar_k, then
u = (psi_{j+1} - psi_{j-1}) / 2h + u_inf,x,  v = -(psi_{i+1} - psi_{i-1}) / 2h + u_inf,y
at fluid nodes; both components are then extended to A- at third order with
the boundary velocity u_b (Sec. 3.2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import poisson, lgf
from .geometry import Geometry


class Reconstruction:
    """Result of one reconstruction: gamma, psibar, psi (ring array, ghosts
    filled), velocity arrays U, V (ring arrays, extended to A-)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


class Reconstructor:
    def __init__(self, geom: Geometry, lgf_tab=None):
        self.geom = g = geom
        grid = g.grid
        self.h = grid.h
        self.ext = grid.exterior
        if self.ext == "box":
            self._G = lambda s: poisson.box_dirichlet(s, self.h)
            self._tab = None
        elif self.ext == "periodic":
            self._G = lambda s: poisson.periodic(s, self.h)
            self._tab = None
        else:
            out = self.ext == "outflow"
            mx = (4 if out else 2) * g.nx
            my = 2 * g.ny
            self._tab = lgf_tab if lgf_tab is not None else lgf.cached_lgf_table(mx // 2, my // 2)
            self._fs = poisson.FreeSpace(g.nx, g.ny, self.h, table=self._tab, outflow=out)
            self._G = self._fs
        nbc = g.nbc
        # B 1_k for the circulating bodies
        self.B1 = np.zeros((g.na, nbc))
        for col, k in enumerate(g.circ_bodies):
            ones = (g.c_body == k).astype(np.float64)
            self.B1[:, col] = g.Bop @ ones
        self.n = g.na + nbc
        self.body_rows = np.zeros((nbc, g.na))
        for col, k in enumerate(g.circ_bodies):
            self.body_rows[col, g.a_body == k] = 1.0
        self.psib_t = g.psi_tilde_b()
        self.matvecs = 0

    # ------------------------------------------------------------------
    def G(self, s):
        return self._G(s)

    def masked(self, omega):
        return np.where(self.geom.fluid, omega, 0.0)

    def scatter(self, gamma):
        g = self.geom
        s = np.zeros(g.nx * g.ny)
        s[g.a_lin] = gamma
        return s.reshape(g.ny, g.nx)

    def gather(self, psi_ring):
        return self.geom.Aop @ psi_ring[1:-1, 1:-1].ravel()

    def rect_sums(self, omega):
        out = np.zeros(self.geom.nbc)
        for col, (i0, i1, j0, j1) in enumerate(self.geom.rects):
            out[col] = omega[j0:j1 + 1, i0:i1 + 1].sum()
        return out

    # ------------------------------------------------------------------
    def matvec(self, x):
        g = self.geom
        gam, pb = x[:g.na], x[g.na:]
        self.matvecs += 1
        y = np.empty_like(x)
        y[:g.na] = gam + self.gather(self.G(self.scatter(gam))) - self.B1 @ pb
        y[g.na:] = self.body_rows @ gam
        return y

    def rhs(self, omega, Gamma):
        g = self.geom
        w = self.masked(omega)
        b = np.empty(self.n)
        b[:g.na] = self.gather(self.G(w)) + g.Bop @ self.psib_t
        b[g.na:] = self.rect_sums(w) - np.asarray(Gamma, dtype=np.float64) / self.h ** 2
        return b

    def dense_matrix(self):
        """The Schur system as a dense matrix (columns = unknowns)."""
        g = self.geom
        n, na = self.n, g.na
        S = np.zeros((n, n))
        if self._tab is not None:
            # A G E_a through direct lattice Green's function lookups
            cols = np.unique(g.Aop.tocsr().indices)       # grid nodes read by A
            Ar = g.Aop[:, cols]
            ri, rj = cols % g.nx, cols // g.nx
            di = np.abs(ri[:, None] - g.a_i[None, :])
            dj = np.abs(rj[:, None] - g.a_j[None, :])
            GRA = self.h ** 2 * self._tab[dj, di]
            if self.ext == "outflow":
                dm = np.abs(ri[:, None] + g.a_i[None, :] - (2 * g.nx - 1))
                GRA = GRA + self.h ** 2 * self._tab[dj, dm]
            S[:na, :na] = np.eye(na) + Ar @ GRA
        else:
            for q in range(na):
                e = np.zeros(na)
                e[q] = 1.0
                S[:na, q] = e + self.gather(self.G(self.scatter(e)))
        S[:na, na:] = -self.B1
        S[na:, :na] = self.body_rows
        return S

    # ------------------------------------------------------------------
    def solve(self, omega, Gamma, method="direct", x0=None, tol=1e-14, restart=60, maxiter=2000):
        b = self.rhs(omega, Gamma)
        info = {}
        if method == "direct":
            x = np.linalg.solve(self.dense_matrix(), b)
            info["iters"] = 0
        else:
            x, info = gmres(self.matvec, b, x0=x0, tol=tol, restart=restart, maxiter=maxiter)
        info["res"] = np.linalg.norm(self.matvec(x) - b) / max(np.linalg.norm(b), 1e-300)
        return x, b, info

    def recover(self, omega, x):
        """psi from gamma, ghost fill, velocity and its extension."""
        g = self.geom
        h = self.h
        gam, pb = x[:g.na], x[g.na:]
        w = self.masked(omega)
        psi = self.G(w - self.scatter(gam))
        # ghost values of psi (fourth order with psi_b_tilde + psibar_k)
        bc = self.psib_t.copy()
        for col, k in enumerate(g.circ_bodies):
            bc[g.c_body == k] += pb[col]
        grid_psi = psi[1:-1, 1:-1].ravel()
        ghost = g.E4b_f @ grid_psi + g.E4b_b @ bc
        psi_g = psi.copy()
        psi_g[g.g_j + 1, g.g_i + 1] = ghost
        uix, uiy = g.grid.u_inf
        U = np.zeros_like(psi)
        V = np.zeros_like(psi)
        P = psi_g
        fl = g.fluid
        Uc = uix + (P[2:, 1:-1] - P[:-2, 1:-1]) / (2 * h)
        Vc = uiy - (P[1:-1, 2:] - P[1:-1, :-2]) / (2 * h)
        U[1:-1, 1:-1] = np.where(fl, Uc, 0.0)
        V[1:-1, 1:-1] = np.where(fl, Vc, 0.0)
        # ring: normal components on the four edges
        U[1:-1, 0] = uix + (P[2:, 0] - P[:-2, 0]) / (2 * h)
        U[1:-1, -1] = uix + (P[2:, -1] - P[:-2, -1]) / (2 * h)
        V[0, 1:-1] = uiy - (P[0, 2:] - P[0, :-2]) / (2 * h)
        V[-1, 1:-1] = uiy - (P[-1, 2:] - P[-1, :-2]) / (2 * h)
        # extension of the velocity to A- (third order with u_b)
        Ug = g.E3b_f @ U[1:-1, 1:-1].ravel() + g.E3b_b @ g.c_ub[:, 0]
        Vg = g.E3b_f @ V[1:-1, 1:-1].ravel() + g.E3b_b @ g.c_ub[:, 1]
        U[g.g_j + 1, g.g_i + 1] = Ug
        V[g.g_j + 1, g.g_i + 1] = Vg
        return Reconstruction(gamma=gam, psibar=pb, psi=psi, psi_g=psi_g, U=U, V=V)

    def reconstruct(self, omega, Gamma, method="direct", x0=None, tol=1e-14):
        x, b, info = self.solve(omega, Gamma, method=method, x0=x0, tol=tol)
        rec = self.recover(omega, x)
        rec.x, rec.b, rec.info = x, b, info
        return rec


def gmres(A, b, x0=None, tol=1e-14, restart=60, maxiter=2000):
    """Restarted GMRES with modified Gram-Schmidt and Givens rotations; stops
    when ||b - A x|| <= tol ||b||."""
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), {"iters": 0, "converged": True}
    total = 0
    while total < maxiter:
        r = b - A(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x, {"iters": total, "converged": True}
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        e = np.zeros(m + 1)
        e[0] = beta
        V[0] = r / beta
        k_done = 0
        for k in range(m):
            w = A(V[k])
            total += 1
            for i in range(k + 1):
                H[i, k] = np.dot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            e[k + 1] = -sn[k] * e[k]
            e[k] = cs[k] * e[k]
            k_done = k + 1
            if abs(e[k + 1]) <= tol * bnorm or total >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), e[:k_done])
        x = x + V[:k_done].T @ y
    r = b - A(x)
    return x, {"iters": total, "converged": np.linalg.norm(r) <= tol * bnorm}
