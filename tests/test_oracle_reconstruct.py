"""Pins of the oracle's IIM velocity reconstruction (Sec. 4.2-4.3)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import exp1

import workloads as wl
from oracle import geometry as G
from oracle.reconstruct import Reconstructor


def _box_case():
    n = 40
    h = 2.0 / n
    grid = wl.GridDesc(nx=n, ny=n, x0=-1 + h / 2, y0=-1 + h / 2, h=h, exterior="box")
    body = wl.BodyDesc(points=wl.circle_points((0.053, -0.021), 0.31, 128), center=(0.05, -0.02),
                       omega_rigid=0.7, u_rigid=(0.2, -0.1))
    return grid, [body]


def test_schur_matches_unreduced_direct_solve():
    """Solve the unreduced system (psi on every node, gamma, psibar) with a
    sparse direct solver, assembled here from its definition, and compare with
    the Schur complement solution (dense and GMRES)."""
    grid, bodies = _box_case()
    geo = G.Geometry(grid, bodies)
    R = Reconstructor(geo)
    rng = np.random.default_rng(3)
    X, Y = wl.node_coords(grid)
    omega = np.where(geo.fluid, np.sin(3 * X) * np.cos(2 * Y) + rng.uniform(-0.1, 0.1, X.shape), 0.0)
    Gam = np.array([0.37])
    n, h = grid.nx, grid.h
    N = n * n
    # -lap_h with zero psi on the box faces (reflection across the faces)
    def d1(m):
        main = np.full(m, 2.0)
        main[0] = main[-1] = 3.0
        return sp.diags([main, -np.ones(m - 1), -np.ones(m - 1)], [0, 1, -1])
    L = (sp.kron(sp.eye(n), d1(n)) + sp.kron(d1(n), sp.eye(n))) / h ** 2
    na = geo.na
    ones = (geo.c_body == 0).astype(float)
    top = sp.hstack([L, geo.Ea, sp.csr_matrix((N, 1))])
    mid = sp.hstack([-geo.Aop, sp.eye(na), sp.csr_matrix(-(geo.Bop @ ones)[:, None])])
    circ = np.zeros((1, na))
    circ[0, geo.a_body == 0] = 1.0
    bot = sp.hstack([sp.csr_matrix((1, N)), sp.csr_matrix(circ), sp.csr_matrix((1, 1))])
    M = sp.vstack([top, mid, bot]).tocsc()
    i0, i1, j0, j1 = geo.rects[0]
    rhs = np.concatenate([omega.ravel(), geo.Bop @ geo.c_psib,
                          [omega[j0:j1 + 1, i0:i1 + 1].sum() - Gam[0] / h ** 2]])
    sol = spla.spsolve(M, rhs)
    psi_ref, gam_ref, pb_ref = sol[:N].reshape(n, n), sol[N:N + na], sol[-1]
    for method in ("direct", "gmres"):
        rec = R.reconstruct(omega, Gam, method=method, tol=1e-15)
        assert np.max(np.abs(rec.gamma - gam_ref)) < 1e-10 * np.max(np.abs(gam_ref))
        assert abs(rec.psibar[0] - pb_ref) < 1e-12
        assert np.max(np.abs(rec.psi[1:-1, 1:-1] - psi_ref)) < 1e-12 * np.max(np.abs(psi_ref))
    # zero extension: psi vanishes at solid nodes (two-sided corrections)
    assert np.max(np.abs(psi_ref[geo.solid])) < 1e-13


def _tc_error(n):
    w = wl.taylor_couette(n)
    geo = G.Geometry(w.grid, w.bodies)
    R = Reconstructor(geo)
    X, Y = wl.node_coords(w.grid)
    r = np.hypot(X, Y)
    omega = np.where(geo.fluid, -0.25, 0.0)
    i0, i1, j0, j1 = geo.rects[0]
    # circulation on dR_1: pi/8 on the cylinder plus omega times the fluid area
    Gam = np.pi / 8 - 0.25 * ((i1 - i0 + 1) * (j1 - j0 + 1) * geo.h ** 2 - np.pi * 0.25 ** 2)
    rec = R.reconstruct(omega, [Gam])
    A, B = -0.125, 0.0703125
    ut = A * r + B / r
    err = np.hypot(rec.U[1:-1, 1:-1] + ut * Y / r, rec.V[1:-1, 1:-1] - ut * X / r)[geo.fluid]
    psi_solid = np.max(np.abs(rec.psi[1:-1, 1:-1][geo.solid]))
    return np.sqrt(np.mean(err ** 2)), err.max(), psi_solid


def test_taylor_couette_second_order():
    e = [_tc_error(n) for n in (64, 128, 256)]
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[0] / b[0]) > 1.9
        assert np.log2(a[1] / b[1]) > 1.75
    assert max(x[2] for x in e) < 1e-14


def _lamb_oseen_error(n):
    G0, nut, x0 = 1.0, 0.0025, (0.501, 0.501)
    a = 4 * nut

    def psi_lo(x, y):
        r2 = (x - x0[0]) ** 2 + (y - x0[1]) ** 2
        return -G0 / (4 * np.pi) * (np.log(r2 / a) + exp1(r2 / a))

    def u_lo(x, y):
        dx, dy = x - x0[0], y - x0[1]
        r2 = dx * dx + dy * dy
        f = G0 / (2 * np.pi * r2) * (1 - np.exp(-r2 / a))
        return (-f * dy, f * dx)

    w = wl.two_c_shapes_lamb_oseen(n)
    geo = G.Geometry(w.grid, w.bodies, bc_override=(psi_lo, u_lo))
    R = Reconstructor(geo)
    X, Y = wl.node_coords(w.grid)
    om = G0 / (4 * np.pi * nut) * np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2) / a)
    Gam = [geo.h ** 2 * om[j0:j1 + 1, i0:i1 + 1].sum() for (i0, i1, j0, j1) in geo.rects]
    rec = R.reconstruct(om, Gam)
    ue, ve = u_lo(X, Y)
    err = np.hypot(rec.U[1:-1, 1:-1] - ue, rec.V[1:-1, 1:-1] - ve)[geo.fluid]
    return np.sqrt(np.mean(err ** 2)), err.max()


def test_lamb_oseen_nonconvex_second_order():
    e = [_lamb_oseen_error(n) for n in (64, 128, 256)]
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[0] / b[0]) > 1.9
        assert np.log2(a[1] / b[1]) > 1.85


def _circulation(psi, i0, i1, j0, j1):
    P = psi[1:-1, 1:-1]
    right = (P[j0:j1 + 1, i1 + 1] - P[j0:j1 + 1, i1]).sum()
    left = (P[j0:j1 + 1, i0] - P[j0:j1 + 1, i0 - 1]).sum()
    top = (P[j1 + 1, i0:i1 + 1] - P[j1, i0:i1 + 1]).sum()
    bot = (P[j0, i0:i1 + 1] - P[j0 - 1, i0:i1 + 1]).sum()
    return -(right - left + top - bot)


@pytest.mark.parametrize("make", [wl.cylinder_small, lambda: wl.taylor_couette(96)])
def test_discrete_stokes_on_enclosing_rectangles(make):
    """-h sum_dR grad_h psi . n = Gamma_k + h^2 sum_{R minus R_k} omega for every
    grid-aligned R containing R_k and no other body (Sec. 4.2, Sec. 5.1)."""
    w = make()
    geo = G.Geometry(w.grid, w.bodies)
    R = Reconstructor(geo)
    rng = np.random.default_rng(9)
    omega = np.where(geo.fluid, wl.seeded_vortices(w.grid, 4, count=5), 0.0)
    Gam = rng.uniform(-0.4, 0.4, geo.nbc)
    rec = R.reconstruct(omega, Gam)
    i0, i1, j0, j1 = geo.rects[0]
    scale = np.abs(omega).sum() * geo.h ** 2 + 1
    for d in (0, 1, 2):
        lhs = _circulation(rec.psi, i0 - d, i1 + d, j0 - d, j1 + d)
        inner = omega[j0:j1 + 1, i0:i1 + 1].sum()
        outer = omega[j0 - d:j1 + d + 1, i0 - d:i1 + d + 1].sum()
        assert abs(lhs - (Gam[0] + geo.h ** 2 * (outer - inner))) < 1e-12 * scale
