"""The periodic exterior (Sec. 4.1: a rectangle periodic in both
directions, the mean velocity in place of the free stream, a periodic
stream function of zero mean, and the solvability condition
int omega = -sum Gamma_k), pinned independently of the oracle's formulas:

* the zero-mean periodic inverse of the 5-point Laplacian against a sparse
  direct solve of the periodic 5-point system bordered by the zero-mean row;
* the Schur reconstruction against the unreduced system (psi on every node,
  gamma, psibar, the gauge row) solved directly, with circulations that meet
  the discrete solvability condition;
* the wrapped transport right-hand side against the free-space right-hand
  side of the field tiled 3 x 3 (the middle tile);
* steps from a seeded state keep the discrete solvability sum and the mean
  velocity on a full grid column;
* the paper's own transport study (Sec. 3: the periodic cosine wave with
  the C-shaped body, u = (1, 2), k = (4 pi, 2 pi), dt = 0.9 dt_max; up to a
  short final time instead of the paper's T = 1, to keep the test quick):
  third order where advection dominates, second order where diffusion
  does."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import geometry as OG
from oracle import ns as ONS
from oracle import poisson as OP
from oracle import transport as OT
from oracle.reconstruct import Reconstructor


def _periodic_laplacian(nx, ny, h):
    """-lap_h on the periodic lattice, from the 5-point definition."""
    def d1(m):
        D = sp.diags([np.full(m, 2.0), -np.ones(m - 1), -np.ones(m - 1)], [0, 1, -1]).tolil()
        D[0, m - 1] = -1.0
        D[m - 1, 0] = -1.0
        return D.tocsr()
    return (sp.kron(sp.eye(ny), d1(nx)) + sp.kron(d1(ny), sp.eye(nx))) / h ** 2


def test_periodic_poisson_against_bordered_direct_solve():
    nx, ny, h = 16, 12, 0.1
    rng = np.random.default_rng(4)
    s = rng.standard_normal((ny, nx))
    psi = OP.periodic(s, h)
    N = nx * ny
    L = _periodic_laplacian(nx, ny, h)
    # bordered system: [L 1; 1^T 0] [psi; c] = [s; 0]  (c absorbs the mean of s)
    M = sp.bmat([[L, sp.csr_matrix(np.ones((N, 1)))], [sp.csr_matrix(np.ones((1, N))), None]]).tocsc()
    sol = spla.spsolve(M, np.concatenate([s.ravel(), [0.0]]))
    ref = sol[:N].reshape(ny, nx)
    assert np.max(np.abs(psi[1:-1, 1:-1] - ref)) < 1e-12 * np.max(np.abs(ref))
    assert abs(sol[N] - s.mean()) < 1e-12
    # zero mean, residual = the source minus its mean, ring = periodic images
    assert abs(psi[1:-1, 1:-1].mean()) < 1e-14 * np.max(np.abs(ref))
    p = psi[1:-1, 1:-1]
    lap = (np.roll(p, 1, 0) + np.roll(p, -1, 0) + np.roll(p, 1, 1) + np.roll(p, -1, 1) - 4 * p) / h ** 2
    assert np.max(np.abs(-lap - (s - s.mean()))) < 1e-11 * np.max(np.abs(s))
    assert np.array_equal(psi[0, 1:-1], p[-1]) and np.array_equal(psi[-1, 1:-1], p[0])
    assert np.array_equal(psi[1:-1, 0], p[:, -1]) and np.array_equal(psi[1:-1, -1], p[:, 0])


def _small_periodic():
    w = wl.periodic_cylinder(nx=64, ny=32, h=1.0 / 8, points=96, center=(2.0, 0.0), mean=(0.7, 0.2))
    geo = OG.Geometry(w.grid, w.bodies)
    return w, geo


def _solvable_state(geo, grid, seed):
    """Seeded vorticity and the circulation that meets the discrete
    solvability condition h^2 sum_{outside R} omega = -Gamma."""
    om = np.where(geo.fluid, wl.seeded_vortices(grid, seed, count=5, amp=1.0), 0.0)
    i0, i1, j0, j1 = geo.rects[0]
    inside = np.zeros_like(geo.fluid)
    inside[j0:j1 + 1, i0:i1 + 1] = True
    G = np.array([-grid.h ** 2 * om[~inside].sum()])
    return om, G


def test_periodic_schur_matches_unreduced_direct_solve():
    w, geo = _small_periodic()
    grid = w.grid
    om, G = _solvable_state(geo, grid, 8)
    nx, ny, h = grid.nx, grid.ny, grid.h
    N, na = nx * ny, geo.na
    L = _periodic_laplacian(nx, ny, h)
    ones_c = (geo.c_body == 0).astype(float)
    top = sp.hstack([L, geo.Ea, sp.csr_matrix((N, 1))]).tolil()
    # the Poisson rows sum to the circulation row (solvable data): replace
    # the first by the gauge row, sum psi = 0
    top[0, :] = 0.0
    top[0, :N] = 1.0
    mid = sp.hstack([-geo.Aop, sp.eye(na), sp.csr_matrix(-(geo.Bop @ ones_c)[:, None])])
    circ = np.zeros((1, na))
    circ[0, geo.a_body == 0] = 1.0
    bot = sp.hstack([sp.csr_matrix((1, N)), sp.csr_matrix(circ), sp.csr_matrix((1, 1))])
    M = sp.vstack([top.tocsr(), mid, bot]).tocsc()
    i0, i1, j0, j1 = geo.rects[0]
    b0 = om.ravel().copy()
    b0[0] = 0.0
    rhs = np.concatenate([b0, geo.Bop @ geo.psi_tilde_b(), [om[j0:j1 + 1, i0:i1 + 1].sum() - G[0] / h ** 2]])
    sol = spla.spsolve(M, rhs)
    psi_ref, gam_ref, pb_ref = sol[:N].reshape(ny, nx), sol[N:N + na], sol[-1]
    # the dropped row holds for the solution
    assert abs((L @ sol[:N] + geo.Ea @ gam_ref)[0] - om.ravel()[0]) < 1e-9 * np.abs(om).max()
    R = Reconstructor(geo)
    for method in ("direct", "gmres"):
        rec = R.reconstruct(om, G, method=method, tol=1e-15)
        assert np.max(np.abs(rec.gamma - gam_ref)) < 1e-10 * np.max(np.abs(gam_ref)), method
        assert abs(rec.psibar[0] - pb_ref) < 1e-11 * (1 + abs(pb_ref)), method
        assert np.max(np.abs(rec.psi[1:-1, 1:-1] - psi_ref)) < 1e-11 * np.max(np.abs(psi_ref)), method
    assert np.max(np.abs(psi_ref[geo.solid])) < 1e-11 * np.max(np.abs(psi_ref))


def test_periodic_transport_equals_tiled_free_space():
    nx, ny, h, nu = 24, 16, 0.05, 0.02
    g = wl.GridDesc(nx=nx, ny=ny, x0=0.0, y0=0.0, h=h, exterior=wl.EXT_PERIODIC, u_inf=(0.5, -0.3), nu=nu)
    rng = np.random.default_rng(9)
    X, Y = wl.node_coords(g)
    Lx, Ly = nx * h, ny * h
    om = np.sin(2 * np.pi * X / Lx) * np.cos(4 * np.pi * Y / Ly) + 0.2 * rng.standard_normal((ny, nx))
    Un = 0.5 + 0.8 * np.cos(2 * np.pi * Y / Ly + 0.4) + 0.1 * rng.standard_normal((ny, nx))
    Vn = -0.3 + 0.7 * np.sin(2 * np.pi * X / Lx) + 0.1 * rng.standard_normal((ny, nx))
    ring = lambda a: np.pad(a, 1, mode="wrap")
    dw, _, _, _ = OT.rhs(OG.Geometry(g, []), om, ring(Un), ring(Vn), nu, wb=np.zeros(0))
    gt = wl.GridDesc(nx=3 * nx, ny=3 * ny, x0=0.0, y0=0.0, h=h, exterior=wl.EXT_FREE, nu=nu)
    tile = lambda a: np.tile(a, (3, 3))
    dwt, _, _, _ = OT.rhs(OG.Geometry(gt, []), tile(om), np.pad(tile(Un), 1), np.pad(tile(Vn), 1), nu,
                          wb=np.zeros(0))
    mid = dwt[ny:2 * ny, nx:2 * nx]
    assert np.max(np.abs(dw - mid)) < 1e-12 * np.max(np.abs(mid))
    # the edges matter: plain free space differs there
    gf = wl.GridDesc(nx=nx, ny=ny, x0=0.0, y0=0.0, h=h, exterior=wl.EXT_FREE, nu=nu)
    dwf, _, _, _ = OT.rhs(OG.Geometry(gf, []), om, ring(Un), ring(Vn), nu, wb=np.zeros(0))
    assert np.max(np.abs(dwf - mid)) > 1e-2 * np.max(np.abs(mid))


def test_periodic_steps_keep_solvability_and_mean_velocity():
    w, geo = _small_periodic()
    om, G = _solvable_state(geo, w.grid, 12)
    st = ONS.Stepper(geo)
    i0, i1, j0, j1 = geo.rects[0]
    inside = np.zeros_like(geo.fluid)
    inside[j0:j1 + 1, i0:i1 + 1] = True
    h = w.grid.h
    scale = h ** 2 * np.abs(om).sum()
    for _ in range(4):
        om, G = st.step(om, G, 0.02)
        assert abs(h ** 2 * om[~inside].sum() + G[0]) < 1e-13 * scale
    rec = st.rec.reconstruct(om, G)
    # the mean velocity on a grid column (and row) clear of the body
    U, V = rec.U[1:-1, 1:-1], rec.V[1:-1, 1:-1]
    assert abs(U[:, 2].mean() - w.grid.u_inf[0]) < 1e-13
    assert abs(V[2, :].mean() - w.grid.u_inf[1]) < 1e-13


def _cosine_error(n, nu, T):
    w = wl.cosine_wave_transport(n, nu)
    g, ex = w.grid, w.extra["exact"]
    geo = OG.Geometry(g, w.bodies)
    X, Y = wl.node_coords(g)
    U = np.full((n + 2, n + 2), w.extra["u"][0])
    V = np.full((n + 2, n + 2), w.extra["u"][1])
    steps = int(np.ceil(T / w.dt))
    dt = T / steps
    cs = ONS.rk3_stage_times()
    om = np.where(geo.fluid, ex(X, Y, 0.0), 0.0)
    for k in range(steps):
        t = k * dt
        rhs = lambda st, s: [OT.rhs(geo, st[0], U, V, nu, wb=ex(geo.c_x, geo.c_y, t + cs[s] * dt))[0]]
        om = ONS.rk3_williamson([om], rhs, dt)[0]
    e = (om - ex(X, Y, T))[geo.fluid]
    return np.sqrt(np.mean(e ** 2)), np.abs(e).max()


def test_cosine_wave_transport_orders():
    """Sec. 3's periodic transport case: cell Reynolds number above one (nu
    0.002): third order; below one (nu 0.064): second order."""
    e = [_cosine_error(n, 0.002, 0.1) for n in (64, 128, 256)]
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[0] / b[0]) > 2.7 and np.log2(a[1] / b[1]) > 2.5, e
    # (a short time: diffusion-limited steps; the orders approach two from
    # below, 1.78 then 1.89 in L2)
    e = [_cosine_error(n, 0.064, 0.005) for n in (64, 128, 256)]
    r2 = [np.log2(a[0] / b[0]) for a, b in zip(e[:-1], e[1:])]
    ri = [np.log2(a[1] / b[1]) for a, b in zip(e[:-1], e[1:])]
    assert min(r2) > 1.7 and r2[-1] > 1.85 and min(ri) > 1.8, e
