"""Pins of the oracle's time integration (Sec. 5.5, App. B)."""
import json
import os

import numpy as np

import workloads as wl
from oracle import geometry as G, ns

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_rk3_amplification_polynomial():
    for z in (-0.3, 0.1 + 0.7j, -1.2 + 0.2j, 0.05):
        lam = z
        y = ns.rk3_williamson([np.array([1.0 + 0j])], lambda s, k: [lam * s[0]], 1.0)[0][0]
        assert abs(y - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


def test_rk3_third_order_in_time():
    f = lambda s, k: [np.cos(s[0]) + 0.3 * s[0]]
    def run(n):
        y = [np.array([0.4])]
        for _ in range(n):
            y = ns.rk3_williamson(y, f, 1.0 / n)
        return y[0][0]
    ref = run(4096)
    e1, e2 = abs(run(16) - ref), abs(run(32) - ref)
    assert 2.8 < np.log2(e1 / e2) < 3.2


def test_dt_max_on_stability_triangle():
    tri = json.load(open(os.path.join(GOLD, "paper_constants.json")))["rk3_stability_triangle"]
    Cmax, rmax = tri["vertices_C_r"][1][0], tri["vertices_C_r"][2][1]
    for h, nu, a in ((1 / 64, 0.01, 0.3536), (0.01, 1e-4, 2.0), (0.05, 0.1, 0.0)):
        dt = ns.dt_max(h, nu, a)
        C, r = a * dt / h, nu * dt / h ** 2
        assert abs(C / Cmax + r / rmax - 1.0) < 1e-14
    # every named workload's step lies inside the triangle for its own speed
    # bound (the workloads choose dt by a Courant and a diffusion number)
    w = wl.taylor_couette(128)
    assert w.dt <= 0.51 * ns.dt_max(w.grid.h, w.grid.nu, np.sqrt(2) * 0.25)
    assert abs(w.dt - 3.462e-3) < 1e-6
    w = wl.multi_body(512)
    assert w.dt <= 0.7 * ns.dt_max(w.grid.h, w.grid.nu, 2.0 * np.sqrt(2.0))
    for w in wl.batch_serving(8, 5):
        assert w.dt <= 0.7 * ns.dt_max(w.grid.h, w.grid.nu, 3.0)
    for n in (64, 256):
        w = wl.cosine_wave_transport(n, 0.002)
        assert w.dt <= 0.9 * ns.dt_max(w.grid.h, w.grid.nu, 3.0)


def test_free_space_total_circulation_stays_zero():
    """From rest in free space, Gamma_k + h^2 sum_{outside R_k} omega = 0 for
    all time (discrete Kelvin theorem, Sec. 5.1)."""
    w = wl.cylinder_small()
    geo = G.Geometry(w.grid, w.bodies)
    st = ns.Stepper(geo)
    om = np.zeros((geo.ny, geo.nx))
    Gam = np.zeros(1)
    i0, i1, j0, j1 = geo.rects[0]
    for _ in range(4):
        om, Gam = st.step(om, Gam, w.dt)
        tot = Gam[0] + geo.h ** 2 * (om.sum() - om[j0:j1 + 1, i0:i1 + 1].sum())
        assert abs(tot) < 1e-13
    assert np.max(np.abs(om)) > 1.0          # vorticity was created at the wall
    assert np.all(om[geo.solid] == 0.0)


def test_no_bodies_reduces_to_plain_poisson_and_conserves_circulation():
    """With no immersed body the reconstruction is the plain free-space
    Poisson solve (no corrections), and the conservative transport keeps the
    total circulation while the vorticity stays clear of the grid edges."""
    import workloads as wl
    from oracle import geometry as OG, poisson as OP, reconstruct as ORC, ns as ONS
    g = wl.GridDesc(nx=96, ny=80, x0=-0.48, y0=-0.4, h=0.01, exterior="free", u_inf=(0.3, 0.1), nu=0.01)
    geo = OG.Geometry(g, [])
    assert geo.na == 0 and geo.nbc == 0
    X, Y = wl.node_coords(g)
    om = np.exp(-(X ** 2 + Y ** 2) / (2 * 0.05 ** 2)) - 0.5 * np.exp(-((X - 0.1) ** 2 + Y ** 2) / (2 * 0.04 ** 2))
    rec = ORC.Reconstructor(geo).reconstruct(om, np.zeros(0))
    psi = OP.FreeSpace(g.nx, g.ny, g.h)(om)
    u = (psi[2:, 1:-1] - psi[:-2, 1:-1]) / (2 * g.h) + g.u_inf[0]
    v = -(psi[1:-1, 2:] - psi[1:-1, :-2]) / (2 * g.h) + g.u_inf[1]
    assert np.max(np.abs(rec.U[1:-1, 1:-1] - u)) < 1e-13
    assert np.max(np.abs(rec.V[1:-1, 1:-1] - v)) < 1e-13
    om2, G2 = ONS.Stepper(geo).step(om, np.zeros(0), 0.002)
    assert abs(om2.sum() - om.sum()) < 1e-12 * np.abs(om).sum()
