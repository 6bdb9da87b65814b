"""Convergence order of the library's transport right-hand side (iim_rhs,
Sec. 3) at resolutions beyond the oracle's: a Gaussian vortex carried by the
uniform velocity (1, 2) with no body, exact solution a carried and spreading
Gaussian; RK3 steps of the library's right-hand side (the low-storage
combination done here with tensor arithmetic).  Third order where advection
dominates, second order where diffusion does."""
import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim

pytestmark = pytest.mark.gpu
U0, S0, C0 = (1.0, 2.0), 0.12, (-0.3, -0.45)
RK_A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK_B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)


def _error(n, nu, T, c0=C0, cfl=0.5):
    h = 2.0 / n
    g = wl.GridDesc(nx=n, ny=n, x0=-1 + 0.5 * h, y0=-1 + 0.5 * h, h=h, nu=nu)
    ctx = iim.Context(g, [], solver=iim.SOLVER_DIRECT)
    X, Y = wl.node_coords(g)

    def exact(t):
        s2 = S0 * S0 + 2 * nu * t
        return (S0 * S0 / s2) * np.exp(-((X - c0[0] - U0[0] * t) ** 2 + (Y - c0[1] - U0[1] * t) ** 2) / (2 * s2))

    dev = torch.device("cuda:0")
    u = torch.full((n + 2, n + 2), U0[0], dtype=torch.float64, device=dev)
    v = torch.full((n + 2, n + 2), U0[1], dtype=torch.float64, device=dev)
    steps = int(np.ceil(T / (cfl * ctx.dt_max(abs(U0[0]) + abs(U0[1])))))
    dt = T / steps
    om = torch.as_tensor(exact(0.0), device=dev).contiguous()
    Q = torch.zeros_like(om)
    r = torch.zeros_like(om)
    for _ in range(steps):
        for s in range(3):
            ctx.rhs(om, u, v, r)
            Q.mul_(RK_A[s]).add_(r, alpha=dt)
            om.add_(Q, alpha=RK_B[s])
    torch.cuda.synchronize()
    e = om.cpu().numpy() - exact(T)
    ctx.close()
    return np.sqrt(np.mean(e ** 2)), np.abs(e).max()


def test_third_order_where_advection_dominates():
    e = [_error(n, 1e-5, 0.2) for n in (128, 256, 512)]
    print(e)
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[0] / b[0]) > 2.8 and np.log2(a[1] / b[1]) > 2.7, e


def test_second_order_where_diffusion_dominates():
    # centred, so that the spread vortex stays below 1e-8 at the domain's
    # edge (beyond which the free-space transport takes no vorticity)
    e = [_error(n, 0.5, 0.01, c0=(0.0, 0.0)) for n in (64, 128, 256)]
    print(e)
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[0] / b[0]) > 1.75 and np.log2(a[1] / b[1]) > 1.75, e
