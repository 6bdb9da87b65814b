"""The velocity-reconstruction convergence study of Sec. 4.3 on the GPU, at
resolutions beyond the oracle's reach: a Lamb-Oseen vortex (x_0 = (0.501,
0.501), Gamma = 1, nu t = 0.0025) over the two C-shaped bodies of the
study's table on the unit square, N = 128 ... 1024 points a side, free space.
The bodies carry the exact velocity and stream function of the vortex as
boundary samples; each body's circulation is h^2 times the sum of the vortex
vorticity over its bounding region.  The L2 and L-infinity norms of the
velocity error over the fluid nodes fall at second order."""
import dataclasses

import numpy as np
import pytest
import torch
from scipy.special import exp1

import workloads as wl
import paper_2109_13628_amd as iim
from gpu_util import to_dev, ring_zeros

pytestmark = pytest.mark.gpu
G0, NUT, X0 = 1.0, 0.0025, (0.501, 0.501)
A = 4 * NUT


def _psi(x, y):
    r2 = (x - X0[0]) ** 2 + (y - X0[1]) ** 2
    return -G0 / (4 * np.pi) * (np.log(r2 / A) + exp1(r2 / A))


def _vel(x, y):
    dx, dy = x - X0[0], y - X0[1]
    r2 = dx * dx + dy * dy
    f = G0 / (2 * np.pi * r2) * (-np.expm1(-r2 / A))
    return -f * dy, f * dx


def _error(n):
    w = wl.two_c_shapes_lamb_oseen(n)
    bodies = []
    for b in w.bodies:
        p = b.points
        u, v = _vel(p[:, 0], p[:, 1])
        bodies.append(dataclasses.replace(b, bc_samples=np.stack([u, v, _psi(p[:, 0], p[:, 1])], axis=1)))
    ctx = iim.Context(w.grid, bodies, solver=iim.SOLVER_DIRECT)
    geo = ctx.geometry()
    X, Y = wl.node_coords(w.grid)
    om = G0 / (4 * np.pi * NUT) * np.exp(-((X - X0[0]) ** 2 + (Y - X0[1]) ** 2) / A)
    h = w.grid.h
    Gam = np.array([h * h * om[j0:j1 + 1, i0:i1 + 1].sum() for (i0, i1, j0, j1) in geo["rects"]])
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    ctx.reconstruct(to_dev(om), Gam, psi, U, V)
    torch.cuda.synchronize()
    ue, ve = _vel(X, Y)
    fl = geo["cls"] == 0
    err = np.hypot(U.cpu().numpy()[1:-1, 1:-1] - ue, V.cpu().numpy()[1:-1, 1:-1] - ve)[fl]
    ctx.close()
    return np.sqrt(np.mean(err ** 2)), err.max()


def test_lamb_oseen_two_c_shapes_second_order():
    e = [_error(n) for n in (128, 256, 512, 1024)]
    print(e)
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[0] / b[0]) > 1.85, e
        assert np.log2(a[1] / b[1]) > 1.7, e
