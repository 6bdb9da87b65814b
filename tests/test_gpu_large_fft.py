"""FFT sizes of the register kernels beyond the 1024 x 512 cylinder's: row
passes of 2048 and 4096 complex points (real rows of 4096 and 8192) and column
passes of 2048 and 4096 points, against the FP64 oracle's zero-padded
lattice-Green's-function convolution (free space and outflow); then one
reconstruction and one RK3 step on the widest torus (outflow, 8192 x 256)
against the oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle import poisson as OP
from oracle.reconstruct import Reconstructor
from oracle import ns as ONS
from gpu_util import to_dev, ring_zeros, rel

pytestmark = pytest.mark.gpu
TOL64 = 1e-11

# (nx, ny, exterior, padded torus the library must choose)
CASES = [
    (1500, 100, "free", (4096, 256)),
    (1100, 100, "outflow", (8192, 256)),
    (300, 700, "free", (1024, 2048)),
    (200, 1500, "free", (512, 4096)),
]


@pytest.mark.parametrize("nx,ny,ext,torus", CASES)
def test_poisson_large_torus(nx, ny, ext, torus):
    g = wl.GridDesc(nx=nx, ny=ny, x0=0.0, y0=0.0, h=1.0 / 64, exterior=ext, u_inf=(1.0, 0.0), nu=0.01)
    # powers of two: these cases exercise the 2048- and 4096-point plans (the
    # default tuner may prefer a compact torus for some of these grids)
    ctx = iim.Context(g, [], fft_sizes=iim.FFT_SIZES_POW2)
    assert (ctx.info["fft_mx"], ctx.info["fft_my"]) == torus
    src = np.random.default_rng(nx + ny).standard_normal((ny, nx))
    psi = ring_zeros(g)
    ctx.poisson(to_dev(src), psi)
    torch.cuda.synchronize()
    ref = OP.FreeSpace(nx, ny, g.h, outflow=ext == "outflow")(src)
    e = rel(psi.cpu().numpy(), ref)
    assert e < 1e-13, e
    ctx.close()


def test_step_on_the_widest_torus():
    w = wl.cylinder(nx=1100, ny=100, h=1.0 / 32, points=128, dt=0.005, steps=1, center=(1.5, 0.0))
    w.grid.exterior = wl.EXT_OUTFLOW
    geo = OG.Geometry(w.grid, w.bodies)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 71, count=8, box=(0.5, 30.0, -1.4, 1.4)), 0.0)
    G = np.array([0.2])
    ref = Reconstructor(geo).reconstruct(om, G)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT, fft_sizes=iim.FFT_SIZES_POW2)
    assert ctx.info["fft_mx"] == 8192
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    ctx.reconstruct(to_dev(om), G, psi, U, V)
    torch.cuda.synchronize()
    fl = np.pad(geo.fluid, 1)
    e = rel(np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]]), np.stack([ref.U[fl], ref.V[fl]]))
    assert e < TOL64, e
    om_ref, G_ref = ONS.Stepper(geo).step(om, G, w.dt)
    d = to_dev(om)
    G1, _ = ctx.rk3_steps(d, G, w.dt, 1)
    torch.cuda.synchronize()
    e = rel(d.cpu().numpy(), om_ref, mask=geo.fluid)
    assert e < TOL64, e
    assert abs(G1[0] - G_ref[0]) < TOL64 * (abs(G_ref[0]) + 1.0)
    ctx.close()
