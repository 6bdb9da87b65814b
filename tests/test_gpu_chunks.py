"""Many correction sources per FFT column: three bodies on a 256x128 grid give
more affected points than the column pass holds in one LDS buffer (256-point
column FFTs: 273 slots), so their row transforms are staged in several
chunks.  Reconstruction and one RK3 step against the FP64 oracle, free space
and the outflow exterior (mirrored sources), dense and Krylov solvers."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle.reconstruct import Reconstructor
from oracle import ns as ONS
from gpu_util import to_dev, ring_zeros, rel

pytestmark = pytest.mark.gpu
TOL64 = 1e-11
LDS_SLOTS_256 = 256 + 256 // 16 + 1


def _three_bodies(exterior):
    h = 1.0 / 32
    nx, ny = 256, 128
    grid = wl.GridDesc(nx=nx, ny=ny, x0=0.5 * h, y0=-0.5 * ny * h + 0.5 * h, h=h, exterior=exterior,
                       u_inf=(1.0, 0.0), nu=0.01)
    bodies = [wl.BodyDesc(points=wl.circle_points((cx, cy), 0.5, 128, phase=0.013 * k), center=(cx, cy))
              for k, (cx, cy) in enumerate([(1.5, 0.6), (3.5, -0.5), (5.5, 0.4)])]
    return grid, bodies


@pytest.mark.parametrize("exterior", [wl.EXT_FREE, wl.EXT_OUTFLOW])
@pytest.mark.parametrize("solver", [iim.SOLVER_DIRECT, iim.SOLVER_KRYLOV])
def test_chunked_correction_sources(exterior, solver):
    grid, bodies = _three_bodies(exterior)
    geo = OG.Geometry(grid, bodies)
    assert geo.na > LDS_SLOTS_256, geo.na
    rng = np.random.default_rng(31)
    om = np.where(geo.fluid, wl.seeded_vortices(grid, 32, count=8), 0.0)
    G = rng.uniform(-0.4, 0.4, size=geo.nbc)
    ctx = iim.Context(grid, bodies, solver=solver, tol=1e-13)
    assert ctx.info["fft_my"] >= 256
    psi, U, V = ring_zeros(grid), ring_zeros(grid), ring_zeros(grid)
    ctx.reconstruct(to_dev(om), G, psi, U, V)
    torch.cuda.synchronize()
    ref = Reconstructor(geo).reconstruct(om, G)
    fl = np.pad(geo.fluid, 1)
    e = rel(np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]]), np.stack([ref.U[fl], ref.V[fl]]))
    assert e < TOL64, e
    dt = 0.004
    om_ref, G_ref = ONS.Stepper(geo).step(om, G, dt)
    omd = to_dev(om)
    G1, _ = ctx.rk3_steps(omd, G, dt, 1)
    torch.cuda.synchronize()
    e = rel(omd.cpu().numpy(), om_ref, mask=geo.fluid)
    assert e < TOL64, e
    assert np.max(np.abs(G1 - G_ref)) < TOL64 * (np.abs(G_ref).max() + 1.0)
    ctx.close()
