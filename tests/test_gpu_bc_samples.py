"""Prescribed (non-rigid) boundary data on the GPU: a cylinder whose surface
moves tangentially with a speed varying along it, given as samples at the
boundary points.  Reconstruction and one RK3 step against the FP64 oracle
(dense and Krylov); samples of a rigid translation reproduce the rigid-motion
run."""
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


@pytest.mark.parametrize("solver", [iim.SOLVER_DIRECT, iim.SOLVER_KRYLOV])
def test_surface_driven_cylinder_matches_oracle(solver):
    w = wl.surface_driven_cylinder()
    geo = OG.Geometry(w.grid, w.bodies)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 41, count=5), 0.0)
    G = np.array([0.3])
    ctx = iim.Context(w.grid, w.bodies, solver=solver, tol=1e-13)
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    ctx.reconstruct(to_dev(om), G, psi, U, V)
    torch.cuda.synchronize()
    ref = Reconstructor(geo).reconstruct(om, G)
    fl = np.pad(geo.fluid, 1)
    e = rel(np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]]), np.stack([ref.U[fl], ref.V[fl]]))
    assert e < TOL64, e
    om_ref, G_ref = ONS.Stepper(geo).step(om, G, w.dt)
    omd = to_dev(om)
    G1, _ = ctx.rk3_steps(omd, G, w.dt, 1)
    torch.cuda.synchronize()
    e = rel(omd.cpu().numpy(), om_ref, mask=geo.fluid)
    assert e < TOL64, e
    assert abs(G1[0] - G_ref[0]) < TOL64 * (abs(G_ref[0]) + 1.0)
    ctx.close()


def test_translation_samples_equal_rigid_translation():
    Ut = (0.4, -0.2)
    w = wl.cylinder_small()
    b = w.bodies[0]
    p = b.points
    rigid = [dataclasses.replace(b, u_rigid=Ut)]
    smp = np.stack([np.full(len(p), Ut[0]), np.full(len(p), Ut[1]), Ut[0] * p[:, 1] - Ut[1] * p[:, 0]], 1)
    sampled = [dataclasses.replace(b, bc_samples=smp)]
    geo = OG.Geometry(w.grid, rigid)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 43, count=5), 0.0)
    out = []
    for bodies in (rigid, sampled):
        ctx = iim.Context(w.grid, bodies, solver=iim.SOLVER_DIRECT)
        omd = to_dev(om)
        G1, _ = ctx.rk3_steps(omd, np.array([0.1]), w.dt, 2)
        torch.cuda.synchronize()
        out.append((omd.cpu().numpy(), G1))
        ctx.close()
    assert rel(out[1][0], out[0][0], mask=geo.fluid) < 1e-13
    assert abs(out[1][1][0] - out[0][1][0]) < 1e-13
