"""Surface loads (Sec. 5.4) on the GPU against the FP64 oracle: boundary
vorticity, shear, vorticity flux, relative surface pressure and the force and
torque on each body, from the same vorticity and circulations.  The tolerance
allows for the reconstruction's 1e-11 velocity agreement carried through two
differences at spacing h (omega_b, then d omega/dn).  Stationary bodies, a
body in rigid translation and rotation (the rigid-motion terms of the
traction and of the tangential pressure gradient), and a body with sampled
boundary data.  The symmetric start from rest gives no lift and no torque."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle.reconstruct import Reconstructor
from oracle import ns as ONS
from oracle import loads as OL
from gpu_util import to_dev, ring_zeros

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _lib_loads(ctx, grid, om, G):
    psi, U, V = ring_zeros(grid), ring_zeros(grid), ring_zeros(grid)
    d = to_dev(om)
    ctx.reconstruct(d, G, psi, U, V)
    out = ctx.surface_loads(d, U, V)
    torch.cuda.synchronize()
    return out


def _close(a, b, tol):
    scale = max(np.max(np.abs(b)), 1e-300)
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= tol * scale


def _rigid_motion_cylinder():
    w = wl.cylinder_small()
    w.bodies[0] = dataclasses.replace(w.bodies[0], u_rigid=(0.2, -0.1), omega_rigid=1.3)
    return w


CASES = {"cylinder": wl.cylinder_small, "two_c_shapes": lambda: wl.two_c_shapes_lamb_oseen(128),
         "rigid_motion": _rigid_motion_cylinder, "sampled_surface": wl.surface_driven_cylinder}


@pytest.mark.parametrize("name", list(CASES))
def test_surface_loads_match_oracle(name):
    w = CASES[name]()
    geo = OG.Geometry(w.grid, w.bodies)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 51, count=6), 0.0)
    G = wl.seeded_gammas(geo.nbc, 52, scale=0.3)
    ref = Reconstructor(geo).reconstruct(om, G)
    L_ref = OL.surface_loads(geo, om, ref.U, ref.V)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    L = _lib_loads(ctx, w.grid, om, G)
    for key in ("omega_b", "tau", "dwdn", "p"):
        assert _close(L[key], L_ref[key], TOL), (key, np.max(np.abs(L[key] - L_ref[key])))
    assert _close(L["forces"], L_ref["forces"], TOL), (L["forces"], L_ref["forces"])
    ctx.close()


def test_symmetric_start_has_no_lift_or_torque():
    w = wl.cylinder_small()
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    om = torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0")
    G, _ = ctx.rk3_steps(om, np.zeros(1), w.dt, 4)
    torch.cuda.synchronize()
    L = _lib_loads(ctx, w.grid, om.cpu().numpy(), G)
    Fx, Fy, T = L["forces"][0]
    assert Fx > 0.0
    assert abs(Fy) < 1e-10 * Fx and abs(T) < 1e-10 * Fx, (Fx, Fy, T)
    ctx.close()
