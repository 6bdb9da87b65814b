"""Control-volume terms (Sec. 5.4: Noca's momentum formulation for the force,
the paper's analogue for the moment) on the GPU against the FP64 oracle:
S_t, S_gamma, the cut-cell volume term I and S_lambda, from the same velocity
and vorticity (1e-12), and end to end from the oracle's own reconstruction
(the 1e-11 velocity agreement carried through one difference at spacing h:
1e-9).
Boxes that leave the grid or touch the body, and moving bodies inside the
box, are rejected."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle.reconstruct import Reconstructor
from oracle import loads as OL
from gpu_util import to_dev, ring_zeros

pytestmark = pytest.mark.gpu


def _box(grid, x0, x1, y0, y1):
    h = grid.h
    return (int(round((x0 - grid.x0) / h)), int(round((x1 - grid.x0) / h)),
            int(round((y0 - grid.y0) / h)), int(round((y1 - grid.y0) / h)))


CASES = {"cylinder": (wl.cylinder_small, (0.7, 2.4, -0.8, 0.8), (1.5, 0.0)),
         "outflow": (wl.cylinder_outflow_small, (0.6, 3.1, -1.1, 0.9), (0.0, 0.0))}


@pytest.mark.parametrize("name", list(CASES))
def test_cv_terms_match_oracle(name):
    make, xy, origin = CASES[name]
    w = make()
    geo = OG.Geometry(w.grid, w.bodies)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 81, count=6), 0.0)
    G = wl.seeded_gammas(geo.nbc, 82, scale=0.3)
    box = _box(w.grid, *xy)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    d = to_dev(om)
    ctx.reconstruct(d, G, psi, U, V)
    got = ctx.cv_terms(d, U, V, box, origin)
    torch.cuda.synchronize()
    W = OL.fluid_weights(geo)
    # the kernels alone: the oracle's box integrals of the library's fields
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    St, Sg = OL.control_volume_terms(w.grid, om, Uh, Vh, box, origin)
    I, Sl = OL.cv_moment_terms(geo, om, Uh, Vh, box, origin, W)
    scale = max(np.abs(St).max(), np.abs(Sg).max())
    assert np.abs(got["S_t"] - St).max() < 1e-12 * scale, (got, St)
    assert np.abs(got["S_gamma"] - Sg).max() < 1e-12 * scale, (got, Sg)
    assert abs(got["I"] - I) < 1e-12 * abs(I), (got["I"], I)
    assert abs(got["S_lambda"] - Sl) < 1e-12 * abs(Sl), (got["S_lambda"], Sl)
    # end to end: from the oracle's reconstruction of the same state
    ref = Reconstructor(geo).reconstruct(om, G)
    St, Sg = OL.control_volume_terms(w.grid, om, ref.U, ref.V, box, origin)
    I, Sl = OL.cv_moment_terms(geo, om, ref.U, ref.V, box, origin, W)
    assert np.abs(got["S_t"] - St).max() < 1e-9 * scale
    assert np.abs(got["S_gamma"] - Sg).max() < 1e-9 * scale
    assert abs(got["I"] - I) < 1e-9 * abs(I)
    assert abs(got["S_lambda"] - Sl) < 1e-9 * abs(Sl)
    ctx.close()


def test_cv_box_checks():
    w = wl.cylinder_small()
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    om = torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0")
    U, V = ring_zeros(w.grid), ring_zeros(w.grid)
    nx, ny = w.grid.nx, w.grid.ny
    for box in [(0, 20, 5, 20), (5, nx - 1, 5, 20), (20, 10, 5, 20), (5, 20, 5, ny - 1)]:
        with pytest.raises(iim.IIMError) as e:
            ctx.cv_terms(om, U, V, box)
        assert e.value.code == iim.IIM_EINVAL
    # an edge through the cylinder (centre column of the body)
    ic = int(round((1.5 - w.grid.x0) / w.grid.h))
    with pytest.raises(iim.IIMError) as e:
        ctx.cv_terms(om, U, V, (ic, ic + 30, 10, 80))
    assert e.value.code == iim.IIM_EINVAL and "fluid" in str(e.value)
    ctx.close()
    # a rotating body inside the box: not a stationary wall
    b = dataclasses.replace(w.bodies[0], omega_rigid=0.5)
    ctx = iim.Context(w.grid, [b], solver=iim.SOLVER_DIRECT)
    with pytest.raises(iim.IIMError) as e:
        ctx.cv_terms(om, U, V, _box(w.grid, 0.7, 2.4, -0.8, 0.8))
    assert e.value.code == iim.IIM_EUNSUPPORTED
    ctx.close()
