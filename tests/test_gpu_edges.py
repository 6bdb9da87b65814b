"""Edge cases on the GPU: no immersed body (no correction unknowns), a ragged
rectangular grid with the outflow exterior, device-side error paths (grid too
large for the FFT plan, non-finite vorticity, zero steps)."""
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


def _no_body_grid():
    # ragged sizes (200 x 150; FFT 512 x 512), free stream at an angle
    return wl.GridDesc(nx=200, ny=150, x0=-1.0, y0=-0.75, h=0.01, exterior="free", u_inf=(0.3, 0.1), nu=0.01)


@pytest.mark.parametrize("solver", [iim.SOLVER_KRYLOV, iim.SOLVER_DIRECT])
def test_no_bodies(solver):
    g = _no_body_grid()
    geo = OG.Geometry(g, [])
    om = wl.seeded_vortices(g, 3, count=4)
    dt = 0.002
    om_ref, _ = ONS.Stepper(geo).step(om, np.zeros(0), dt)
    ctx = iim.Context(g, [], solver=solver)
    assert ctx.n_circ == 0 and ctx.info["n_affected"] == 0
    d = to_dev(om)
    G, st = ctx.rk3_steps(d, np.zeros(0), dt, 2 if solver == iim.SOLVER_DIRECT else 1)
    torch.cuda.synchronize()
    if solver == iim.SOLVER_KRYLOV:
        assert rel(d.cpu().numpy(), om_ref) < TOL64
        assert st["iters"] == [0, 0, 0]
    # velocity of the same state
    psi, U, V = ring_zeros(g), ring_zeros(g), ring_zeros(g)
    ctx.reconstruct(to_dev(om), np.zeros(0), psi, U, V)
    torch.cuda.synchronize()
    ref = Reconstructor(geo).reconstruct(om, np.zeros(0))
    fl = np.pad(geo.fluid, 1)
    assert rel(np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]]), np.stack([ref.U[fl], ref.V[fl]])) < TOL64


def test_ragged_outflow_grid():
    # 300 x 170 nodes: FFT torus 2048 x 512 with the mirrored outflow source
    w = wl.cylinder(nx=300, ny=170, h=1.0 / 32, points=128, dt=0.005, steps=2, center=(2.5, 0.0))
    w = dataclasses.replace(w, grid=dataclasses.replace(w.grid, exterior=wl.EXT_OUTFLOW))
    geo = OG.Geometry(w.grid, w.bodies)
    rng = np.random.default_rng(8)
    om = np.where(geo.fluid, wl.seeded_vortices(w.grid, 12, count=6), 0.0)
    G = rng.uniform(-0.3, 0.3, size=geo.nbc)
    ref = Reconstructor(geo).reconstruct(om, G)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    ctx.reconstruct(to_dev(om), G, psi, U, V)
    torch.cuda.synchronize()
    fl = np.pad(geo.fluid, 1)
    e = rel(np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]]), np.stack([ref.U[fl], ref.V[fl]]))
    assert e < TOL64, e


def test_device_error_paths():
    # FFT plan limit: mx / 2 <= 4096
    g = wl.GridDesc(nx=4200, ny=64, x0=0.0, y0=0.0, h=0.01, exterior="free", u_inf=(1.0, 0.0), nu=0.01)
    with pytest.raises(iim.IIMError) as e:
        iim.Context(g, [])
    assert e.value.code == iim.IIM_EINVAL
    w = wl.cylinder_small()
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_KRYLOV, tol=1e-12)
    om = torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0")
    # zero steps: nothing changes
    G, _ = ctx.rk3_steps(om, np.array([0.25]), w.dt, 0)
    assert float(G[0]) == 0.25 and float(om.abs().max()) == 0.0
    # non-positive dt
    with pytest.raises(iim.IIMError) as e:
        ctx.rk3_steps(om, np.zeros(1), 0.0, 1)
    assert e.value.code == iim.IIM_EINVAL
    # a NaN in the vorticity reaches the Krylov residual and is reported
    om[w.grid.ny // 2, 5] = float("nan")
    with pytest.raises(iim.IIMError) as e:
        ctx.rk3_steps(om, np.zeros(1), w.dt, 1)
    assert e.value.code == iim.IIM_ENONFINITE


def test_krylov_limit_reports_no_convergence():
    """An iteration limit below what the tolerance needs: IIM_ENOCONV, with the
    statistics filled and the (unconverged) result written."""
    w = wl.cylinder_small()
    geo = OG.Geometry(w.grid, w.bodies)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 5, count=5), 0.0)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_KRYLOV, tol=1e-13, max_iter=3,
                      guess=iim.GUESS_ZERO)
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    st = ctx.reconstruct(to_dev(om), np.array([0.1]), psi, U, V, allow_noconv=True)
    torch.cuda.synchronize()
    assert st["converged"] == 0 and 1 <= st["iters"][0] <= 3, st
    assert 1e-13 < st["res"][0] < st["res0"][0], st
    assert np.all(np.isfinite(U.cpu().numpy())) and np.abs(U.cpu().numpy()).max() > 0
    d = to_dev(om)
    with pytest.raises(iim.IIMError) as e:
        ctx.rk3_steps(d, np.array([0.1]), w.dt, 1)
    assert e.value.code == iim.IIM_ENOCONV
    ctx.close()


def test_binding_refuses_undersized_device_tensors():
    """Grid fields [ny][nx], ring fields [ny+2][nx+2] and per-control-point
    arrays smaller than the kernels index are refused before any launch."""
    import numpy as _np
    import torch as _torch
    import workloads as _wl
    import paper_2109_13628_amd as _iim
    w = _wl.cylinder_small()
    g = w.grid
    ctx = _iim.Context(g, w.bodies, solver=_iim.SOLVER_DIRECT)
    z = lambda *s: _torch.zeros(s, dtype=_torch.float64, device="cuda:0")
    om, ring, small = z(g.ny, g.nx), z(g.ny + 2, g.nx + 2), z(g.ny, g.nx - 1)
    G = _np.zeros(ctx.n_circ)
    with pytest.raises(ValueError, match="ring"):
        ctx.reconstruct(om, G, None, om, ring)        # a grid-sized tensor where a ring is needed
    with pytest.raises(ValueError, match="grid"):
        ctx.rk3_steps(small, G, w.dt, 1)
    with pytest.raises(ValueError, match="control"):
        ctx.rhs_given_wb(om, ring, ring, z(max(0, ctx.info["n_control"] - 1)), om)
    ctx.reconstruct(om, G, None, ring, z(g.ny + 2, g.nx + 2))   # the right sizes still run
    _torch.cuda.synchronize()
    ctx.close()
