"""Status codes of the step calls on the GPU: a NaN or Inf in the new state
is reported as IIM_ENONFINITE on every solver path (the dense solver's
captured step graph included, and the batch), a time step above the
stability limit is refused with IIM_EINVAL before anything runs, and the
context keeps working after either."""
import numpy as np
import pytest
import torch

import paper_2109_13628_amd as iim
import workloads as wl
from oracle import geometry as OG
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("solver", [iim.SOLVER_DIRECT, iim.SOLVER_KRYLOV])
def test_nonfinite_reported_on_every_path(solver):
    w = wl.cylinder_small()
    geo = OG.Geometry(w.grid, w.bodies)
    om0 = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 4, count=4), 0.0)
    ctx = iim.Context(w.grid, w.bodies, solver=solver, tol=1e-12)
    d = to_dev(om0)
    G, _ = ctx.rk3_steps(d, np.array([0.1]), w.dt, 2)     # the direct path captures its step graph here
    torch.cuda.synchronize()
    assert torch.isfinite(d).all()
    bad = d.clone()
    bad[w.grid.ny // 2, 3] = float("inf")
    with pytest.raises(iim.IIMError) as e:
        ctx.rk3_steps(bad, G.copy(), w.dt, 1)
    assert e.value.code in (iim.IIM_ENONFINITE,), e.value
    # the flag was cleared: a finite state steps normally afterwards
    G2, _ = ctx.rk3_steps(d, G.copy(), w.dt, 1)
    torch.cuda.synchronize()
    assert torch.isfinite(d).all() and np.all(np.isfinite(G2))
    ctx.close()


def test_step_above_stability_limit_refused():
    w = wl.cylinder_small()
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    lim = ctx.dt_limit()
    assert w.dt < lim
    d = to_dev(np.zeros((w.grid.ny, w.grid.nx)))
    with pytest.raises(iim.IIMError) as e:
        ctx.rk3_steps(d, np.zeros(1), 1.01 * lim, 1)
    assert e.value.code == iim.IIM_EINVAL and "stability limit" in str(e.value)
    torch.cuda.synchronize()
    assert float(d.abs().max()) == 0.0          # nothing ran
    G, _ = ctx.rk3_steps(d, np.zeros(1), w.dt, 1)
    torch.cuda.synchronize()
    assert float(d.abs().max()) > 0.0           # impulsive start: vorticity appears at the wall
    ctx.close()


def test_batch_status_codes():
    ws = wl.batch_serving(3, seed=11, nmin=120, nmax=200)
    b = iim.Batch(ws)
    oms = [torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0") for w in ws]
    Gs = [np.zeros(len(w.bodies)) for w in ws]
    dts = [w.dt for w in ws]
    b.step(oms, Gs, dts, 1)
    # a time step above one simulation's limit: refused, nothing runs
    big = list(dts)
    big[1] = 100.0 * dts[1]
    before = [o.clone() for o in oms]
    with pytest.raises(iim.IIMError) as e:
        b.step(oms, Gs, big, 1)
    assert e.value.code == iim.IIM_EINVAL and "simulation 1" in str(e.value)
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(oms, before))
    # a NaN in one simulation's state: reported with that simulation named
    oms[2][ws[2].grid.ny // 2, 2] = float("nan")
    with pytest.raises(iim.IIMError) as e:
        b.step(oms, Gs, dts, 1)
    assert e.value.code == iim.IIM_ENONFINITE and "simulation 2" in str(e.value)
    oms[2].zero_()
    Gs[2][:] = 0.0
    st = b.step(oms, Gs, dts, 1)
    torch.cuda.synchronize()
    assert st["steps"] == 1 and all(bool(torch.isfinite(o).all()) for o in oms)
    b.close()
