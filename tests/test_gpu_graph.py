"""The direct-solver RK3 step replayed from a captured HIP graph equals the
eagerly launched step, replay after replay, with host work and
synchronisation between replays."""
import os

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from gpu_util import to_dev, seeded_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("make", [wl.cylinder_small, lambda: wl.taylor_couette(128)])
def test_graph_replays_match_eager(make):
    w = make()
    geo = OG.Geometry(w.grid, w.bodies)
    om, G = seeded_state(w, geo, 31)
    dt = w.dt
    ctx_g = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    os.environ["IIM_NO_GRAPH"] = "1"
    try:
        ctx_e = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    finally:
        del os.environ["IIM_NO_GRAPH"]
    a, b = to_dev(om), to_dev(om)
    Ga, Gb = G.copy(), G.copy()
    for rep in range(4):
        Ga, _ = ctx_g.rk3_steps(a, Ga, dt, 1)
        torch.cuda.synchronize()
        scratch = torch.randn(1000, device="cuda:0").sum().item()   # unrelated eager work
        Gb, _ = ctx_e.rk3_steps(b, Gb, dt, 1)
        torch.cuda.synchronize()
        assert torch.equal(a, b), rep
        assert np.array_equal(Ga, Gb), rep
    assert np.isfinite(scratch)
