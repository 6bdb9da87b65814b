"""The error gate of the FP64 path on developed flow: states injected from the
library's own run of the impulsively started cylinder (free space and
outflow) at steps 0, 1, 10 and 100, each advanced one RK3 step by the library
and by the oracle; omega, Gamma and the library's own reconstructed velocity,
in L2 and L-infinity, within ten times the oracle's measured rounding floor
on the same step.  The later states carry the thin boundary layer and the
near-wall vorticity gradients that a state built from smooth seeded vortices
does not."""
import functools

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle import ns as ONS
from gpu_util import to_dev, rel, step_errors, assert_within_floor

pytestmark = pytest.mark.gpu
STEPS = (0, 1, 10, 100)


@functools.lru_cache(maxsize=None)
def _run(name):
    w = wl.cylinder_small() if name == "free" else wl.cylinder_outflow_small()
    geo = OG.Geometry(w.grid, w.bodies)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    om = torch.zeros((w.grid.ny, w.grid.nx), dtype=torch.float64, device="cuda:0")
    G = np.zeros(ctx.n_circ)
    states, n = {}, 0
    for s in STEPS:
        if s > n:
            G, _ = ctx.rk3_steps(om, G, w.dt, s - n)
            n = s
        torch.cuda.synchronize()
        states[s] = (om.cpu().numpy().copy(), np.array(G, dtype=np.float64))
    return w, geo, ctx, states


# The oracle's rounding floor on the same steps (states of the oracle's own
# run): the larger of the spread between the free-space convolution on a 2n
# and on a 3n torus and the spread under a one-unit-roundoff change of the
# input omega.  Columns: omega L2, omega L-infinity, velocity L2, velocity
# L-infinity (relative), circulation (max |dGamma| / (1 + max |Gamma|)).
FLOOR = {
    ("free", 0): (4.3e-14, 4.7e-14, 3.9e-14, 1.7e-13, 1.5e-21),
    ("free", 1): (2.3e-14, 2.3e-14, 4.1e-14, 2.2e-13, 5.6e-20),
    ("free", 10): (1.5e-14, 2.4e-14, 4.1e-14, 1.9e-13, 1.2e-18),
    ("free", 100): (1.7e-14, 4.5e-14, 4.0e-14, 1.7e-13, 9.4e-17),
    ("outflow", 0): (1.4e-13, 1.5e-13, 1.1e-13, 3.7e-13, 6.9e-20),
    ("outflow", 1): (7.1e-14, 9.1e-14, 1.1e-13, 2.7e-13, 2.1e-19),
    ("outflow", 10): (2.9e-14, 4.7e-14, 1.1e-13, 2.6e-13, 7.2e-19),
    ("outflow", 100): (3.7e-14, 1.1e-13, 1.1e-13, 3.3e-13, 5.4e-17),
}


@pytest.mark.parametrize("step", STEPS)
@pytest.mark.parametrize("name", ["free", "outflow"])
def test_gate_on_injected_state(name, step):
    w, geo, ctx, states = _run(name)
    om, G = states[step]
    st = ONS.Stepper(geo)
    err = step_errors(ctx, st, geo, w, om, G)
    print(name, step, {k: v for k, v in err.items() if k != "stats"})
    assert_within_floor(err, FLOOR[(name, step)])
