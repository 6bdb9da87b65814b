"""GPU vs oracle at the benchmark size (1024 x 512 free-space cylinder, FFT
torus 2048 x 1024), in the launch configuration bench.py times."""
import functools

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle import poisson as OP
from oracle.reconstruct import Reconstructor
from oracle import ns as ONS
from gpu_util import DEV, to_dev, ring_zeros, seeded_state, rel, step_errors, assert_within_floor, oracle_step

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _setup(name):
    if name.startswith("multi"):
        w = wl.multi_body(int(name[5:]))
    elif name == "cyl1024":
        w = wl.cylinder()
    else:
        w = wl.cylinder(nx=512, ny=256, h=1.0 / 32, points=256, dt=0.005)
    geo = OG.Geometry(w.grid, w.bodies)
    return w, geo, ONS.Stepper(geo)


@functools.lru_cache(maxsize=None)
def _reference(name):
    """The seeded wake-like state of the case and the oracle's step from it."""
    w, geo, st = _setup(name)
    om, G = seeded_state(w, geo, 21, body_scale=1.0 if name.startswith("cyl") else 0.1)
    return om, G, oracle_step(st, w, om, G)


@pytest.mark.parametrize("name", ["cyl512", "cyl1024"])
def test_poisson_fullsize(name):
    w, geo, st = _setup(name)
    rng = np.random.default_rng(2)
    src = rng.standard_normal((w.grid.ny, w.grid.nx))
    ctx = iim.Context(w.grid, w.bodies)
    psi = ring_zeros(w.grid)
    ctx.poisson(to_dev(src), psi)
    torch.cuda.synchronize()
    ref = st.rec._fs(src)
    assert rel(psi.cpu().numpy(), ref) < 1e-13


# Rounding floors of the oracle itself on these states (one RK3 step from the
# seeded state), the largest of three measured spreads: (1) the free-space
# convolution on a 3n torus instead of 2n (the same operator in exact
# arithmetic, different rounding), with the dense Schur matrix built from that
# operator's columns; (2) the Schur solves by dense LU against GMRES to
# 1e-15, or against LU refined with long-double residuals; (3) the input
# omega changed by one unit roundoff per node.  Columns: omega L2, omega
# L-infinity, velocity L2, velocity L-infinity (relative to the oracle's
# result), circulation (max |dGamma| / (1 + max |Gamma|)).
FLOOR = {
    "cyl512": (3.2e-13, 3.4e-13, 2.7e-13, 7.2e-13, 2.4e-17),
    "cyl1024": (1.0e-12, 1.7e-12, 8.6e-13, 4.3e-12, 0.0),
    "multi512": (4.1e-11, 3.3e-11, 1.8e-11, 6.8e-11, 3.9e-17),
    # four nonconvex bodies, outflow, 1024 x 1024 (FFT torus 4096 x 2048);
    # floors (1) and (3) only: the GMRES-to-1e-15 floor takes too long here
    "multi1024": (1.3e-10, 1.4e-10, 8.0e-11, 3.8e-10, 1.2e-16),
}


@pytest.mark.parametrize("solver", [iim.SOLVER_DIRECT, iim.SOLVER_KRYLOV])
@pytest.mark.parametrize("name", ["cyl512", "cyl1024", "multi512", "multi1024"])
def test_step_fullsize(name, solver):
    """One RK3 step from a seeded wake-like state, library against oracle:
    omega, Gamma and the library's own reconstructed velocity, each in L2
    and L-infinity, within ten times the oracle's measured rounding floor."""
    w, geo, st = _setup(name)
    om, G, ref = _reference(name)
    # GMRES to 1e-13 on one body; the four-body system (nonconvex C-shapes,
    # 1-norm condition number 6e11) stops at 1e-12
    tol = 1e-12 if name.startswith("multi") else 1e-13
    ctx = iim.Context(w.grid, w.bodies, tol=tol, solver=solver)
    err = step_errors(ctx, st, geo, w, om, G, ref)
    print(name, solver, {k: v for k, v in err.items() if k != "stats"}, err["stats"])
    assert_within_floor(err, FLOOR[name])
    ctx.close()


def test_step_repeatable_multi1024():
    """The same RK3 steps run twice from the same state agree bit for bit:
    every sum of the step (block reductions, the dense product's ordered
    partial sums) adds its terms in a fixed order."""
    w, geo, st = _setup("multi1024")
    om, G = seeded_state(w, geo, 21, body_scale=0.1)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    out = []
    for _ in range(2):
        d = to_dev(om)
        G1, _ = ctx.rk3_steps(d, np.array(G, dtype=np.float64), w.dt, 3)
        torch.cuda.synchronize()
        out.append((d.cpu().numpy(), np.array(G1)))
    ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
