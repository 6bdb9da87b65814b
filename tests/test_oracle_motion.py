"""Time-dependent rigid motion in the oracle: the boundary data follow the
motion at each RK3 stage's time (stages at 0, 1/3 and 3/4 of the step, from
the step's own recurrences applied to the time).

* a constant schedule reproduces the body's fixed rigid rotation exactly;
* the Lamb-Oseen vortex on its co-rotating cylinder (an exact Navier-Stokes
  solution, the paper's convergence case of Sec. 6) from t = 1 to 1.05 at
  N = 32, 64, 128: the velocity error converges at second order and the
  vorticity error decreases;
* the wall-vorticity stencils on the exact velocity of that vortex: second
  order."""
import dataclasses

import numpy as np

from oracle import geometry as OG
from oracle import ns as ONS
import e3_lamb_oseen as E3


def test_stage_times():
    assert np.allclose(ONS.rk3_stage_times(), [0.0, 1.0 / 3.0, 0.75], rtol=0, atol=1e-15)


def test_constant_schedule_equals_fixed_rotation():
    grid, body = E3.case(48, 1.0)
    geo = OG.Geometry(grid, [body])
    om, G = E3.initial(grid, geo.fluid, geo.rects[0], 1.0)
    st = ONS.Stepper(geo)
    a = st.step(om, G, 2e-3)
    geo2 = OG.Geometry(grid, [dataclasses.replace(body, omega_rigid=0.0)])
    st2 = ONS.Stepper(geo2)
    b = st2.step(om, G, 2e-3, motion=lambda t: [(0.0, 0.0, body.omega_rigid)], t=1.0)
    assert np.max(np.abs(a[0] - b[0])) < 1e-13 * np.abs(a[0]).max()
    assert abs(a[1][0] - b[1][0]) < 1e-13


def _run(n, t0=1.0, t1=1.05):
    grid, body = E3.case(n, t0)
    geo = OG.Geometry(grid, [body])
    om, G = E3.initial(grid, geo.fluid, geo.rects[0], t0)
    steps, dt = E3.time_step(ONS.dt_max(grid.h, grid.nu, E3.a_max(t0)), t0, t1)
    st = ONS.Stepper(geo)
    mot = lambda t: [(0.0, 0.0, E3.rotation(t))]
    for k in range(steps):
        om, G = st.step(om, G, dt, motion=mot, t=t0 + k * dt)
    st.set_motion(mot(t1))
    rec = st.rec.reconstruct(om, G)
    return E3.errors(grid, geo.fluid, om, rec.U, rec.V, t1)


def test_lamb_oseen_on_rotating_cylinder_converges():
    e = [_run(n) for n in (32, 64, 128)]
    for a, b in zip(e[:-1], e[1:]):
        assert np.log2(a[2] / b[2]) > 1.9, e        # velocity L2
        assert np.log2(a[3] / b[3]) > 1.5, e        # velocity Linf
        assert b[0] < a[0] and b[1] < a[1], e       # vorticity


def test_wall_vorticity_stencil_second_order_on_the_exact_vortex():
    """The boundary-vorticity stencils applied to the exact velocity of the
    vortex (wall vorticity 0.90, a small difference of velocity derivatives of
    size 22): second order."""
    from oracle.transport import boundary_vorticity
    t = 1.0
    wex = E3.G0 / (4 * np.pi * E3.NU * t) * np.exp(-E3.R ** 2 / (4 * E3.NU * t))
    err = []
    for n in (64, 128, 256):
        grid, body = E3.case(n, t)
        geo = OG.Geometry(grid, [body])
        xs = grid.h * np.arange(-1, n + 1)
        X, Y = np.meshgrid(xs, xs)
        _, U, V = E3.exact(X, Y, t)
        err.append(np.abs(boundary_vorticity(geo, U, V) - wex).mean())
    assert np.log2(err[1] / err[2]) > 1.8, err
