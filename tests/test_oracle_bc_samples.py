"""Prescribed boundary data (samples of u_x, u_y, psi_b at the boundary points)
in the oracle, pinned without the oracle's own formulas:

* spline interpolation is linear in the data and the control point lies on
  the coordinate spline at the same parameter, so samples of any field that
  is linear in the point coordinates come out exactly (to rounding) as that
  field at the control point: a rigid translation (velocity and stream
  function) and the velocity of a rigid rotation;
* for a smooth non-linear field the interpolation error falls at the cubic
  spline's fourth order as the points double;
* the library's host-only geometry reproduces the oracle's boundary data."""
import dataclasses

import numpy as np

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG


def _with_samples(w, fn):
    b = w.bodies[0]
    p = b.points
    return dataclasses.replace(w, bodies=[dataclasses.replace(b, bc_samples=fn(p[:, 0], p[:, 1]))])


def test_samples_of_a_translation_are_exact():
    U = (0.7, -0.3)
    w = _with_samples(wl.cylinder_small(),
                      lambda x, y: np.stack([np.full_like(x, U[0]), np.full_like(x, U[1]), U[0] * y - U[1] * x], 1))
    g = OG.Geometry(w.grid, w.bodies)
    assert np.max(np.abs(g.c_ub[:, 0] - U[0])) < 1e-14
    assert np.max(np.abs(g.c_ub[:, 1] - U[1])) < 1e-14
    assert np.max(np.abs(g.c_psib - (U[0] * g.c_y - U[1] * g.c_x))) < 1e-13


def test_samples_of_a_rotation_velocity_are_exact():
    Om, (cx, cy) = 1.3, wl.cylinder_small().bodies[0].center
    w = _with_samples(wl.cylinder_small(),
                      lambda x, y: np.stack([-Om * (y - cy), Om * (x - cx), np.zeros_like(x)], 1))
    g = OG.Geometry(w.grid, w.bodies)
    assert np.max(np.abs(g.c_ub[:, 0] + Om * (g.c_y - cy))) < 1e-13
    assert np.max(np.abs(g.c_ub[:, 1] - Om * (g.c_x - cx))) < 1e-13


def test_interpolation_converges_at_fourth_order():
    errs = []
    for P in (64, 128):
        w = wl.surface_driven_cylinder(points=P)
        g = OG.Geometry(w.grid, w.bodies)
        cx, cy = w.bodies[0].center
        phi = np.arctan2(g.c_y - cy, g.c_x - cx)
        U = 0.5 + 0.3 * np.sin(3 * phi)
        exact = np.stack([-U * np.sin(phi), U * np.cos(phi)], 1)
        errs.append(np.max(np.abs(g.c_ub - exact)))
        assert np.max(np.abs(g.c_psib)) == 0.0
    assert errs[1] < errs[0] / 10.0, errs


def test_library_boundary_data_matches_oracle():
    for w in (wl.surface_driven_cylinder(), wl.cylinder_small()):
        ctx = iim.Context(w.grid, w.bodies, host_only=True)
        geo = ctx.geometry()
        ref = OG.Geometry(w.grid, w.bodies)
        assert np.max(np.abs(geo["c_ub"] - ref.c_ub)) < 1e-12
        assert np.max(np.abs(geo["c_psib"] - ref.c_psib)) < 1e-12
        ctx.close()
