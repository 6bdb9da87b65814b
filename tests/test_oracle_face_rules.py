"""Pins of the oracle's boundary-face rules of the advective flux (Sec. 3.2,
the 2D boundary-flux figure and its caption) and of its outflow mirror
(Sec. 5.2), independent of the oracle's own formulas.

Face rules: hand-built lines of node classes with integer vorticities, whose
fluxes were worked out by hand from the caption's five cases (upwind
direction to the left, flow to the right):
  (a) outflow face whose upwind stencil crosses the boundary at both ends,
  (b) fluid-fluid face whose upwind stencil reaches a ghost at its upwind end,
  (c) inflow face: downwind stencil, ghost at its upwind end,
  (d) inflow face whose downwind stencil crosses at both ends,
  (e) outflow face whose upwind stencil reaches a ghost at its downwind end;
a ghost at the upwind end of a stencil takes the extension with the wall
vorticity (E3b), one at the downwind end the extension without it (E3n), and
diffusion takes the fourth-order extension (E4b).  The stencils are
(-1/6, 5/6, 1/3) on (i-1, i, i+1) (upwind to the left) and (1/3, 5/6, -1/6)
on (i, i+1, i+2).  A swapped E3b/E3n, or the two-ghost upwind stencil at an
inflow face, changes every expected value below.

Outflow: the right-hand side with the outflow plane at the face x_{nx-1/2}
equals, at the last two columns, the free-space right-hand side of the
explicitly mirrored field on the doubled grid (vorticity and u_x even, u_y
odd about the plane)."""
import numpy as np
import pytest

import workloads as wl
from oracle import geometry as OG
from oracle import transport as OT

F, G, S = OG.FLUID, OG.GHOST, OG.SOLID


def _line(cls, w, e3b, e3n, e4b, u):
    """One row of the padded arrays _face_fluxes takes: ghosts carry their
    extensions, fluid nodes their vorticity; nu = h = 1."""
    cls = np.array([cls])
    ww = np.array([[float(v) for v in w]])
    b = np.array([[float(v) for v in e3b]])
    n = np.array([[float(v) for v in e3n]])
    q = np.array([[float(v) for v in e4b]])
    uu = np.array([[float(v) for v in u]])
    Fx, Qx = OT._face_fluxes(cls, ww, q, b, n, uu, 1.0, 1.0)
    # face between columns I and I+1 sits at index I - 1
    return (lambda I: Fx[0, I - 1]), (lambda I: Qx[0, I - 1])


# columns:   0  1   2  3   4  5   6   7   8   9  10  11
CLS_A = [S, G, F, G, S, G, F, F, F, F, G, S]
W_A = [0, 0, 12, 0, 0, 0, 6, 18, 24, 30, 0, 0]
E3B_A = [0, 6, 0, -48, 0, 12, 0, 0, 0, 0, -90, 0]
E3N_A = [0, -60, 0, 36, 0, -72, 0, 0, 0, 0, 42, 0]
E4B_A = [0, 100, 0, 200, 0, 300, 0, 0, 0, 0, 400, 0]
U_A = [0, 2, 1, 0.5, 0, 3, 1, 1, 1, 1, 1.5, 0]


def test_figure_cases_flow_to_the_right():
    Fx, Qx = _line(CLS_A, W_A, E3B_A, E3N_A, E4B_A, U_A)
    # (d) inflow face 1|2: downwind stencil on columns 1, 2, 3
    #     1/3 (2*6) + 5/6 (1*12) - 1/6 (0.5*36) = 4 + 10 - 3
    assert Fx(1) == pytest.approx(11.0, abs=1e-13)
    # (a) outflow face 2|3: upwind stencil on columns 1, 2, 3
    #     -1/6 (2*6) + 5/6 (12) + 1/3 (0.5*36) = -2 + 10 + 6
    assert Fx(2) == pytest.approx(14.0, abs=1e-13)
    # (c) inflow face 5|6: downwind stencil on columns 5, 6, 7
    #     1/3 (3*12) + 5/6 (6) - 1/6 (18) = 12 + 5 - 3
    assert Fx(5) == pytest.approx(14.0, abs=1e-13)
    # (b) fluid face 6|7: upwind stencil on columns 5, 6, 7
    #     -1/6 (3*12) + 5/6 (6) + 1/3 (18) = -6 + 5 + 6
    assert Fx(6) == pytest.approx(5.0, abs=1e-13)
    # interior face 7|8: -1/6 (6) + 5/6 (18) + 1/3 (24) = -1 + 15 + 8
    assert Fx(7) == pytest.approx(22.0, abs=1e-13)
    # (e) outflow face 9|10: upwind stencil on columns 8, 9, 10
    #     -1/6 (24) + 5/6 (30) + 1/3 (1.5*42) = -4 + 25 + 21
    assert Fx(9) == pytest.approx(42.0, abs=1e-13)
    # diffusion with E4b at the ghosts: Q = -(w_right - w_left)
    assert Qx(1) == pytest.approx(88.0) and Qx(2) == pytest.approx(-188.0)
    assert Qx(5) == pytest.approx(294.0) and Qx(6) == pytest.approx(-12.0)
    assert Qx(9) == pytest.approx(-370.0)
    # faces without a fluid endpoint carry nothing
    assert Fx(3) == 0.0 and Fx(4) == 0.0 and Qx(4) == 0.0


def test_figure_cases_flow_to_the_left():
    """The same line mirrored with the velocity reversed: the upwind side is
    now the right, and every flux changes sign at the mirrored face."""
    rev = lambda a: list(reversed(a))
    Fx, Qx = _line(rev(CLS_A), rev(W_A), rev(E3B_A), rev(E3N_A), rev(E4B_A), [-v for v in rev(U_A)])
    n = len(CLS_A)
    mirrored = lambda I: n - 2 - I        # face I|I+1 <-> face (n-2-I)|(n-1-I)
    for I, f, q in ((1, 11.0, 88.0), (2, 14.0, -188.0), (5, 14.0, 294.0), (6, 5.0, -12.0), (7, 22.0, None),
                    (9, 42.0, -370.0)):
        assert Fx(mirrored(I)) == pytest.approx(-f, abs=1e-13), I
        if q is not None:
            assert Qx(mirrored(I)) == pytest.approx(-q), I


def test_inflow_face_after_two_ghosts_takes_the_downwind_stencil():
    """Two ghosts in a row before the fluid (ghosts may neighbour each other
    along a line when both have fluid neighbours across it): the inflow face
    still uses the downwind stencil, which reaches one node past the
    boundary; the upwind stencil there would reach two."""
    # columns: 0  1  2  3  4  5  6  7  8
    cls = [S, G, G, F, F, F, G, G, S]
    w = [0, 0, 0, 6, 12, 18, 0, 0, 0]
    e3b = [0, 30, 24, 0, 0, 0, 48, 60, 0]
    e3n = [0, -30, -6, 0, 0, 0, -12, 66, 0]
    e4b = [0] * 9
    Fx, _ = _line(cls, w, e3b, e3n, e4b, [1.0] * 9)
    # inflow face 2|3: 1/3 (24) + 5/6 (6) - 1/6 (12) = 8 + 5 - 2 (the upwind
    # stencil on columns 1, 2, 3 would give -5 + 20 + 2 = 17)
    assert Fx(2) == pytest.approx(11.0, abs=1e-13)
    # outflow face 5|6: -1/6 (12) + 5/6 (18) + 1/3 (-12) = -2 + 15 - 4
    assert Fx(5) == pytest.approx(9.0, abs=1e-13)


def test_face_direction_from_the_extended_velocity():
    """The upwind side comes from the face velocity, the mean of the two
    node velocities, the ghost's extended one included: here the fluid node
    moves left but the face velocity points right, so the ghost face is an
    inflow face with E3b at its upwind (ghost) end."""
    cls = [S, G, F, F, F, F]
    w = [0, 0, 6, 12, 18, 24]
    e3b = [0, 30, 0, 0, 0, 0]
    e3n = [0, -30, 0, 0, 0, 0]
    u = [0, 1.0, -0.2, 0.5, 1, 1]
    Fx, _ = _line(cls, w, e3b, e3n, [0] * 6, u)
    # face velocity (1.0 - 0.2)/2 > 0: downwind stencil on columns 1, 2, 3
    #     1/3 (1*30) + 5/6 (-0.2*6) - 1/6 (0.5*12) = 10 - 1 - 1
    assert Fx(1) == pytest.approx(8.0, abs=1e-13)


def _outflow_case(nx=24, ny=20):
    h = 0.05
    grid = wl.GridDesc(nx=nx, ny=ny, x0=0.0, y0=0.0, h=h, exterior=wl.EXT_OUTFLOW, u_inf=(1.0, 0.0), nu=0.03)
    rng = np.random.default_rng(5)
    X, Y = wl.node_coords(grid)
    om = wl.seeded_vortices(grid, 17, count=5, box=(0.6, 1.1, 0.2, 0.8))
    # ring velocities (nodes -1..nx, -1..ny) of a smooth field, with the ring
    # column past the plane (node nx) even in u_x and odd in u_y
    xr = grid.x0 + h * np.arange(-1, nx + 1)
    yr = grid.y0 + h * np.arange(-1, ny + 1)
    XR, YR = np.meshgrid(xr, yr)
    # u_x changes sign along the plane, so that both stencils of the face
    # x_{nx-1/2} (and with them both mirrored nodes) are used
    U = 0.2 + 0.8 * np.cos(4 * YR + 0.3) + 0.2 * np.sin(3 * XR) + 0.05 * rng.standard_normal(XR.shape)
    V = 0.4 * np.cos(2 * XR) * np.sin(5 * YR) + 0.05 * rng.standard_normal(XR.shape)
    U[:, nx + 1] = U[:, nx]          # ring index nx+1 is node nx, mirror of node nx-1
    V[:, nx + 1] = -V[:, nx]
    return grid, om, U, V


def test_outflow_mirror_equals_explicit_mirror():
    grid, om, U, V = _outflow_case()
    nx, ny = grid.nx, grid.ny
    geo = OG.Geometry(grid, [])
    dw, _, _, _ = OT.rhs(geo, om, U, V, grid.nu, wb=np.zeros(0))
    # the doubled free-space grid with the mirror image written out
    g2 = wl.GridDesc(nx=2 * nx, ny=ny, x0=grid.x0, y0=grid.y0, h=grid.h, exterior=wl.EXT_FREE,
                     u_inf=grid.u_inf, nu=grid.nu)
    om2 = np.concatenate([om, om[:, ::-1]], axis=1)
    # ring of the doubled grid: node i' = 2nx-1-i mirrors node i (u even, v odd)
    U2 = np.zeros((ny + 2, 2 * nx + 2))
    V2 = np.zeros((ny + 2, 2 * nx + 2))
    U2[:, :nx + 1] = U[:, :nx + 1]
    V2[:, :nx + 1] = V[:, :nx + 1]
    for ip in range(nx, 2 * nx + 1):             # nodes nx .. 2nx (ring index ip+1)
        i = 2 * nx - 1 - ip
        U2[:, ip + 1] = U[:, i + 1]
        V2[:, ip + 1] = -V[:, i + 1]
    dw2, _, _, _ = OT.rhs(OG.Geometry(g2, []), om2, U2, V2, grid.nu, wb=np.zeros(0))
    last = slice(nx - 2, nx)
    face = U[1:-1, nx] + U[1:-1, nx + 1]
    assert np.any(face > 0) and np.any(face < 0)
    assert np.max(np.abs(dw[:, last] - dw2[:, last])) < 1e-12 * np.max(np.abs(dw2[:, last]))
    # the plane matters: without the mirror (plain free space) the last
    # columns differ
    gf = wl.GridDesc(nx=nx, ny=ny, x0=grid.x0, y0=grid.y0, h=grid.h, exterior=wl.EXT_FREE,
                     u_inf=grid.u_inf, nu=grid.nu)
    dwf, _, _, _ = OT.rhs(OG.Geometry(gf, []), om, U, V, grid.nu, wb=np.zeros(0))
    assert np.max(np.abs(dwf[:, last] - dw2[:, last])) > 1e-3 * np.max(np.abs(dw2[:, last]))
