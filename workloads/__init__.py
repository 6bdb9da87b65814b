"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module holds no arithmetic of the method itself: it only produces
boundary point sets (closed, ordered curves), grid descriptors, flow
parameters and seeded vorticity fields.  Both the FP64 oracle and the HIP
library consume these plain arrays/dicts; neither imports the other.

Conventions (shared by every consumer):
  * grid node (i, j) sits at (x0 + i*h, y0 + j*h); fields are stored [ny][nx];
  * a body is a closed polygon of boundary points, ordered so that the fluid
    lies to the RIGHT of the direction of travel (counter-clockwise for an
    obstacle, clockwise for an enclosing wall), first point not repeated;
  * rigid-motion boundary data: u_b(x) = u_rigid + omega_rigid * k x (x - center).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional, Tuple

import dataclasses

import numpy as np

EXT_BOX = "box"          # Dirichlet box (stream function zero on the box faces)
EXT_FREE = "free"        # unbounded domain
EXT_OUTFLOW = "outflow"  # unbounded, with an even mirror plane at the x_max face
EXT_PERIODIC = "periodic"  # periodic in both directions, u_inf = the mean velocity


@dataclass
class GridDesc:
    nx: int
    ny: int
    x0: float
    y0: float
    h: float
    exterior: str = EXT_FREE
    u_inf: Tuple[float, float] = (0.0, 0.0)
    nu: float = 0.01


@dataclass
class BodyDesc:
    points: np.ndarray                 # (P, 2) float64
    is_enclosure: bool = False
    center: Tuple[float, float] = (0.0, 0.0)
    u_rigid: Tuple[float, float] = (0.0, 0.0)
    omega_rigid: float = 0.0
    rect: Optional[Tuple[int, int, int, int]] = None   # (i0, i1, j0, j1) or None = automatic
    bc_samples: Optional[np.ndarray] = None            # (P, 3): u_x, u_y, psi_b at the points; None = rigid


@dataclass
class Workload:
    name: str
    grid: GridDesc
    bodies: List[BodyDesc]
    dt: float
    steps: int
    extra: dict = field(default_factory=dict)

    def describe(self) -> dict:
        g = asdict(self.grid)
        return {"workload": self.name, "nx": g["nx"], "ny": g["ny"], "h": g["h"],
                "exterior": g["exterior"], "nu": g["nu"], "u_inf": list(g["u_inf"]),
                "bodies": len(self.bodies), "dt": self.dt, "steps": self.steps}


# ----------------------------------------------------------------------------
# boundary point sets
# ----------------------------------------------------------------------------

def circle_points(center, radius, n, clockwise=False, phase=0.0):
    t = phase + 2.0 * np.pi * np.arange(n) / n
    if clockwise:
        t = -t
    return np.stack([center[0] + radius * np.cos(t), center[1] + radius * np.sin(t)], axis=1)


def ellipse_points(center, a, b, angle, n, phase=0.0):
    t = phase + 2.0 * np.pi * np.arange(n) / n
    ca, sa = math.cos(angle), math.sin(angle)
    x = a * np.cos(t)
    y = b * np.sin(t)
    return np.stack([center[0] + ca * x - sa * y, center[1] + sa * x + ca * y], axis=1)


def c_shape_points(center, ra, rb, theta_a, theta_b, n):
    """Counter-clockwise boundary of the set of points within rb of the circular
    arc of radius ra about `center`, starting at angle theta_a and spanning
    theta_b radians (round end caps).  Points are spaced uniformly in arc length.
    """
    cx, cy = center
    t_end = theta_a + theta_b
    # pieces: outer arc (ccw), end cap at t_end, inner arc (cw), start cap
    L_outer = (ra + rb) * theta_b
    L_inner = (ra - rb) * theta_b
    L_cap = math.pi * rb
    total = L_outer + L_inner + 2 * L_cap
    s = (np.arange(n) + 0.5) * total / n
    pts = np.empty((n, 2))
    for k, sk in enumerate(s):
        if sk < L_outer:
            a = theta_a + sk / (ra + rb)
            pts[k] = (cx + (ra + rb) * math.cos(a), cy + (ra + rb) * math.sin(a))
            continue
        sk -= L_outer
        if sk < L_cap:
            ex, ey = cx + ra * math.cos(t_end), cy + ra * math.sin(t_end)
            a = t_end + sk / rb
            pts[k] = (ex + rb * math.cos(a), ey + rb * math.sin(a))
            continue
        sk -= L_cap
        if sk < L_inner:
            a = t_end - sk / (ra - rb)
            pts[k] = (cx + (ra - rb) * math.cos(a), cy + (ra - rb) * math.sin(a))
            continue
        sk -= L_inner
        sx, sy = cx + ra * math.cos(theta_a), cy + ra * math.sin(theta_a)
        a = theta_a + math.pi + sk / rb
        pts[k] = (sx + rb * math.cos(a), sy + rb * math.sin(a))
    return pts


# ----------------------------------------------------------------------------
# named workloads (shapes and parameters of the paper's flows)
# ----------------------------------------------------------------------------

def step_size(h, nu, a, courant, diffusion):
    """The time step of a workload: dt = min(courant h / a, diffusion h^2 / nu),
    i.e. a chosen bound on the Courant number a dt / h and on the diffusion
    number nu dt / h^2 (an input of the run, picked well inside the explicit
    RK3 stability region)."""
    dt = diffusion * h * h / nu if nu > 0 else math.inf
    if a > 0:
        dt = min(dt, courant * h / a)
    return dt


def taylor_couette(n=128, points=256, steps=20):
    """Annulus between a rotating inner circle (r=0.25, omega=1) and a fixed outer
    wall (r=0.75), cell-centred n x n grid on [-1,1]^2, Dirichlet box."""
    h = 2.0 / n
    grid = GridDesc(nx=n, ny=n, x0=-1.0 + 0.5 * h, y0=-1.0 + 0.5 * h, h=h,
                    exterior=EXT_BOX, u_inf=(0.0, 0.0), nu=0.01)
    inner = BodyDesc(points=circle_points((0.0, 0.0), 0.25, points), center=(0.0, 0.0),
                     omega_rigid=1.0)
    outer = BodyDesc(points=circle_points((0.0, 0.0), 0.75, points, clockwise=True),
                     is_enclosure=True, center=(0.0, 0.0))
    # diffusion number 0.1418: the step 3.462e-3 of the 128 x 128 configuration
    a_max = math.sqrt(2.0) * 0.25
    dt = step_size(h, grid.nu, a_max, 0.6, 0.1418)
    return Workload("taylor_couette_%dx%d_box" % (n, n), grid, [inner, outer], dt, steps)


def cylinder(nx=1024, ny=512, h=1.0 / 64, points=256, nu=0.01, dt=0.0025, steps=1000,
             center=(2.0, 0.0), diameter=1.0, y_extent=None):
    """Impulsively started cylinder in free space, u_inf = (1, 0), cell-centred grid
    on [0, nx*h) x [-ny*h/2, ny*h/2)."""
    y0 = -0.5 * ny * h + 0.5 * h
    grid = GridDesc(nx=nx, ny=ny, x0=0.5 * h, y0=y0, h=h, exterior=EXT_FREE,
                    u_inf=(1.0, 0.0), nu=nu)
    body = BodyDesc(points=circle_points(center, 0.5 * diameter, points), center=center)
    return Workload("cylinder_Re%d_%dx%d_free" % (round(diameter / nu), nx, ny), grid,
                    [body], dt, steps)


def cylinder_small():
    """A small free-space cylinder case (D=1 at h=1/32, 128x96 nodes) that the
    oracle solves in seconds."""
    return cylinder(nx=128, ny=96, h=1.0 / 32, points=128, dt=0.005, steps=5,
                    center=(1.5, 0.0))


def cylinder_mid():
    """A free-space cylinder case (D=1 at h=1/32, 256x128 nodes) whose FFT
    sizes (512 x 256) take the register FFT kernels."""
    return cylinder(nx=256, ny=128, h=1.0 / 32, points=128, dt=0.005, steps=5,
                    center=(2.0, 0.0))


def two_c_shapes_lamb_oseen(n):
    """Two C-shaped bodies of the reconstruction convergence study on the unit
    square, x_ij = (i/n, j/n), free space."""
    h = 1.0 / n
    grid = GridDesc(nx=n, ny=n, x0=0.0, y0=0.0, h=h, exterior=EXT_FREE,
                    u_inf=(0.0, 0.0), nu=0.01)
    npts = max(256, int(8.0 / h))
    b1 = BodyDesc(points=c_shape_points((0.309, 0.679), 0.167, 0.057, 0.5, 1.8, npts),
                  center=(0.309, 0.679))
    b2 = BodyDesc(points=c_shape_points((0.559, 0.451), 0.157, 0.057, 3.7, 2.0, npts),
                  center=(0.559, 0.451))
    return Workload("lamb_oseen_two_c_%d" % n, grid, [b1, b2], dt=0.0, steps=0,
                    extra={"x0": (0.501, 0.501), "Gamma": 1.0, "nut": 0.0025})


# ----------------------------------------------------------------------------
# seeded fields
# ----------------------------------------------------------------------------

def node_coords(grid: GridDesc):
    x = grid.x0 + grid.h * np.arange(grid.nx)
    y = grid.y0 + grid.h * np.arange(grid.ny)
    return np.meshgrid(x, y)   # X[j, i], Y[j, i]


def seeded_vortices(grid: GridDesc, seed: int, count=6, box=None, amp=2.0, width=(0.05, 0.2)):
    """Sum of seeded Gaussian vortices, stored [ny][nx].  `box` = (xmin, xmax,
    ymin, ymax) restricts vortex centres; default: the middle of the grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = node_coords(grid)
    if box is None:
        xs = grid.x0 + grid.h * (grid.nx - 1)
        ys = grid.y0 + grid.h * (grid.ny - 1)
        box = (grid.x0 + 0.2 * (xs - grid.x0), xs - 0.2 * (xs - grid.x0),
               grid.y0 + 0.2 * (ys - grid.y0), ys - 0.2 * (ys - grid.y0))
    w = np.zeros((grid.ny, grid.nx))
    for _ in range(count):
        cx = rng.uniform(box[0], box[1])
        cy = rng.uniform(box[2], box[3])
        s = rng.uniform(width[0], width[1])
        a = rng.uniform(-amp, amp)
        w += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return w


def seeded_gammas(n_bodies: int, seed: int, scale=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=n_bodies)


def surface_driven_cylinder(nx=128, ny=96, h=1.0 / 32, points=128, center=(1.5, 0.0), speed=(0.5, 0.3, 3)):
    """A fixed cylinder (D = 1) whose surface moves tangentially with speed
    U(phi) = s0 + s1 sin(m phi) (phi: polar angle about the centre): boundary
    data given as samples at the boundary points (zero normal velocity, so
    psi_b is constant, here 0), in free stream u_inf = (1, 0)."""
    w = cylinder(nx=nx, ny=ny, h=h, points=points, dt=0.005, steps=5, center=center)
    pts = w.bodies[0].points
    phi = np.arctan2(pts[:, 1] - center[1], pts[:, 0] - center[0])
    s0, s1, m = speed
    U = s0 + s1 * np.sin(m * phi)
    samples = np.stack([-U * np.sin(phi), U * np.cos(phi), np.zeros_like(phi)], axis=1)
    body = dataclasses.replace(w.bodies[0], bc_samples=samples)
    return dataclasses.replace(w, name="surface_driven_cylinder_%dx%d" % (nx, ny), bodies=[body])


def periodic_cylinder(nx=128, ny=64, h=1.0 / 16, points=128, dt=0.01, center=(2.0, 0.0), mean=(1.0, 0.0),
                      diameter=1.0):
    """A cylinder (diameter D, 1 by default) in a box periodic in both
    directions (a row-and-column array of cylinders) with the mean velocity
    `mean`; cell-centred grid on [0, nx*h) x [-ny*h/2, ny*h/2); nx, ny powers
    of two."""
    w = cylinder(nx=nx, ny=ny, h=h, points=points, dt=dt, steps=5, center=center, diameter=diameter)
    w.grid.exterior = EXT_PERIODIC
    w.grid.u_inf = tuple(mean)
    w.name = "periodic_cylinder_%dx%d" % (nx, ny)
    return w


def cosine_wave_transport(n, nu, u=(1.0, 2.0), k=(4 * math.pi, 2 * math.pi)):
    """The transport study of Sec. 3 (its periodic case): the unit square,
    x_ij = (i/n, j/n), periodic in both directions, a C-shaped body (centre
    (0.507, 0.531), r_a 0.201, r_b 0.054, theta_a 0.5, theta_b 2.4), the
    uniform velocity u and the exact field omega = cos(k.(x - u t))
    exp(-nu |k|^2 t) (returned by extra['exact'](x, y, t)); dt at Courant number 0.8 (for
    the speed |u_x| + |u_y|) or diffusion number 0.12, whichever is smaller."""
    h = 1.0 / n
    grid = GridDesc(nx=n, ny=n, x0=0.0, y0=0.0, h=h, exterior=EXT_PERIODIC, u_inf=tuple(u), nu=nu)
    body = BodyDesc(points=c_shape_points((0.507, 0.531), 0.201, 0.054, 0.5, 2.4, max(256, int(8.0 / h))),
                    center=(0.507, 0.531), u_rigid=tuple(u))
    kk = k[0] * k[0] + k[1] * k[1]

    def exact(x, y, t):
        return np.cos(k[0] * (x - u[0] * t) + k[1] * (y - u[1] * t)) * math.exp(-nu * kk * t)

    dt = step_size(h, nu, abs(u[0]) + abs(u[1]), 0.8, 0.12)
    return Workload("cosine_wave_transport_%d" % n, grid, [body], dt, 0, extra={"exact": exact, "u": u})


def cylinder_outflow_small():
    """The small free-space cylinder with an outflow plane at the x_max face."""
    w = cylinder_small()
    w.grid.exterior = EXT_OUTFLOW
    w.name = w.name.replace("_free", "_outflow")
    return w


def side_by_side_cylinders(re=100.0, gap=3.0, d_over_h=64, length=30.0, height=12.0, points=512, dt=0.0025,
                           steps=80000):
    """A side-by-side cylinder pair (Sec. 6): two cylinders of diameter 1 with
    centres `gap` apart across a uniform stream U = 1, one diameter downstream
    of the inflow edge, on a cell-centred grid of length x height diameters
    with the outflow plane at the downstream face; nu = 1/Re.  The grid and
    the pair are mirror-symmetric about y = 0 (started from rest, the pair
    sheds in antiphase)."""
    h = 1.0 / d_over_h
    nx, ny = int(round(length / h)), int(round(height / h))
    grid = GridDesc(nx=nx, ny=ny, x0=0.5 * h, y0=-0.5 * ny * h + 0.5 * h, h=h, exterior=EXT_OUTFLOW,
                    u_inf=(1.0, 0.0), nu=1.0 / re)
    bodies = [BodyDesc(points=circle_points((1.0, c), 0.5, points), center=(1.0, c))
              for c in (-0.5 * gap, 0.5 * gap)]
    return Workload("side_by_side_Re%d_LD%g_%dx%d_outflow" % (round(re), gap, nx, ny), grid, bodies, dt, steps,
                    extra={"Re": re, "L/D": gap, "D/h": d_over_h})


def multi_body(n=2048, seed=3, steps=500):
    """Four seeded nonconvex/elongated bodies in a uniform stream on [0,1]^2
    with an outflow plane at x = 1: two ellipses (aspect 1.5-3) and two
    C-shaped arcs (gap angle 60-120 degrees), outer sizes 0.05-0.15, centres in
    [0.1,0.55] x [0.15,0.85], kept apart by rejection on their bounding
    circles.  Re ~ U[200, 1000] with nu = 0.1/Re (length scale 0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    re = rng.uniform(200.0, 1000.0)
    nu = 0.1 / re
    grid = GridDesc(nx=n, ny=n, x0=0.5 * h, y0=0.5 * h, h=h, exterior=EXT_OUTFLOW,
                    u_inf=(1.0, 0.0), nu=nu)
    placed = []          # (cx, cy, R)
    bodies = []
    kinds = ["ellipse", "ellipse", "c", "c"]
    for kind in kinds:
        for _ in range(1000):
            size = rng.uniform(0.05, 0.15)          # outer extent (diameter)
            R = 0.5 * size
            cx = rng.uniform(0.1, 0.55)
            cy = rng.uniform(0.15, 0.85)
            if all(np.hypot(cx - px, cy - py) > R + pR + 0.03 for (px, py, pR) in placed):
                break
        placed.append((cx, cy, R))
        if kind == "ellipse":
            aspect = rng.uniform(1.5, 3.0)
            a, b = R, R / aspect
            ang = rng.uniform(0.0, np.pi)
            per = np.pi * (3 * (a + b) - np.sqrt((3 * a + b) * (a + 3 * b)))
            pts = ellipse_points((cx, cy), a, b, ang, max(256, int(np.ceil(2 * per / h))))
        else:
            thick = rng.uniform(0.2, 0.35)           # thickness / centre-line radius
            ra = R / (1.0 + 0.5 * thick)             # outer radius = ra + rb = R
            rb = 0.5 * thick * ra
            gap = np.deg2rad(rng.uniform(60.0, 120.0))
            theta_a = rng.uniform(0.0, 2 * np.pi)
            theta_b = 2 * np.pi - gap
            per = 2 * np.pi * ra * 2 + 2 * np.pi * rb
            pts = c_shape_points((cx, cy), ra, rb, theta_a, theta_b, max(256, int(np.ceil(2 * per / h))))
        bodies.append(BodyDesc(points=pts, center=(cx, cy)))
    a_max = 2.0 * np.sqrt(2.0)
    dt = step_size(h, nu, a_max, 0.6, 0.1)
    return Workload("multi_body_%d_outflow_seed%d" % (n, seed), grid, bodies, dt, steps,
                    extra={"Re": re})


def batch_serving(n_sims=64, seed=5, nmin=256, nmax=1024, length=4.0):
    """Independent free-space simulations: square grids of N x N nodes with
    N uniform in [nmin, nmax] on a domain of side `length`, 1-6 seeded
    circles or ellipses each (semi-axes 0.12-0.3, aspect 1-2, placed apart),
    uniform inflow U = 1, Reynolds number uniform in [50, 500] on the mean
    body diameter, dt at Courant number 0.6 (speed 3) or diffusion number
    0.1, whichever is smaller."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in range(n_sims):
        n = int(rng.integers(nmin, nmax + 1))
        h = length / n
        nb = int(rng.integers(1, 7))
        bodies, placed = [], []
        tries = 0
        while len(bodies) < nb and tries < 2000:
            tries += 1
            a = rng.uniform(0.12, 0.3)
            b = a / rng.uniform(1.0, 2.0) if rng.uniform() < 0.5 else a
            cx = rng.uniform(0.7, length - 0.7)
            cy = rng.uniform(-length / 2 + 0.7, length / 2 - 0.7)
            if any(np.hypot(cx - px, cy - py) < a + pa + 0.3 for px, py, pa in placed):
                continue
            npts = max(64, int(2.5 * np.pi * a / h))
            if b == a:
                pts = circle_points((cx, cy), a, npts, phase=rng.uniform(0, 2 * np.pi))
            else:
                pts = ellipse_points((cx, cy), a, b, rng.uniform(0, np.pi), npts, phase=rng.uniform(0, 2 * np.pi))
            bodies.append(BodyDesc(points=pts, center=(cx, cy)))
            placed.append((cx, cy, a))
        D = 2.0 * float(np.mean([p[2] for p in placed]))
        re = rng.uniform(50.0, 500.0)
        nu = 1.0 * D / re
        grid = GridDesc(nx=n, ny=n, x0=0.0, y0=-length / 2, h=h, exterior=EXT_FREE, u_inf=(1.0, 0.0), nu=nu)
        dt = step_size(h, nu, 3.0, 0.6, 0.1)
        out.append(Workload(name="batch%d_%dx%d_%dbodies" % (s, n, n, len(bodies)), grid=grid, bodies=bodies,
                            dt=dt, steps=10, extra={"Re": re, "D": D}))
    return out
