"""Helpers shared by the GPU parity tests (oracle on the CPU, library on cuda:0)."""
import numpy as np
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from oracle.reconstruct import Reconstructor
from oracle import transport as OT
from oracle import ns as ONS

DEV = torch.device("cuda:0")


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def ring_zeros(grid):
    return torch.zeros((grid.ny + 2, grid.nx + 2), dtype=torch.float64, device=DEV)


def seeded_state(w, geo, seed, body_scale=None):
    """Seeded vorticity (zero in the solid) and circulations of the workload's
    shape.  body_scale: place vortices of the body's size within a few body
    sizes of the first body (a wake-like state) instead of domain-sized blobs."""
    if body_scale is not None:
        cx, cy = np.mean(w.bodies[0].points, axis=0)
        D = body_scale
        om = wl.seeded_vortices(w.grid, seed, count=8, amp=3.0,
                                box=(cx - 1.0 * D, cx + 4.0 * D, cy - 1.5 * D, cy + 1.5 * D),
                                width=(0.05 * D, 0.25 * D))
        om = np.where(geo.fluid, om, 0.0)
        return om, wl.seeded_gammas(geo.nbc, seed + 1, scale=0.5)
    xs = w.grid.x0 + w.grid.h * (w.grid.nx - 1)
    ys = w.grid.y0 + w.grid.h * (w.grid.ny - 1)
    om = wl.seeded_vortices(w.grid, seed, count=8, amp=3.0,
                            box=(w.grid.x0 + 0.1 * (xs - w.grid.x0), xs - 0.3 * (xs - w.grid.x0),
                                 w.grid.y0 + 0.25 * (ys - w.grid.y0), ys - 0.25 * (ys - w.grid.y0)),
                            width=(0.03 * (xs - w.grid.x0), 0.08 * (xs - w.grid.x0)))
    om = np.where(geo.fluid, om, 0.0)
    G = wl.seeded_gammas(geo.nbc, seed + 1, scale=0.5)
    return om, G


def rel(a, b, mask=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a, b = a[mask], b[mask]
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d
