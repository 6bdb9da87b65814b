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


def linf_rel(a, b, mask=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a, b = a[mask], b[mask]
    n = np.max(np.abs(b))
    d = np.max(np.abs(a - b))
    return d / n if n > 0 else d


def oracle_step(st, w, om, G):
    """The oracle's RK3 step and its velocity reconstruction."""
    om_ref, G_ref = st.step(om, G, w.dt)
    return om_ref, G_ref, st.rec.reconstruct(om_ref, G_ref)


def step_errors(ctx, st, geo, w, om, G, ref=None):
    """One RK3 step of the library (ctx, on the device) and of the oracle
    (st, or its result `ref` from oracle_step) from the same state, and the library's own velocity reconstruction
    of its result against the oracle's reconstruction of the oracle's result:
    relative L2 and L-infinity errors of omega (fluid nodes) and of (u, v)
    (fluid nodes of the grid and its ring), and the largest circulation
    error with the size of the circulations."""
    om_ref, G_ref, b = ref if ref is not None else oracle_step(st, w, om, G)
    d = to_dev(om)
    G1, stats = ctx.rk3_steps(d, np.array(G, dtype=np.float64), w.dt, 1)
    psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
    ctx.reconstruct(d, G1, psi, U, V)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    fl = np.pad(geo.fluid, 1)
    uv = np.stack([U.cpu().numpy()[fl], V.cpu().numpy()[fl]])
    uv_ref = np.stack([b.U[fl], b.V[fl]])
    return {"omega_l2": rel(got, om_ref, geo.fluid), "omega_linf": linf_rel(got, om_ref, geo.fluid),
            "vel_l2": rel(uv, uv_ref), "vel_linf": linf_rel(uv, uv_ref),
            "gamma_abs": float(np.max(np.abs(G1 - G_ref))) if len(G_ref) else 0.0,
            "gamma_max": float(np.max(np.abs(G_ref))) if len(G_ref) else 0.0, "stats": stats}


def assert_within_floor(err, floor, factor=10.0):
    """err (from step_errors) against `factor` times the measured rounding
    floor: floor = (omega L2, omega Linf, velocity L2, velocity Linf,
    circulation), the first four relative to the oracle's result, the last
    relative to 1 + max |Gamma| and never below one unit in the last place of
    max |Gamma|."""
    names = ("omega_l2", "omega_linf", "vel_l2", "vel_linf")
    bad = {k: (err[k], factor * f) for k, f in zip(names, floor[:4]) if not err[k] <= factor * f}
    g_floor = max(floor[4] * (1.0 + err["gamma_max"]), float(np.spacing(err["gamma_max"])))
    if not err["gamma_abs"] <= factor * g_floor:
        bad["gamma_abs"] = (err["gamma_abs"], factor * g_floor)
    assert not bad, (bad, {k: err[k] for k in names})
