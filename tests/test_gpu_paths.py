"""Alternative code paths that the library selects at context creation give
the default path's result: the chained boundary kernels (ghost psi,
velocity extension, omega_b, vorticity extensions in sequence; also the
fallback where the composed forms cannot be built), the LDS-only FFT
kernels, and eager steps instead of the captured step graph."""
import os

import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from gpu_util import to_dev, rel

pytestmark = pytest.mark.gpu


def _steps(w, om, G, env):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    d = to_dev(om)
    G1, _ = ctx.rk3_steps(d, np.array(G, dtype=np.float64), w.dt, 3)
    torch.cuda.synchronize()
    ctx.close()
    return d.cpu().numpy(), G1


@pytest.mark.parametrize("env", [{"IIM_CHAINED_BOUNDARY": "1"}, {"IIM_FFT_LDS_ONLY": "1"}, {"IIM_NO_GRAPH": "1"}])
def test_alternative_paths_match_default(env):
    w = wl.cylinder_mid()
    geo = OG.Geometry(w.grid, w.bodies)
    om = np.where(geo.fluid, 0.5 * wl.seeded_vortices(w.grid, 61, count=6), 0.0)
    G = wl.seeded_gammas(geo.nbc, 62, scale=0.3)
    ref, G_ref = _steps(w, om, G, {})
    got, G_got = _steps(w, om, G, env)
    assert rel(got, ref, mask=geo.fluid) < 1e-12, env
    assert np.max(np.abs(G_got - G_ref)) < 1e-12 * (np.abs(G_ref).max() + 1.0)
