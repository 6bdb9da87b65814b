"""FFT tile shapes (FFTs per workgroup of the row passes and of the column
pass, as the autotuner sets them) distribute the same arithmetic over
different workgroups: the Poisson operator and a reconstruction (correction
sources added in the column pass) must come out bitwise the same for every
shape."""
import numpy as np
import pytest
import torch

import workloads as wl
import paper_2109_13628_amd as iim
from oracle import geometry as OG
from gpu_util import to_dev, ring_zeros, seeded_state

pytestmark = pytest.mark.gpu

CASES = {"cyl_mid": wl.cylinder_mid, "cyl_outflow": wl.cylinder_outflow_small, "cyl_bench": wl.cylinder}
SHAPES = [(0, 0), (1, 1), (2, 2), (4, 4), (1, 4), (4, 1)]


@pytest.mark.parametrize("name", list(CASES))
def test_tile_shapes_do_not_change_results(name):
    w = CASES[name]()
    geo = OG.Geometry(w.grid, w.bodies)
    om, G = seeded_state(w, geo, 21)
    src = to_dev(np.random.default_rng(22).standard_normal((w.grid.ny, w.grid.nx)))
    omd = to_dev(om)
    ctx = iim.Context(w.grid, w.bodies, solver=iim.SOLVER_DIRECT)
    ref = None
    for r, c in SHAPES:
        ctx.set_fft_shape(r, c)
        p0 = ring_zeros(w.grid)
        ctx.poisson(src, p0)
        psi, U, V = ring_zeros(w.grid), ring_zeros(w.grid), ring_zeros(w.grid)
        ctx.reconstruct(omd, G, psi, U, V)
        torch.cuda.synchronize()
        out = [t.cpu().numpy() for t in (p0, psi, U, V)]
        if ref is None:
            ref = out
            continue
        for k, (a, b) in enumerate(zip(out, ref)):
            assert np.array_equal(a, b), (name, (r, c), k, np.max(np.abs(a - b)))
    ctx.close()
