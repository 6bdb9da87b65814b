"""Pins of the oracle's lattice Green's function (free-space exact inverse of
the 5-point Laplacian, Sec. 4.2) against closed forms and the defining
equation."""
import json
import os

import numpy as np
import pytest

from oracle import lgf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _full(g):
    """Mirror a quadrant table g[n, m] (m, n >= 0) to all signs."""
    top = np.concatenate([g[:, :0:-1], g], axis=1)
    return np.concatenate([top[:0:-1, :], top], axis=0)


def test_exact_resistances():
    spec = json.load(open(os.path.join(GOLD, "lgf_exact.json")))
    g = lgf.lgf_table(4, 4)
    pi = np.pi
    for v in spec["values"]:
        exact = eval(v["R"], {"__builtins__": {}}, {"pi": np.pi})
        assert abs(-2.0 * g[v["n"], v["m"]] - exact) < 2e-15, v


def test_delta_residual_and_symmetry():
    n = 48
    g = lgf.lgf_table(n, n)
    assert np.allclose(g, g.T, atol=0, rtol=0) or np.max(np.abs(g - g.T)) < 1e-15
    f = _full(g)
    lap = f[1:-1, 2:] + f[1:-1, :-2] + f[2:, 1:-1] + f[:-2, 1:-1] - 4 * f[1:-1, 1:-1]
    res = -lap
    c = n - 1
    res[c, c] -= 1.0
    assert np.max(np.abs(res)) < 5e-15


@pytest.mark.parametrize("m,n", [(40, 0), (30, 30), (60, 17), (25, 48)])
def test_far_field(m, n):
    g = lgf.lgf_table(max(m, n), max(m, n))
    r = np.hypot(m, n)
    # next term of the expansion is O(r^-4)
    assert abs(g[n, m] - lgf.lgf_far_field(m, n)) < 0.1 / r ** 4


def test_rectangular_table_matches_square():
    a = lgf.lgf_table(20, 7)
    b = lgf.lgf_table(20, 20)
    assert np.array_equal(a, b[:8, :21])
