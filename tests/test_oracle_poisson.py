"""Pins of the oracle's solution operators G = (-lap_h)^-1 (Sec. 4.2)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import poisson, lgf


def _lap_box(nx, ny, h):
    """5-point -lap_h with psi(-1) = -psi(0), psi(n) = -psi(n-1) (zero on the faces)."""
    def d1(n):
        main = np.full(n, 2.0)
        main[0] = main[-1] = 3.0
        return sp.diags([main, -np.ones(n - 1), -np.ones(n - 1)], [0, 1, -1])
    return (sp.kron(sp.eye(ny), d1(nx)) + sp.kron(d1(ny), sp.eye(nx))) / h ** 2


def test_box_matches_sparse_direct():
    rng = np.random.default_rng(0)
    nx, ny, h = 23, 17, 0.1
    s = rng.standard_normal((ny, nx))
    psi = poisson.box_dirichlet(s, h)
    ref = spla.spsolve(_lap_box(nx, ny, h).tocsc(), s.ravel()).reshape(ny, nx)
    assert np.max(np.abs(psi[1:-1, 1:-1] - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.allclose(psi[0, 1:-1], -psi[1, 1:-1])
    assert np.allclose(psi[1:-1, -1], -psi[1:-1, -2])


def test_free_space_is_exact_inverse_with_ring():
    rng = np.random.default_rng(1)
    nx, ny, h = 20, 13, 0.05
    s = rng.standard_normal((ny, nx))
    fs = poisson.FreeSpace(nx, ny, h)
    psi = fs(s)
    res = poisson.laplacian_residual(psi, s, h)
    assert np.max(np.abs(res)) < 1e-11 * np.max(np.abs(s))


def test_free_space_matches_direct_summation():
    rng = np.random.default_rng(2)
    nx, ny, h = 9, 7, 0.3
    s = rng.standard_normal((ny, nx))
    g = lgf.lgf_table(nx + 1, ny + 1)
    psi = poisson.FreeSpace(nx, ny, h)(s)
    for (i, j) in [(-1, -1), (0, 3), (nx, 2), (4, ny), (nx, ny), (5, 5)]:
        tot = 0.0
        for jj in range(ny):
            for ii in range(nx):
                tot += h * h * g[abs(j - jj), abs(i - ii)] * s[jj, ii]
        assert abs(psi[j + 1, i + 1] - tot) < 1e-13 * np.abs(s).sum()


def test_outflow_is_mirror_sum():
    rng = np.random.default_rng(3)
    nx, ny, h = 8, 6, 0.2
    s = rng.standard_normal((ny, nx))
    g = lgf.lgf_table(2 * nx + 1, ny + 1)
    psi = poisson.FreeSpace(nx, ny, h, outflow=True)(s)
    for (i, j) in [(-1, 0), (3, 2), (nx, ny), (nx - 1, -1)]:
        tot = 0.0
        for jj in range(ny):
            for ii in range(nx):
                tot += h * h * (g[abs(j - jj), abs(i - ii)]
                                + g[abs(j - jj), abs(i + ii - 2 * nx + 1)]) * s[jj, ii]
        assert abs(psi[j + 1, i + 1] - tot) < 1e-13 * np.abs(s).sum()
    # even mirror => zero normal derivative across the outflow face
    big = poisson.FreeSpace(nx, ny, h, outflow=True)
    p = big(s)
    # psi(nx) == psi(nx-1) on every row (even symmetry about x_{nx-1/2})
    assert np.max(np.abs(p[1:-1, -1] - p[1:-1, -2])) < 1e-12 * np.max(np.abs(p))
