"""Lattice Green's function (LGF) of the 5-point Laplacian on the infinite
unit lattice.

The paper needs an exact inverse of the discrete Laplacian with unbounded
boundary conditions (Sec. 4.2, the solution operator written as the inverse
of the 5-point Laplacian); on an unbounded lattice that inverse is a
convolution with the LGF.  We use

    g(m, n) = -A(m, n),   A(m, n) = (2 pi)^-2 * iint_{[-pi,pi]^2}
                  (1 - cos(m a + n b)) / (4 - 2 cos a - 2 cos b) da db,

so that  -(g(m+1,n) + g(m-1,n) + g(m,n+1) + g(m,n-1) - 4 g(m,n)) = delta_{m,n}
and the gauge is g(0,0) = 0.  Integrating over b in closed form gives the
one-dimensional integral

    A(m, n) = 1/(2 pi) int_0^pi (1 - exp(-|n| t) cos(m a)) / sinh t  da,
              cosh t = 2 - cos a,

which is symmetric in (m, n); we put the larger index in the exponent.  With
s = sin(a/2):  t = 2 asinh(s),  sinh t = 2 s sqrt(1 + s^2).

Quadrature: Gauss-Legendre on geometrically graded panels [0, 1/k, 2/k,
4/k, ..., pi] with k = max(|m|, |n|), so that every panel resolves the decay
scale of exp(-k t).
"""
from __future__ import annotations

import os
import hashlib

import numpy as np

_GL_N = 48


def _panels(k):
    if k <= 0:
        return np.array([0.0, np.pi])
    edges = [0.0]
    e = 1.0 / k
    while e < np.pi:
        edges.append(e)
        e *= 2.0
    edges.append(np.pi)
    return np.array(edges)


def _nodes_weights(k):
    xg, wg = np.polynomial.legendre.leggauss(_GL_N)
    edges = _panels(k)
    a, b = edges[:-1], edges[1:]
    mid = 0.5 * (a + b)[:, None]
    half = 0.5 * (b - a)[:, None]
    return (mid + half * xg[None, :]).ravel(), (half * wg[None, :]).ravel()


def potential_A(big, small_values):
    """A(big, s) for one value of the larger index `big` and an array of the
    smaller index values `small_values` (each <= big)."""
    small_values = np.asarray(small_values, dtype=np.float64)
    if big == 0:
        return np.zeros_like(small_values)
    th, w = _nodes_weights(big)
    s = np.sin(0.5 * th)
    t = 2.0 * np.arcsinh(s)
    sinh_t = 2.0 * s * np.sqrt(1.0 + s * s)
    e = np.exp(-big * t)
    base = -np.expm1(-big * t)                      # 1 - exp(-k t), no cancellation
    osc = 2.0 * np.sin(0.5 * np.outer(small_values, th)) ** 2   # 1 - cos(b a)
    integrand = (base[None, :] + e[None, :] * osc) / sinh_t[None, :]
    return integrand @ w / (2.0 * np.pi)


def lgf_table(mx, my):
    """g(m, n) = -A(m, n) for 0 <= m <= mx, 0 <= n <= my, shape (my+1, mx+1)."""
    out = np.zeros((my + 1, mx + 1))
    for k in range(0, max(mx, my) + 1):
        # entries whose larger index equals k
        if k <= mx:                      # m = k, n = 0..min(k, my)
            n = np.arange(0, min(k, my) + 1)
            out[n, k] = -potential_A(k, n)
        if k <= my:                      # n = k, m = 0..min(k-1, mx)
            m = np.arange(0, min(k - 1, mx) + 1)
            if m.size:
                out[k, m] = -potential_A(k, m)
    return out


def cached_lgf_table(mx, my, cache_dir=None):
    """lgf_table with an on-disk cache (the table only depends on its size)."""
    cache_dir = cache_dir or os.environ.get("IIM_ORACLE_CACHE",
                                            os.path.join(os.path.expanduser("~"), ".cache",
                                                         "iim_oracle"))
    try:
        os.makedirs(cache_dir, exist_ok=True)
    except OSError:
        return lgf_table(mx, my)
    tag = hashlib.sha1(("lgf-v1-%d-%d-%d" % (mx, my, _GL_N)).encode()).hexdigest()[:16]
    path = os.path.join(cache_dir, "lgf_%d_%d_%s.npy" % (mx, my, tag))
    if os.path.exists(path):
        try:
            return np.load(path, allow_pickle=False)
        except (OSError, ValueError):
            pass
    tab = lgf_table(mx, my)
    tmp = path + ".tmp%d.npy" % os.getpid()
    np.save(tmp, tab)
    os.replace(tmp, path)
    return tab


def lgf_far_field(m, n):
    """Two-term large-r expansion of g (for pinning the table):
    g ~ -(ln r + euler_gamma + 1.5 ln 2)/(2 pi) + cos(4 phi)/(24 pi r^2)."""
    r = np.hypot(m, n)
    phi = np.arctan2(n, m)
    return -(np.log(r) + np.euler_gamma + 1.5 * np.log(2.0)) / (2 * np.pi) \
        + np.cos(4 * phi) / (24 * np.pi * r * r)
