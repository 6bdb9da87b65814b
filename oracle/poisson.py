"""Solution operators G = (-lap_h)^-1 of the 5-point Laplacian on a rectangular
grid (Sec. 4.2: the FFT-based inverse with unbounded, symmetric or bounded
exterior conditions; Sec. 5.2 for the symmetric outflow plane).

Every operator maps a source s[ny][nx] (supported on the grid) to psi on the
grid plus a one-node ring, returned as an array of shape (ny+2, nx+2) with
psi[j+1, i+1] = psi(i, j) for -1 <= i <= nx, -1 <= j <= ny.

Bounded box (reading of the paper's bounded exterior): the grid is
cell-centred and psi vanishes on the box faces half a cell outside the edge
nodes, i.e. psi(-1, j) = -psi(0, j) and psi(nx, j) = -psi(nx-1, j) (same in
y).  The 5-point operator with these reflections is diagonalised by the
type-II sine transform with eigenvalues (4/h^2) sin^2(pi k / 2N), k = 1..N.

Free space: psi(x) = h^2 sum_x' g(x - x') s(x') with the lattice Green's
function g of oracle.lgf, evaluated by a zero-padded FFT convolution on a
(2 ny) x (2 nx) torus; the ring outputs are exact as well.

Outflow: free space in y and at x_min, with an even mirror of the source
across the face x_{nx-1/2}:  psi(i) = sum_i' [g(i - i') + g(i + i' - 2 nx + 1)] s(i').

Periodic (Sec. 4.1, the periodic exterior): node i + nx is node i (same in
y).  The 5-point operator on the periodic lattice is diagonalised by the
discrete Fourier transform with eigenvalues
(4/h^2) [sin^2(pi kx / nx) + sin^2(pi ky / ny)]; its null space is the
constant, so the source's mean is removed and psi is the solution of zero
mean (the paper's gauge for the periodic part of the stream function).  The
ring holds the periodic images.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import lgf


def box_dirichlet(s, h):
    s = np.asarray(s, dtype=np.float64)
    ny, nx = s.shape
    kx = np.arange(1, nx + 1)
    ky = np.arange(1, ny + 1)
    lam = (4.0 / h ** 2) * (np.sin(np.pi * ky / (2 * ny))[:, None] ** 2
                            + np.sin(np.pi * kx / (2 * nx))[None, :] ** 2)
    sh = sfft.dstn(s, type=2)
    psi = sfft.idstn(sh / lam, type=2)
    out = np.zeros((ny + 2, nx + 2))
    out[1:-1, 1:-1] = psi
    out[0, 1:-1] = -psi[0, :]
    out[-1, 1:-1] = -psi[-1, :]
    out[1:-1, 0] = -psi[:, 0]
    out[1:-1, -1] = -psi[:, -1]
    out[0, 0] = psi[0, 0]
    out[0, -1] = psi[0, -1]
    out[-1, 0] = psi[-1, 0]
    out[-1, -1] = psi[-1, -1]
    return out


def periodic(s, h):
    s = np.asarray(s, dtype=np.float64)
    ny, nx = s.shape
    lam = (4.0 / h ** 2) * (np.sin(np.pi * np.arange(ny) / ny)[:, None] ** 2
                            + np.sin(np.pi * np.arange(nx) / nx)[None, :] ** 2)
    sh = sfft.fft2(s)
    lam[0, 0] = 1.0
    sh = sh / lam
    sh[0, 0] = 0.0                     # zero mean: the gauge of the periodic part
    psi = sfft.ifft2(sh).real
    jj = np.arange(-1, ny + 1) % ny
    ii = np.arange(-1, nx + 1) % nx
    return psi[np.ix_(jj, ii)]


class FreeSpace:
    """Zero-padded LGF convolution on a (2 ny) x (2 nx) torus."""

    def __init__(self, nx, ny, h, table=None, outflow=False):
        self.nx, self.ny, self.h = nx, ny, h
        self.outflow = outflow
        mx, my = 2 * nx, 2 * ny
        if outflow:
            mx = 4 * nx      # room for the mirrored source without wrap-around
        self.mx, self.my = mx, my
        g = table if table is not None else lgf.cached_lgf_table(mx // 2, my // 2)
        # circulant kernel: K[jj, ii] = h^2 g(|ii'|, |jj'|), ii' the signed offset
        ii = np.arange(mx)
        jj = np.arange(my)
        di = np.minimum(ii, mx - ii)
        dj = np.minimum(jj, my - jj)
        K = (h * h) * g[dj[:, None], di[None, :]]
        self.khat = sfft.rfft2(K)

    def __call__(self, s):
        nx, ny, mx, my = self.nx, self.ny, self.mx, self.my
        pad = np.zeros((my, mx))
        pad[:ny, :nx] = s
        if self.outflow:
            # even mirror across the face x_{nx-1/2}: node i' maps to 2 nx - 1 - i'
            pad[:ny, nx:2 * nx] = s[:, ::-1]
        full = sfft.irfft2(sfft.rfft2(pad) * self.khat, s=(my, mx))
        jj = np.arange(-1, ny + 1) % my
        ii = np.arange(-1, nx + 1) % mx
        return full[np.ix_(jj, ii)]


def laplacian_residual(psi_ring, s, h):
    """-lap_h psi - s on the grid nodes, using the ring for the edge nodes."""
    p = psi_ring
    lap = (p[1:-1, 2:] + p[1:-1, :-2] + p[2:, 1:-1] + p[:-2, 1:-1] - 4 * p[1:-1, 1:-1]) / h ** 2
    return -lap - s
