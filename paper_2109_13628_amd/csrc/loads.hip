// HIP kernels of the load diagnostics (Sec. 5.4): the vorticity gradient at
// the control points, and the box integrals of the control-volume force.
// Outside the time step's hot path.
#include <hip/hip_runtime.h>

#include "iim_dev.hpp"

namespace iim {

__global__ void k_surface_dwdn(DGeom g, const double* __restrict__ omega, const double* __restrict__ w3b,
                               const double* __restrict__ wb, double* __restrict__ dwdn) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nc) return;
  const int nxr = g.nx + 2;
  // the stencil's component-1 terms are d_x of the field, its component-0
  // terms minus d_y
  double dx = g.lw_x[c] * wb[c], dy = g.lw_y[c] * wb[c];
  for (int e = g.wbc.ptr[c]; e < g.wbc.ptr[c + 1]; ++e) {
    const int r = g.wbc.ridx[e];
    const int rr = r & ((1 << 30) - 1);
    const int q = (rr / nxr - 1) * g.nx + (rr % nxr - 1);
    const double val = g.cls[q] == 2 ? w3b[q] : omega[q];
    if (r & (1 << 30))
      dx += g.wbc.w[e] * val;
    else
      dy -= g.wbc.w[e] * val;
  }
  dwdn[c] = g.c_n[c].x * dx + g.c_n[c].y * dy;
}

// Vorticity extensions E4b, E3b (with the given wall vorticity wb) and E3n at
// the ghost nodes, for a transport right-hand side whose wall vorticity is
// prescribed instead of computed from the velocity.
__global__ void k_extensions_given_wb(DGeom g, const double* __restrict__ omega, const double* __restrict__ wb,
                                      double* __restrict__ w4, double* __restrict__ w3b, double* __restrict__ w3n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ng) return;
  double a4 = 0.0, a3 = 0.0, an = 0.0;
  for (int e = g.ext4b.ptr[q]; e < g.ext4b.ptr[q + 1]; ++e) a4 += g.ext4b.w[e] * omega[g.ext4b.gidx[e]];
  for (int e = g.ext4b.bptr[q]; e < g.ext4b.bptr[q + 1]; ++e) a4 += g.ext4b.bw[e] * wb[g.ext4b.bc[e]];
  for (int e = g.ext3b.ptr[q]; e < g.ext3b.ptr[q + 1]; ++e) a3 += g.ext3b.w[e] * omega[g.ext3b.gidx[e]];
  for (int e = g.ext3b.bptr[q]; e < g.ext3b.bptr[q + 1]; ++e) a3 += g.ext3b.bw[e] * wb[g.ext3b.bc[e]];
  for (int e = g.ext3n.ptr[q]; e < g.ext3n.ptr[q + 1]; ++e) an += g.ext3n.w[e] * omega[g.ext3n.gidx[e]];
  const int gi = g.g_gidx[q];
  w4[gi] = a4;
  w3b[gi] = a3;
  w3n[gi] = an;
}

void launch_extensions_given_wb(const DGeom& g, const double* omega, const double* wb, double* w4, double* w3b,
                                double* w3n, hipStream_t s) {
  if (g.ng) k_extensions_given_wb<<<(g.ng + 127) / 128, 128, 0, s>>>(g, omega, wb, w4, w3b, w3n);
}

void launch_surface_dwdn(const DGeom& g, const double* omega, const double* w3b, const double* wb, double* dwdn,
                         hipStream_t s) {
  if (g.nc) k_surface_dwdn<<<(g.nc + 127) / 128, 128, 0, s>>>(g, omega, w3b, wb, dwdn);
}

// Control-volume surface terms on the rectangle of grid lines through the
// nodes i0..i1 x j0..j1: one workgroup walks the perimeter (bottom, right,
// top, left edge; trapezoid weights, corners in both their edges), each lane
// summing the terms of its nodes, then a fixed-order tree sum in LDS.
// out[0..3] = (S_t x, S_t y, S_gamma x, S_gamma y) of the force, out[5] =
// S_lambda of the moment.
constexpr int CV_THREADS = 256;

__global__ void __launch_bounds__(CV_THREADS)
    k_cv_terms(CvBox b, const double* __restrict__ omega, const double* __restrict__ U,
               const double* __restrict__ V, double* __restrict__ out) {
  const int mi = b.i1 - b.i0, mj = b.j1 - b.j0;
  const int np = 2 * (mi + 1) + 2 * (mj + 1);
  const int nxr = b.nx + 2;
  const double h = b.h, nu = b.nu, i2h = 0.5 / b.h;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < np; p += CV_THREADS) {
    int i, j, k, m;
    double nx, ny;
    if (p <= mi) {
      k = p, m = mi, i = b.i0 + k, j = b.j0, nx = 0.0, ny = -1.0;
    } else if (p <= mi + 1 + mj) {
      k = p - (mi + 1), m = mj, i = b.i1, j = b.j0 + k, nx = 1.0, ny = 0.0;
    } else if (p <= 2 * mi + 2 + mj) {
      k = p - (mi + 2 + mj), m = mi, i = b.i0 + k, j = b.j1, nx = 0.0, ny = 1.0;
    } else {
      k = p - (2 * mi + 3 + mj), m = mj, i = b.i0, j = b.j0 + k, nx = -1.0, ny = 0.0;
    }
    const double wgt = (k == 0 || k == m) ? 0.5 * h : h;
    const double x = b.x0 + i * h - b.ox, y = b.y0 + j * h - b.oy;
    const size_t r = (size_t)(j + 1) * nxr + (i + 1), q = (size_t)j * b.nx + i;
    const double u = U[r], v = V[r], w = omega[q];
    const double ux_x = (U[r + 1] - U[r - 1]) * i2h, ux_y = (U[r + nxr] - U[r - nxr]) * i2h;
    const double uy_x = (V[r + 1] - V[r - 1]) * i2h, uy_y = (V[r + nxr] - V[r - nxr]) * i2h;
    const double w_x = (omega[q + 1] - omega[q - 1]) * i2h, w_y = (omega[q + b.nx] - omega[q - b.nx]) * i2h;
    const double dtx = -nu * w_y, dty = nu * w_x;                  // div T = nu lap u
    const double sh = ux_y + uy_x;
    const double un = u * nx + v * ny;
    const double nxu = nx * v - ny * u;                            // n x u (k component)
    acc[0] += wgt * (x * un + nxu * y);
    acc[1] += wgt * (y * un - nxu * x);
    const double ke = 0.5 * (u * u + v * v), xd = x * dtx + y * dty, nxx = nx * x + ny * y;
    acc[2] += wgt * (ke * nx - un * u - un * w * y + xd * nx - nxx * dtx + nu * (2.0 * ux_x * nx + sh * ny));
    acc[3] += wgt * (ke * ny - un * v + un * w * x + xd * ny - nxx * dty + nu * (sh * nx + 2.0 * uy_y * ny));
    // lambda(n) = |u|^2/2 (x x n) - (x x u)(u.n) - |x|^2/2 n x (u x omega k)
    //           + |x|^2/2 (div T) x n + x x (T.n)   (k components)
    const double r2 = 0.5 * (x * x + y * y);
    const double tnx = nu * (2.0 * ux_x * nx + sh * ny), tny = nu * (sh * nx + 2.0 * uy_y * ny);
    acc[4] += wgt * (ke * (x * ny - y * nx) - (x * v - y * u) * un + r2 * w * un + r2 * (dtx * ny - dty * nx) +
                     (x * tny - y * tnx));
  }
  __shared__ double red[5][CV_THREADS];
  for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int s = CV_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 4) out[5] = red[4][0];
}

// Volume term of the control-volume moment: I = sum over the box's nodes of
// |x|^2/2 omega times the fluid area of the node's dual cell (W), halved on
// the box's edges; omega extended by E3b at the ghost nodes, zero at the
// other solid nodes.  One workgroup per box row writes the row's sum to
// part[row]; k_cv_sum then adds the rows in a fixed order into out[4].
__global__ void __launch_bounds__(CV_THREADS)
    k_cv_volume(CvBox b, const int8_t* __restrict__ cls, const double* __restrict__ omega,
                const double* __restrict__ w3b, const double* __restrict__ W, double* __restrict__ part) {
  const int j = b.j0 + blockIdx.x;
  const double fj = (j == b.j0 || j == b.j1) ? 0.5 : 1.0;
  const double y = b.y0 + j * b.h - b.oy;
  double acc = 0.0;
  for (int i = b.i0 + threadIdx.x; i <= b.i1; i += CV_THREADS) {
    const size_t q = (size_t)j * b.nx + i;
    const int c = cls[q];
    const double val = c == 2 ? w3b[q] : (c == 3 ? 0.0 : omega[q]);
    const double x = b.x0 + i * b.h - b.ox;
    acc += (i == b.i0 || i == b.i1 ? 0.5 : 1.0) * W[q] * 0.5 * (x * x + y * y) * val;
  }
  __shared__ double red[CV_THREADS];
  red[threadIdx.x] = fj * acc;
  __syncthreads();
  for (int s = CV_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(CV_THREADS) k_cv_sum(const double* __restrict__ part, int n, double* out) {
  double acc = 0.0;
  for (int r = threadIdx.x; r < n; r += CV_THREADS) acc += part[r];
  __shared__ double red[CV_THREADS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = CV_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[4] = red[0];
}

void launch_cv_terms(const CvBox& b, const double* omega, const double* U, const double* V, double* out,
                     hipStream_t s) {
  k_cv_terms<<<1, CV_THREADS, 0, s>>>(b, omega, U, V, out);
}

void launch_cv_volume(const CvBox& b, const int8_t* cls, const double* omega, const double* w3b, const double* W,
                      double* part, double* out, hipStream_t s) {
  const int rows = b.j1 - b.j0 + 1;
  k_cv_volume<<<rows, CV_THREADS, 0, s>>>(b, cls, omega, w3b, W, part);
  k_cv_sum<<<1, CV_THREADS, 0, s>>>(part, rows, out);
}

}  // namespace iim
