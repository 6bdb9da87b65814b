// HIP kernel of the surface-load diagnostics (Sec. 5.4): the vorticity
// gradient at the control points.  Outside the time step's hot path.
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

void launch_surface_dwdn(const DGeom& g, const double* omega, const double* w3b, const double* wb, double* dwdn,
                         hipStream_t s) {
  if (g.nc) k_surface_dwdn<<<(g.nc + 127) / 128, 128, 0, s>>>(g, omega, w3b, wb, dwdn);
}

}  // namespace iim
