// Host-side data structures of the IIM library: geometry, stencil tables and
// the lattice Green's function.  Nothing here touches the device.
#pragma once

#include <array>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace iim {

struct GeomError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

enum NodeClass : int8_t { CLS_FLUID = 0, CLS_GHOST = 1, CLS_SOLID = 2 };

struct BodySpec {
  std::vector<double> xy;  // [n][2]
  bool enclosure = false;
  double center[2] = {0, 0};
  double u_rigid[2] = {0, 0};
  double omega = 0;
  int rect[4] = {-1, -1, -1, -1};
  std::vector<double> samples;  // [n][3] u_x, u_y, psi_b at the points (empty: rigid motion)
};

struct GridSpec {
  int nx = 0, ny = 0;
  double x0 = 0, y0 = 0, h = 1;
  int exterior = 1;
  double u_inf[2] = {0, 0};
  double nu = 0;
};

// A sparse linear form per row: sum_k w_k * field(i_k, j_k [, comp_k]) + sum_m bw_m * bc(c_m)
struct Stencil {
  std::vector<int> ptr{0};
  std::vector<int> ii, jj, comp;
  std::vector<double> w;
  std::vector<int> bptr{0};
  std::vector<int> bc, bcomp;
  std::vector<double> bw;
  int rows() const { return (int)ptr.size() - 1; }
};

struct Geometry {
  GridSpec grid;
  std::vector<BodySpec> bodies;
  // control points (canonical order: ghost node linear index, axis, sigma)
  int nc = 0;
  std::vector<double> c_x, c_y, c_theta, c_nx, c_ny, c_ub, c_psib;  // c_ub: [nc][2]
  std::vector<int> c_axis, c_sigma, c_if, c_jf, c_ig, c_jg, c_body;
  std::vector<int> c_seg;       // spline segment of the crossing; c_t its parameter in (0, 1)
  std::vector<double> c_t;
  // node classes [ny][nx]
  std::vector<int8_t> cls;
  std::vector<int> ghost_id;  // [ny][nx], -1 if not a ghost
  int ng = 0;
  std::vector<int> g_i, g_j;
  std::vector<std::vector<int>> g_ctrl;
  // affected points (row-major)
  int na = 0;
  std::vector<int> a_i, a_j, a_ghost, a_body;
  std::vector<int> a_id;  // [ny][nx]
  // tables
  Stencil ext4b, ext3b, ext3n;  // rows = ghosts
  Stencil aop;                  // rows = affected; bc part = B
  Stencil wbc;                  // rows = control points; comp 0 = u_x, 1 = u_y; bc on u_b components
  // bounding regions
  std::vector<std::array<int, 4>> rects;
  std::vector<int> circ_body;
  // transport: fluid nodes handled by the boundary kernel
  std::vector<int> special;  // linear indices j*nx+i
  // pruned Krylov convolution: rows with sources / rows read by the A operator
  int src_j0 = 0, src_j1 = -1, out_j0 = 0, out_j1 = -1;

  int nbc() const { return (int)circ_body.size(); }
  bool in_grid(int i, int j) const { return i >= 0 && j >= 0 && i < grid.nx && j < grid.ny; }
  int8_t cl(int i, int j) const { return cls[(size_t)j * grid.nx + i]; }
};

// Build everything; throws GeomError / ArgError.
void build_geometry(Geometry& g, const GridSpec& grid, const std::vector<BodySpec>& bodies);

// Lattice Green's function g(m, n), 0 <= m <= mx, 0 <= n <= my: out[n*(mx+1)+m].
void lgf_table(int mx, int my, double* out, int threads = 0);

// Real, even circulant kernel K(i, j) = h^2 g(|i'|, |j'|) on an mx x my torus
// -> its (real) Fourier transform on kx in [0, mx/2], ky in [0, my/2],
// scaled by 1/(mx my): out[kx*(my/2+1) + ky].
// mirror_nx > 0 adds the outflow image term is not handled here.
void lgf_spectrum(int mx, int my, double h, const double* table, int tab_mx, double* out);

}  // namespace iim
