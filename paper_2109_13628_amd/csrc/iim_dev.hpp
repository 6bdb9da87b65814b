// Device-side data of one IIM context and the launch wrappers of the HIP
// kernels (kernels.hip).  Host code (api.cpp) fills these structs; kernels
// receive them by value.
#pragma once
#include <climits>

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace iim {

// Sparse table on the device: row r reads node entries [ptr[r], ptr[r+1]) and
// boundary entries [bptr[r], bptr[r+1]).
struct DStencil {
  const int* ptr = nullptr;
  const int* ridx = nullptr;   // ring-array index (j+1)*(nx+2) + (i+1); bit 30 = component 1 (wbc only)
  const int* gidx = nullptr;   // grid-array index j*nx + i
  const double* w = nullptr;
  const int* bptr = nullptr;
  const int* bc = nullptr;     // control point
  const double* bw = nullptr;
  int rows = 0;
  int nnz = 0;                 // node entries (ptr[rows])
};

struct DGeom {
  int nx, ny, nxr;             // nxr = nx + 2
  double h, inv_h, nu;
  double uinf_x, uinf_y;
  int nc, ng, na, nbc, nsp;
  int n;                       // Krylov unknowns: na + nbc
  int outflow;                 // 1: even mirror plane at the face x_{nx-1/2}
  int periodic;                // 1: periodic in x and y (node i + nx is node i)
  const int8_t* cls;           // [ny][nx]: 0 bulk fluid, 1 boundary-kernel fluid, 2 ghost, 3 solid
  const int* g_ridx;           // ghost -> ring index
  const int* g_gidx;           // ghost -> grid index
  const int* a_gidx;           // affected -> grid index
  const int* a_id;             // [ny][nx] grid -> affected index (-1: none)
  const int* a_col;            // affected -> circulation column (-1: none)
  const int* row_ptr;          // per grid row: affected points of that row
  const int* row_i;            //   column i
  const int* row_a;            //   affected index
  const int2* row_ia;          //   (column i, affected index) packed, same order
  int a_j0, a_j1;              // first and last grid row holding affected points (a_j0 > a_j1: none)
  const int* corr_rows;        // the grid rows holding affected points, ascending [n_corr_rows]
  const int* row_slot;         // per grid row: its index in corr_rows, or -1 [ny]
  int n_corr_rows;
  const int* special;          // boundary-kernel fluid nodes (grid index)
  const int* c_col;            // control point -> circulation column (-1: none)
  const double* c_psibt;       // psi_b - psi_inf at control points
  const double* c_ub;          // [nc][2]
  const double* wb_const;      // boundary-velocity part of omega_b
  const double* bpsi;          // B psi_b_tilde  [na]
  const double* b1;            // B 1_k, [nbc][na]
  const int* rects;            // [nbc][4]
  DStencil ext4b, ext3b, ext3n, aop, wbc;
  // surface loads: the boundary-value weights of the boundary-vorticity
  // stencil split into its d_x part (lw_x) and minus its d_y part (lw_y),
  // and the unit normal into the fluid at each control point
  const double* lw_x;
  const double* lw_y;
  const double2* c_n;
  // set to 1 by the RK update of the transport when a new vorticity or
  // circulation value is not finite (never cleared by a kernel of the step)
  int* nonfinite;
};

// The boundary quantities of a stage as affine forms of psi (ring), omega
// (grid) and the body constants psibar: row r = kc[r] + sum over its entries
// of w * value, with entry idx = kind << 28 | index (kind 0: psi[index],
// 1: omega[index], 2: psibar[index]); dst = kind << 28 | index names the
// output (0 psi ghost (ring), 1 u (ring), 2 v (ring), 3 omega_b, 4 E4b,
// 5 E3b, 6 E3n (grid)).  Indices stay below 2^28, kinds below 8.
struct DBnd {
  int rows = 0;
  // > 0: every row holds exactly `stride` entries from row * stride on (the
  // pads repeat the row's last entry with weight zero) and ptr is unused;
  // 0: rows delimited by ptr
  int stride = 0;
  const int* ptr = nullptr;
  const int* idx = nullptr;
  const double* w = nullptr;
  const double* kc = nullptr;
  const int* dst = nullptr;
};

// FFT convolution plan (free space / outflow)
struct DFft {
  int mx, my;                  // padded torus
  int hx;                      // mx / 2 (complex length of the row transforms)
  int ld;                      // leading dimension of the spectrum buffer (>= ny + 2)
  const double* ghat;          // [mx/2+1][my/2+1]
  const double2* tw_x;         // exp(-2 pi i k / hx), k < hx
  const double2* tw_xr;        // exp(-2 pi i k / mx), k <= mx/2 (real-FFT post-processing)
  const double2* tw_y;         // exp(-2 pi i k / my), k < my
  double2* spec;               // [mx/2+1][ld] row transforms of the dense source
  double2* spec_out;           // [mx/2+1][ld] column pass output
  // FP32 copies for the inner products of the mixed-precision solve (null
  // unless the context is mixed precision)
  const float* ghat32 = nullptr;
  const float2* tw_x32 = nullptr;
  const float2* tw_xr32 = nullptr;
  const float2* tw_y32 = nullptr;
  float2* spec32 = nullptr;
  float2* spec32_out = nullptr;
  // row transforms of the correction sources, [mx/2+1][n_corr_rows] (complex
  // of the pass's precision), formed by a pre-pass when there are many
  // affected points (null: the column pass forms them itself)
  void* corr = nullptr;
  bool outflow;
  bool periodic = false;       // unpadded torus of the grid itself: every row and column carries data
  bool use_reg = true;         // register-resident FFT kernels (sizes >= 256)
  int row_per = 0, col_per = 0; // FFTs per workgroup of the row / column passes (0: default; tuned)
};

struct DDst {                  // box: dense orthonormal sine transforms
  const double* phx;           // [nx][nx]   phi_x[k][n] (orthonormal DST-II)
  const double* phxT;          // transpose
  const double* phy;           // [ny][ny]
  const double* phyT;
  const double* lam_inv;       // [ny][nx]
  double* t1;                  // [ny][nx]
  double* t2;
  double* src;                 // [ny][nx] assembled source
};

// Krylov state (device)
struct DKrylov {
  int n, m;                    // unknowns, restart length
  double* V;                   // [(m+1)][n]
  double* H;                   // [(m+1)][m] column-major: H[k*(m+1) + i]
  double* cs;                  // [m]
  double* sn;                  // [m]
  double* g;                   // [m+1]
  double* x;                   // [n]
  double* b;                   // [n]
  double* w;                   // [n] work
  double* st;                  // status: see KS_* offsets
};
enum {
  KS_DONE = 0, KS_K = 1, KS_ITERS = 2, KS_BNORM = 3, KS_BETA = 4, KS_RES = 5, KS_RES0 = 6, KS_TOL = 7,
  KS_NFAIL = 8, KS_SIZE = 16
};

// ---------------------------------------------------------------- profiling
// Event pairs around selected kernel launches (kernel ids below); read back
// with Prof::collect after the stream has drained.
enum KId { KID_ROWS_FWD = 0, KID_COLS = 1, KID_ROWS_INV = 2, KID_TRANSPORT = 3, KID_ARNOLDI = 4, KID_GEMM = 5,
           KID_N = 6 };
struct Prof {
  unsigned mask = 0;
  struct Rec { int id; int ea, eb; double bytes; };
  std::vector<hipEvent_t> pool;
  int used = 0;
  std::vector<Rec> recs;
  double total_ms[KID_N] = {0};
  double bytes[KID_N] = {0};
  long count[KID_N] = {0};
  // the largest launch of each timed kernel, kept for back-to-back replays
  std::function<void(hipStream_t)> replay[KID_N];
  long replay_grid[KID_N] = {0};
  double replay_bytes[KID_N] = {0};
  template <class F>
  void keep(int id, long grid, double b, F&& f) {
    if (grid >= replay_grid[id]) {
      replay[id] = std::forward<F>(f);
      replay_grid[id] = grid;
      replay_bytes[id] = b;
    }
  }
  int ev(hipStream_t s) {
    if (used == (int)pool.size()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
      pool.push_back(e);
    }
    (void)hipEventRecord(pool[used], s);
    return used++;
  }
  bool on(int id) const { return ((mask >> id) & 1u) && recs.size() <= 200000; }
  // Two pooled events for a launch made with hipExtLaunchKernelGGL, which
  // records them in the dispatch packet around the kernel itself.
  void pair(int id, double b, hipEvent_t& ea, hipEvent_t& eb) {
    auto get = [&]() -> int {
      if (used == (int)pool.size()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        pool.push_back(e);
      }
      return used++;
    };
    const int a = get(), c = get();
    if (a < 0 || c < 0) { ea = eb = nullptr; return; }
    recs.push_back(Rec{id, a, c, b});
    ea = pool[a];
    eb = pool[c];
  }
  int begin(int id, hipStream_t s) {
    if (!((mask >> id) & 1u) || recs.size() > 200000) return -1;
    Rec r{id, ev(s), -1, 0.0};
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int h, double b, hipStream_t s) {
    if (h < 0) return;
    recs[h].eb = ev(s);
    recs[h].bytes = b;
  }
  void collect() {
    for (auto& r : recs) {
      if (r.ea < 0 || r.eb < 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pool[r.ea], pool[r.eb]) == hipSuccess) {
        total_ms[r.id] += ms;
        bytes[r.id] += r.bytes;
        count[r.id] += 1;
      }
    }
    recs.clear();
    used = 0;
  }
  void reset() {
    recs.clear();
    used = 0;
    for (int i = 0; i < KID_N; ++i) total_ms[i] = bytes[i] = 0.0, count[i] = 0;
  }
  Prof() = default;
  Prof(const Prof&) = delete;              // owns its events
  Prof& operator=(const Prof&) = delete;
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

inline long grid_size(dim3 g) { return (long)g.x * g.y * g.z; }

// Launch `kern` on stream s; when prof times kernel id, bracket it with
// dispatch-packet events (hipExtLaunchKernelGGL).
#define IIM_LAUNCH(prof, id, bytes, kern, grid, block, s, ...)                       \
  do {                                                                               \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                                         \
    if ((prof) && (prof)->on(id)) {                                                  \
      (prof)->pair((id), (bytes), ea_, eb_);                                         \
      (prof)->keep((id), iim::grid_size(dim3(grid)), (bytes),                       \
                   [=](hipStream_t s_) { kern<<<(grid), (block), 0, s_>>>(__VA_ARGS__); }); \
    }                                                                                \
    if (ea_)                                                                         \
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, ea_, eb_, 0, __VA_ARGS__); \
    else                                                                             \
      kern<<<(grid), (block), 0, s>>>(__VA_ARGS__);                                  \
  } while (0)

// ---------------------------------------------------------------- launchers
// Poisson operator (free space): psi_ring rows [oj0, oj1] from sources in rows [rj0, rj1].
// source = mask(omega) (omega may be null) + sgn * scatter(gam) (gam may be null).
// fp32: FFTs and kernel multiply in FP32 (inputs and psi stay FP64); needs the
// FP32 tables and FFT sizes >= 256 (otherwise FP64).
// The row pass transforms the dense part (omega) into spec; the sparse part
// (gam) enters the column pass directly, which writes spec_out, read by the
// inverse row pass.  spec is written by the row pass only, so with
// rows_ready the row pass is skipped and the row transforms that an earlier
// call left in spec are used: they must be those of the same omega over the
// same rows [rj0, rj1] and precision.
bool conv_reg_supported(int hx, int my);
// whether the register FFT kernels selected by f's tile shapes (row_per,
// col_per; FP64 or the FP32 copies) can be launched on the current device;
// why (nullable) names the failing kernel and its limits
bool reg_shapes_fit(const DFft& f, bool fp32, std::string* why);
// affected points above which the correction sources' row transforms are
// formed by a pre-pass (DFft::corr)
constexpr int CORR_PREPASS_MIN = 1024;
void launch_conv(const DGeom& g, const DFft& f, const double* omega, const double* gam, double sgn,
                 int rj0, int rj1, int oj0, int oj1, double* psi_ring, const double* done_flag,
                 hipStream_t s, Prof* prof = nullptr, bool fp32 = false, bool rows_ready = false);
void launch_dst(const DGeom& g, const DDst& d, const double* omega, const double* gam, double sgn,
                double* psi_ring, const double* done_flag, hipStream_t s);

void launch_rhs_vector(const DGeom& g, const double* psi_ring, const double* omega,
                       const double* Gamma, double* b, hipStream_t s);
void launch_krylov_start(const DGeom& g, const DKrylov& k, bool x_is_zero, hipStream_t s);
void launch_arnoldi(const DGeom& g, const DKrylov& k, const double* psi_ring, int j, hipStream_t s,
                    Prof* prof = nullptr);
void launch_gmres_update(const DKrylov& k, hipStream_t s);
void launch_matvec_finish(const DGeom& g, const DKrylov& kr, const double* psi_ring, const double* v,
                          double* out, hipStream_t s);

void launch_recover_fields(const DGeom& g, const double* x, double* psi_ring, double* U, double* V,
                           hipStream_t s);
void launch_omega_bc(const DGeom& g, const double* omega, const double* U, const double* V,
                     double* wb, double* w4, double* w3b, double* w3n, hipStream_t s);
// every boundary quantity of a stage from its composed form (DBnd); then
// launch_velocity for the other nodes
void launch_boundary_forms(const DGeom& g, const DBnd& b, const double* omega, const double* x, double* psi_ring,
                           double* U, double* V, double* wb, double* w4, double* w3b, double* w3n, hipStream_t s);
// velocity at every ring node except the ghosts
void launch_velocity(const DGeom& g, const double* psi_ring, double* U, double* V, hipStream_t s);
// Transport of every fluid node and the Kelvin circulation update, one launch.
// mode 0: out = domega/dt, dG = dGamma/dt (Q, Gamma, QG unused);
// mode 1: Q = a Q + dt rhs, out = omega + b Q, and the same for (Gamma, QG)
// with dG the rate; a = 0 overwrites the registers without reading them.
// Kelvin: dG = -h sum (F+Q).n over dR_k.
// Velocities: psi null: U, V on the ring; otherwise formed from psi (ring,
// ghost values already in place) at every node but the ghosts, whose
// extension values are read from U, V (the velocity kernel is not needed).
void launch_transport_all(const DGeom& g, const double* omega, const double* psi, const double* U, const double* V,
                          const double* w4, const double* w3b, const double* w3n, double* out, double* Q, double* dG,
                          double* Gamma, double* QG, double a, double b, double dt, int mode, hipStream_t s,
                          Prof* prof = nullptr);
void launch_fill(double* p, double v, size_t n, hipStream_t s);
void launch_fill_int(int* p, int v, size_t n, hipStream_t s);
// dense Schur complement: in-place Gauss-Jordan inverse, transposed GEMV, unit vector
void launch_gj_invert(double* M, int n, int* perm, double* fcol, double* info, hipStream_t s);
// x = Mt^T b (Mt row-major n x n); `part` holds gemv_t_parts(n) x n doubles
int gemv_t_parts(int n);
void launch_gemv_t(const double* Mt, int n, const double* b, double* x, double* part, hipStream_t s);
// b (right-hand side, as launch_rhs_vector) and x = Mt^T b in one launch; b is
// stored too.  Returns false, launching nothing, when n differs from
// na + nbc or exceeds the kernel's LDS capacity.
bool launch_rhs_solve(const DGeom& g, const double* psi_ring, const double* omega, const double* Gamma,
                      const double* Mt, int n, double* b, double* x, hipStream_t s);
void launch_unit(double* v, int n, int q, hipStream_t s);
// d omega / dn at every control point: the boundary-vorticity stencil's d_x
// and d_y parts applied to omega extended with E3b at the ghosts (w3b), with
// omega_b (wb) as the boundary value, projected on the normal into the fluid.
// Control-volume force box: nodes i0..i1 x j0..j1 of an nx-wide grid (node
// (i, j) at (x0 + i h, y0 + j h)), x measured from (ox, oy).
struct CvBox {
  int nx, i0, i1, j0, j1;
  double x0, y0, h, nu, ox, oy;
};
// out[0..3] = (S_t x, S_t y, S_gamma x, S_gamma y), out[5] = S_lambda of the
// box (device); the box and its nodes' four neighbours must lie inside the grid.
void launch_cv_terms(const CvBox& b, const double* omega, const double* U, const double* V, double* out,
                     hipStream_t s);
// out[4] = I, the box's sum of |x|^2/2 omega_ext W (W: fluid area of each
// node's dual cell, [ny][nx]; omega_ext: w3b at ghost nodes, 0 at solid ones);
// part: one partial sum per box row (j1 - j0 + 1 values).
void launch_cv_volume(const CvBox& b, const int8_t* cls, const double* omega, const double* w3b, const double* W,
                      double* part, double* out, hipStream_t s);
void launch_surface_dwdn(const DGeom& g, const double* omega, const double* w3b, const double* wb, double* dwdn,
                         hipStream_t s);
// E4b, E3b, E3n at the ghost nodes from omega and a given wall vorticity wb.
void launch_extensions_given_wb(const DGeom& g, const double* omega, const double* wb, double* w4, double* w3b,
                                double* w3n, hipStream_t s);

}  // namespace iim
