// The IIM context (an opaque iim_ctx at the ABI) and the network object
// (iim_net), shared by the C ABI files.  Host-only declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "iim.h"
#include "iim_dev.hpp"
#include "iim_host.hpp"
#include "net_dev.hpp"

namespace iim {

struct HipError : std::runtime_error {
  int code;
  HipError(const std::string& m, int c) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess)                                                                           \
      throw iim::HipError(std::string(#x) + ": " + hipGetErrorString(e_),                           \
                          e_ == hipErrorOutOfMemory ? IIM_ENOMEM : IIM_EDEVICE);                    \
  } while (0)

// status slot written by the guess preparation: norm of b - b_previous
constexpr int KS_PREVRES = 9;

}  // namespace iim

struct iim_net {
  std::string err;
  int cin = iim::NET_FEATURES, width = 128, layers = 4;
  bool bf16 = true;
  hipStream_t stream = nullptr;
  std::vector<int> lin, lout;          // channels of each layer
  std::vector<size_t> offW, offb;      // offsets in the flat parameter array
  size_t nparam = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  int t = 0;                           // Adam steps taken
  float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  // activations (grown on demand): Z[l], H[l] = [rows][lout[l]]
  size_t cap_rows = 0;
  std::vector<float*> Z, H;
  float *dA = nullptr, *dB = nullptr;  // [rows][max width]
  float* part = nullptr;               // weight-gradient partial sums
  float* fwd_part = nullptr;           // split forward products' partial sums (CONV_FWD_PART_MAX floats)
  size_t part_cap = 0;
  float* dY = nullptr;                 // [rows]
  float* lossbuf = nullptr;            // [1]
  std::vector<void*> allocs, act_allocs;
  ~iim_net();
};

struct iim_ctx {
  std::string err;
  iim::Geometry geo;
  bool host_only = false;
  hipStream_t stream = nullptr;
  int precision = IIM_PREC_FP64;
  double tol = 1e-13;
  int max_iter = 400, restart = 40, guess = IIM_GUESS_PREVIOUS, chunk = 4;
  int fft_sizes = IIM_FFT_SIZES_TUNED;
  double torus_us[2] = {0.0, 0.0};   // TUNED: convolution time on the compact and the power-of-two torus
  double eps32 = 2e-6;            // mixed precision: FP32 operator error (measured ~2e-7) x 10
  long n_fp32_products = 0;       // Arnoldi products applied in FP32
  int max_refine = 8;             // mixed precision: FP64 residual evaluations per solve
  int last_rounds = 0;            // GMRES cycles (FP64 residual evaluations) of the last solve
  std::vector<void*> allocs;
  size_t dev_bytes = 0;
  iim::DGeom dg{};
  iim::DFft df{};
  iim::DDst dd{};
  iim::DKrylov dk{};
  iim::DBnd bnd{};                // composed boundary forms of a stage
  bool bnd_ok = false;
  bool box = false;
  int8_t* cls_zero = nullptr;
  double *psi = nullptr, *U = nullptr, *V = nullptr;
  double *wb = nullptr, *w4 = nullptr, *w3b = nullptr, *w3n = nullptr;
  double* sdwdn = nullptr;        // d omega / dn at the control points (surface loads)
  double* scv = nullptr;          // control-volume terms (6 values), then per-row partial sums
  double* cvw = nullptr;          // fluid area of every node's dual cell (made at first use)
  // time-dependent rigid motion (set by iim_set_body_motion or
  // iim_rk3_steps_moving): the boundary-data tables follow motion_now
  // ([n_bodies][3] = u_x, u_y, omega); motion_stage, while a moving step
  // runs, points at that step's [3 stages][n_bodies][3] schedule
  bool motion_mode = false;
  std::vector<double> motion_now;
  const double* motion_stage = nullptr;
  std::vector<double> motion_buf[3];
  // captured moving steps: the three stages' tables staged on the device
  // before each step ([3][4 nc + na]); each stage of the step graph copies
  // its part into the live tables
  double* motion_dev = nullptr;
  bool motion_from_dev = false;
  std::vector<double> motion_host;
  double *Qw = nullptr, *wtmp = nullptr, *wtmp2 = nullptr, *Gd = nullptr, *QGd = nullptr, *dGd = nullptr;
  double* st_host = nullptr;
  // non-finite flag: set on the device by the transport when a new vorticity
  // or circulation value is NaN or Inf; read (and cleared) after the steps
  int* nf_dev = nullptr;
  int* nf_host = nullptr;          // pinned
  // velocity bound of the step-size check (RK3 stability triangle): set at
  // create from the free stream and the boundary speed; iim_set_speed_bound
  // replaces it, moving steps raise it to the speed of their motion
  double a_max = 0.0;
  bool a_max_user = false;
  bool have_prev = false;
  int solver = IIM_SOLVER_KRYLOV;
  double* Sinv_t = nullptr;       // transpose of the dense Schur inverse (row-major)
  double* gemv_part = nullptr;    // partial sums of the solve's product (gemv_t_parts(n) x n)
  // one RK3 step captured as a HIP graph (direct solver): replayed while the
  // omega buffer and dt stay the same
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* g_omega = nullptr;
  double g_dt = 0.0;
  bool use_graph = true;
  long n_solves = 0, n_matvecs = 0;
  iim::Prof prof;
  // host copies for the geometry view
  std::vector<double> v_cxy, v_cn;
  std::vector<int32_t> v_cint, v_aint, v_rects, v_circ;

  // ---- initial guesses from the solve history (extrapolated / network)
  int cur_stage = -1;             // RK stage of the solve in progress; -1 outside an RK step
  double hist_dt = 0.0;
  int hist_count = 0;             // consecutive solves of the current run held in the ring
  long hist_next = 0;             // ring position of the next solve
  double *hb = nullptr, *hx = nullptr;  // [4][n] right-hand sides and solutions
  int* hs_ring = nullptr;         // [3 stages][4 positions][8] slot tables for the feature kernel
  iim_net* net = nullptr;         // not owned
  long n_net_used = 0, n_net_rejected = 0, n_extra_matvecs = 0;
  // sequences of affected points around each body (network input order)
  int seq_P = 0;
  int *perm = nullptr, *seq = nullptr;  // perm[P]; seq = seg0[P], segl[P], pos[P]
  float* seq_geo = nullptr;             // [P][4]
  float *inf_F = nullptr, *inf_scale = nullptr;
  // recording of solves for training
  int rec_cap = 0, rec_count = 0, run_id = 0;
  double *rb = nullptr, *rx = nullptr;  // [cap][n]
  std::vector<int> rec_stage, rec_run;

  template <class T>
  T* dalloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, n * sizeof(T)));
    allocs.push_back(p);
    dev_bytes += n * sizeof(T);
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  iim_ctx() = default;
  iim_ctx(const iim_ctx&) = delete;        // owns device memory, streams, graphs
  iim_ctx& operator=(const iim_ctx&) = delete;
  ~iim_ctx() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (void* p : allocs) (void)hipFree(p);
    if (st_host) (void)hipHostFree(st_host);
    if (nf_host) (void)hipHostFree(nf_host);
  }
};

namespace iim {

// api.cpp
void apply_G(iim_ctx* c, const DGeom& dg, const double* omega, const double* gam, double sgn, int rj0, int rj1,
             int oj0, int oj1, double* psi, const double* done, bool fp32 = false, bool rows_ready = false);
void build_schur_t(iim_ctx* c, double* St);   // St[q][i] = (S e_q)_i
void read_status(iim_ctx* c);
void set_status(iim_ctx* c);
// one RK3 step of the context's state (kernels enqueued on c->stream)
int run_step(iim_ctx* c, double* omega, double dt, iim_step_stats* stats);
// the non-finite flag of the steps enqueued so far (synchronises the
// context's stream); a set flag is cleared
bool take_nonfinite(iim_ctx* c);
// largest stable step for the velocity bound a (stability triangle)
double dt_limit(const iim_ctx* c, double a);

// warm_start.cpp
// Prepare the initial guess of the Krylov solve whose right-hand side is in
// dk.b: returns the mode used (IIM_GUESS_*), after writing dk.x for the
// extrapolated and network modes.
int prepare_guess(iim_ctx* c);
// after a Krylov solve: push (b, x) into the history ring and the recording
void push_history(iim_ctx* c);
// previous-stage solution, for the fallback of a rejected network guess
void restore_previous(iim_ctx* c);
void net_forward(iim_net* net, const Seq& s, int B, const float* X, bool keep_pre, hipStream_t st);

}  // namespace iim
