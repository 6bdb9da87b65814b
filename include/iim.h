/*
 * iim.h -- C ABI of the MI355X (gfx950) immersed interface method library.
 *
 * The library advances the 2D vorticity-velocity Navier-Stokes equations with
 * immersed bodies as described in Gabbard, Gillis, Chatelain & van Rees,
 * "An immersed interface method for the 2D vorticity-velocity Navier-Stokes
 * equations with multiple bodies" (arXiv:2109.13628):
 *   - velocity reconstruction (Sec. 4.2): the 5-point Poisson problem with
 *     IIM corrections gamma on the affected points, solved as the Schur
 *     complement system with one circulation row per body, by GMRES whose
 *     matrix-vector product is an FFT convolution;
 *   - vorticity transport (Sec. 3): conservative third-order upwind advection
 *     and centred diffusion with the IIM boundary rules, the boundary
 *     vorticity of Sec. 5.3 and the Kelvin circulation ODE of Sec. 5.1;
 *   - the low-storage third-order Runge-Kutta step of Sec. 5.5.
 *
 * Conventions
 *   - Grid node (i, j) sits at (x0 + i h, y0 + j h); a grid field is a
 *     contiguous double array [ny][nx] (row j, column i).
 *   - A "ring" field is a contiguous double array [ny+2][nx+2] holding the
 *     grid plus one node on every side: element [(j+1)*(nx+2) + (i+1)] is
 *     node (i, j), -1 <= i <= nx, -1 <= j <= ny.
 *   - Pointers named *_dev are device pointers (hipMalloc / torch CUDA
 *     tensors) owned by the caller; pointers named *_host are host memory.
 *   - Bodies are closed curves given as boundary points ordered with the
 *     fluid on the right: counter-clockwise for obstacles, clockwise for an
 *     enclosing wall.  Boundary data is a rigid motion
 *     u_b(x) = u_rigid + omega_rigid * k x (x - center).
 *   - Every call returns an int status (IIM_OK = 0, < 0 on error); nothing
 *     throws across the ABI.  A failed call leaves a message readable with
 *     iim_last_error().
 *   - Compute calls are enqueued on the stream given to iim_create (a
 *     hipStream_t passed as void*; NULL = the null stream).  Calls that
 *     return host values (Gamma, statistics) synchronise that stream.
 *   - One context must not be used by two host threads at once.
 */
#ifndef IIM_H
#define IIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IIM_ABI_VERSION 3

enum {
  IIM_OK = 0,
  IIM_EINVAL = -1,        /* invalid argument (sizes, NULL pointers, dt too large) */
  IIM_ENOMEM = -2,        /* device or host allocation failed */
  IIM_EGEOM = -3,         /* geometry cannot be discretised (message names body / node) */
  IIM_ENOCONV = -4,       /* Krylov solver reached its iteration limit; results still written */
  IIM_ENONFINITE = -5,    /* NaN or Inf met in an input or a residual */
  IIM_EDEVICE = -6,       /* HIP runtime error */
  IIM_EUNSUPPORTED = -7   /* feature not available (e.g. compute on a host-only context) */
};

/* exterior condition of the Poisson solve (Sec. 4.1 and Sec. 5.2) */
enum {
  IIM_EXT_BOX = 0,        /* stream function zero on the box faces half a cell outside the edge nodes */
  IIM_EXT_FREE = 1,       /* unbounded domain: lattice Green's function convolution */
  IIM_EXT_OUTFLOW = 2,    /* unbounded, with the vorticity mirrored (even) across the face x_{nx-1/2} */
  IIM_EXT_PERIODIC = 3    /* periodic in x and y (Sec. 4.1): node i + nx is node i, j + ny is j; u_inf is
                             the mean velocity, the periodic part of the stream function has zero mean
                             (its source's mean is dropped), nx and ny are powers of two >= 32, and the
                             bodies' bounding regions lie inside the grid; steps keep the discrete
                             solvability sum h^2 sum_{outside every R_k} omega + sum_k Gamma_k, which the
                             caller's state must start at zero for the reconstruction to solve the
                             paper's problem */
};

/* Precision of the Krylov solve.  MIXED: once the GMRES residual estimate
 * has fallen below tol / 2e-6 (relative), the matrix-vector products apply
 * the Poisson operator with FP32 FFTs and an FP32 kernel spectrum (inexact
 * Krylov with relaxation: the FP32 operator's ~2e-7 relative error, times a
 * safety factor 10, stays below tol / |r_k|).  Free-space exteriors with FFT
 * sizes >= 256; otherwise FP64.  Every GMRES cycle ends with the FP64
 * residual b - S x, which alone decides convergence; cycles repeat until it
 * does (iterative refinement, at most max_refine cycles).  The right-hand
 * side, the psi recovery, the velocity, the IIM stencils, the transport and
 * the circulation sums stay FP64, so results meet the same tolerance as FP64.
 * The dense solver ignores the setting. */
enum { IIM_PREC_FP64 = 0, IIM_PREC_MIXED = 1 };
/* Initial guess of each Schur solve:
 *   ZERO        x = 0;
 *   PREVIOUS    the solution of the previous solve (previous RK stage);
 *   EXTRAPOLATE the line through the last two solutions extended to the
 *               current stage time (stages at t + c dt, c = 0, 1/3, 3/4; needs
 *               two earlier solves of the same run at a fixed dt);
 *   NETWORK     EXTRAPOLATE plus the correction predicted by a trained
 *               network (iim_set_warm_start), kept only when its residual is
 *               below that of PREVIOUS; needs three earlier solves.
 * Modes that lack their history fall back to PREVIOUS (ZERO on the first
 * solve).  With IIM_SOLVER_DIRECT the guess is not used. */
enum { IIM_GUESS_ZERO = 0, IIM_GUESS_PREVIOUS = 1, IIM_GUESS_EXTRAPOLATE = 2, IIM_GUESS_NETWORK = 3 };
/* Schur-system solver: GMRES with the FFT matrix-vector product (the paper's
 * iterative solve), or the dense inverse of the Schur matrix built once at
 * create (bodies are fixed, so the matrix is too). */
enum { IIM_SOLVER_KRYLOV = 0, IIM_SOLVER_DIRECT = 1 };
/* Lengths of the zero-padded free-space torus (at least 2 nx, or 4 nx with
 * the outflow mirror, by 2 ny; Sec. 4.2's free-space convolution is exact on
 * any such torus):
 *   TUNED    (default) times one full convolution on the COMPACT torus and
 *            on the POW2 torus at create (scratch tables, zero source) and
 *            keeps COMPACT only if it is at least 5 % faster; the same as
 *            COMPACT when the two coincide;
 *   COMPACT  the smallest length with a register FFT plan: powers of two and,
 *            for FP64 contexts whose row half-length and column length are
 *            both 256 or more, 320, 384, 640, 768, 1280 and 1536 points per
 *            row half and column (radix-3 and radix-5 passes); mixed precision
 *            uses powers of two;
 *   POW2     the next powers of two.
 * The periodic exterior uses the grid itself (powers of two). */
enum { IIM_FFT_SIZES_TUNED = 0, IIM_FFT_SIZES_COMPACT = 1, IIM_FFT_SIZES_POW2 = 2 };

typedef struct {
  int32_t nx, ny;         /* grid nodes per direction (>= 16) */
  double x0, y0, h;       /* coordinates of node (0,0) and the grid spacing */
  int32_t exterior;       /* IIM_EXT_* */
  double u_inf[2];        /* free stream (free-space exteriors only; ignored for the box) */
  double nu;              /* kinematic viscosity */
} iim_grid_desc;

typedef struct {
  int32_t n_points;       /* >= 4 */
  const double* xy_host;  /* [n_points][2], copied at create */
  int32_t is_enclosure;   /* 1: exterior wall (stream-function constant 0, no circulation unknown) */
  double center[2];       /* rigid-motion centre */
  double u_rigid[2];      /* rigid translation velocity */
  double omega_rigid;     /* rigid angular velocity */
  int32_t rect[4];        /* bounding region R_k as node ranges i0,i1,j0,j1 (inclusive); rect[0] < 0 = automatic */
  const double* bc_samples; /* optional host [n_points][3] = (u_x, u_y, psi_b) at the points, copied at
                             create: boundary velocity and stream function (Sec. 3.1 boundary conditions)
                             interpolated at the control points by periodic cubic splines in the curve's
                             parameter; psi_b is defined up to the body's constant psibar.  NULL: the
                             rigid motion above. */
} iim_body_desc;

typedef struct {
  int32_t precision;      /* IIM_PREC_* */
  double krylov_tol;      /* stop when ||r|| <= tol ||b|| (relative to b, so warm starts count) */
  int32_t krylov_max_iter;/* total matrix-vector products per solve */
  int32_t krylov_restart; /* GMRES restart length (<= 64) */
  int32_t max_refine;     /* mixed precision: maximum refinement rounds (<= 0: 8) */
  int32_t guess;          /* IIM_GUESS_* initial guess of each Schur solve */
  int32_t host_only;      /* 1: build geometry and tables only, allocate nothing on the device */
  int32_t solver;         /* IIM_SOLVER_*; DIRECT stores (|A| + n_circ)^2 doubles on the device */
  int32_t fft_sizes;      /* IIM_FFT_SIZES_* (free-space tori) */
} iim_solver_opts;

typedef struct {
  int32_t iters[3];       /* Krylov matrix-vector products of each RK stage (reconstruct: [0]) */
  int32_t refine_rounds[3];
  double res0[3];         /* initial relative residual of each stage */
  double res[3];          /* final relative residual of each stage */
  int32_t converged;      /* 1 if every stage met the tolerance */
} iim_step_stats;

typedef struct {
  int32_t nx, ny;
  int32_t n_control;      /* |C| */
  int32_t n_affected;     /* |A| = |A+| + |A-| */
  int32_t n_ghost;        /* |A-| */
  int32_t n_circ;         /* bodies carrying a circulation unknown */
  int32_t n_special;      /* fluid nodes handled by the boundary transport kernel */
  int32_t fft_mx, fft_my; /* padded FFT sizes (free space) */
  int32_t win_j0, win_j1; /* source rows / output rows of the pruned Krylov convolution */
  int64_t device_bytes;   /* device memory held by the context */
} iim_info;

/* Host views of the geometry tables (valid until iim_destroy). */
typedef struct {
  int32_t n_control;
  const double* c_xy;     /* [n_control][2] control point coordinates */
  const double* c_theta;  /* [n_control] distance fluid node -> control point, in units of h, (0,1] */
  const double* c_normal; /* [n_control][2] unit normal into the fluid */
  const int32_t* c_int;   /* [n_control][5] axis (0: horizontal line), sigma (+-1: ghost = fluid + sigma),
                             i_fluid, j_fluid, body */
  int32_t n_affected;
  const int32_t* a_int;   /* [n_affected][4] i, j, is_ghost, body */
  const int8_t* cls;      /* [ny][nx] 0 fluid, 1 ghost (A-), 2 solid interior */
  int32_t n_circ;
  const int32_t* rects;   /* [n_circ][4] i0, i1, j0, j1 */
  const int32_t* circ_body; /* [n_circ] body index of each circulation unknown */
  const double* c_ub;     /* [n_control][2] boundary velocity at the control points */
  const double* c_psib;   /* [n_control] boundary stream function psi_b at the control points */
} iim_geometry_view;

typedef struct iim_ctx iim_ctx;

int iim_abi_version(void);
const char* iim_status_string(int status);

/* Build a context: geometry (Sec. 2.2, App. A), stencil tables, the Poisson
 * operator of the exterior condition (Sec. 4.2) and all device workspaces.
 * Host inputs are copied.  Errors: IIM_EINVAL, IIM_EGEOM (with the body named
 * in the message), IIM_ENOMEM, IIM_EDEVICE.  On error *out is NULL. */
int iim_create(const iim_grid_desc* grid, int32_t n_bodies, const iim_body_desc* bodies,
               const iim_solver_opts* opts, void* hip_stream, iim_ctx** out);
int iim_destroy(iim_ctx* ctx);
/* Message of the last failed call on ctx; with ctx == NULL, the message of the
 * last failed iim_create on this host thread.  The string stays valid until
 * the next call on the same context (or thread). */
const char* iim_last_error(const iim_ctx* ctx);
int iim_query(const iim_ctx* ctx, iim_info* out);
int iim_get_geometry(const iim_ctx* ctx, iim_geometry_view* out);

/* Surface loads of the bodies (Sec. 5.4): shear stress tau = nu omega_b and the
 * surface pressure from the vorticity flux, d p / d s = nu d omega / d n on a
 * stationary no-slip wall, integrated along each body's control points in the
 * order of its curve's parameter from the first one (so p is relative to that
 * point), with omega extended past the boundary by E3b (with omega_b) and
 * differentiated with the stencil points of omega_b (Sec. 5.3); n is the unit
 * normal into the fluid, s = k x n.  Inputs on the device: omega [ny][nx], u
 * and v on the ring [ny+2][nx+2] with the ghost values of iim_reconstruct.
 * Outputs on the host: point_host [n_control][4] = (omega_b, tau, d omega/dn,
 * p), control points in the order of iim_get_geometry; body_host
 * [n_bodies][3] = (F_x, F_y, torque about the body's centre) of the traction
 * -p n + nu omega s, trapezoid rule over each closed polygon of control points
 * (a constant in p integrates to zero around a body).  A body in steady rigid
 * motion (constant u_rigid, omega_rigid): viscous traction nu (omega - 2
 * omega_rigid) s and the centripetal term omega_rigid^2 (x - c).s added to
 * d p / d s; bodies with bc_samples are treated as stationary walls.
 * Synchronises the stream.
 * IIM_EINVAL on null arguments; IIM_EUNSUPPORTED for host-only contexts and
 * for contexts given a time-dependent motion (iim_set_body_motion,
 * iim_rk3_steps_moving), whose wall accelerations the traction leaves out. */
int iim_surface_loads(iim_ctx* ctx, const double* omega_dev, const double* u_dev, const double* v_dev,
                      double* point_host, double* body_host);

/* Control-volume force and moment on the bodies inside a box (Sec. 5.4 and
 * its appendix: Noca's momentum formulation and the paper's analogue for the
 * moment, for stationary obstacles with no-slip walls and a stationary
 * control volume):
 *   F = S_gamma - d S_t / dt,    M = d I / dt + S_lambda,
 *   S_t      = oint_S [x (u.n) + x x (n x u)] dS,
 *   S_gamma  = oint_S n . [|u|^2/2 I - u u - u (x x omega k) + x.(div T) I
 *                          - x (div T) + T] dS,   T = nu (grad u + grad u^T),
 *   S_lambda = oint_S [|u|^2/2 (x x n) - (x x u)(u.n)
 *                      - |x|^2/2 n x (u x omega k) + |x|^2/2 (div T) x n
 *                      + x x (T.n)] dS,
 *   I        = int_V |x|^2/2 omega dV over the box minus the bodies.
 * With div u = 0 and u = 0 on the walls, the force's volume integral of u is
 * oint_S x (u.n) dS and the moment's two time-derivative terms are d I / dt,
 * so the caller forms F and M from values at successive times.  S is the
 * rectangle of grid lines through the nodes i0..i1 x j0..j1 (box = {i0, i1,
 * j0, j1}), n its outward normal, the trapezoid rule along its edges;
 * derivatives are centred differences of the node values, div T = nu (-d_y
 * omega, d_x omega).  I sums |x|^2/2 omega times the fluid area of each box
 * node's dual cell (h x h about the node, halved on the box's edges), omega
 * extended by E3b at the ghost nodes and zero at the other solid nodes; a cell
 * cut by a body loses its part inside the polygon of the body's boundary
 * points (an enclosure keeps that part).  x is measured from origin_host[2]
 * (M is the moment about it).  Inputs on the device: omega [ny][nx], u and v
 * on the ring [ny+2][nx+2] as iim_reconstruct writes them.  Output on the
 * host: out_host[6] = (S_t x, S_t y, S_gamma x, S_gamma y, I, S_lambda).
 * The first call computes the cut-cell areas once.  Synchronises the stream.
 * IIM_EINVAL on null arguments, a box outside 1 <= i0 < i1 <= nx-2,
 * 1 <= j0 < j1 <= ny-2, or a box node or one of its four neighbours that is
 * not a fluid node (named in iim_last_error); IIM_EUNSUPPORTED for host-only
 * contexts and when a body with a control point inside the box moves (rigid
 * motion or boundary samples: the formulation is for stationary walls). */
int iim_cv_terms(iim_ctx* ctx, const double* omega_dev, const double* u_dev, const double* v_dev,
                 const int32_t* box, const double* origin_host, double* out_host);

/* Time-dependent rigid motion of the bodies (Sec. 2: the boundary data u_b and
 * psi_b of each body's motion u + omega k x (x - centre) about its centre).
 * The boundary itself stays in place: the motion enters as boundary data,
 * the physical case for a motion that keeps the boundary where it is (a
 * circle rotating about its centre).
 * iim_set_body_motion sets motion_host[n_bodies][3] = (u_x, u_y, omega), in
 * the order of the bodies given to iim_create, for the calls that follow
 * (iim_reconstruct, iim_rhs, iim_rk3_steps).  iim_rk3_steps_moving runs
 * n_steps RK3 steps with the motion given at every stage's time:
 * motion_host[n_steps][3][n_bodies][3], stage s of step n at
 * t_n + c_s dt with c = (0, 1/3, 3/4), the stage times of the low-storage
 * RK3; afterwards the last stage's motion stays set.  The first call switches
 * the context for good from the composed boundary forms to the chained
 * boundary kernels (which read the boundary-data tables); with the dense
 * solver the moving steps run from a captured step graph whose stages copy
 * their tables from device memory staged before each step, and plain steps
 * run without the graph.  Results equal those of a fixed rigid motion when
 * the motion is constant.  Synchronises the stream after every step; stats (may
 * be NULL) receives the last step's.
 * IIM_EINVAL on null or non-finite arguments, dt <= 0 or n_steps < 0;
 * IIM_EUNSUPPORTED for host-only contexts and for bodies with bc_samples.
 * After either call iim_surface_loads returns IIM_EUNSUPPORTED (its
 * traction assumes steady motion) and iim_cv_terms takes the current
 * motion to decide which bodies move. */
int iim_set_body_motion(iim_ctx* ctx, const double* motion_host);
int iim_rk3_steps_moving(iim_ctx* ctx, double* omega_dev, double* Gamma_host, double dt, int32_t n_steps,
                         const double* motion_host, iim_step_stats* stats);

/* Largest stable time step on the RK3 stability triangle of App. B for a
 * velocity bound a_max = max(|u_x| + |u_y|):
 * dt = 1 / (a_max / (1.620 h) + nu / (0.314 h^2)). */
int iim_dt_max(const iim_ctx* ctx, double a_max, double* dt_max_out);
/* The step-size limit that the RK3 steps enforce: iim_dt_max at the
 * context's velocity bound.  That bound is sqrt(2) times the larger of twice
 * the free-stream speed (none for the box) and the largest boundary speed at
 * the control points (Sec. 5.5 leaves the bound open; the free-stream
 * doubling covers the speed-up past a body): set at create from the rigid
 * motion or the boundary samples, raised to the motion's speed by
 * iim_set_body_motion and, per call, by iim_rk3_steps_moving.
 * iim_set_speed_bound replaces it (a_max >= 0, finite) for good, e.g. with
 * the measured maximum of |u| + |v| of a developed flow.  iim_rk3_step(s),
 * iim_rk3_steps_moving and iim_batch_step return IIM_EINVAL, computing
 * nothing, when dt exceeds the limit. */
int iim_dt_limit(const iim_ctx* ctx, double* dt_limit_out);
int iim_set_speed_bound(iim_ctx* ctx, double a_max);

/* Lattice Green's function g(m, n) of the 5-point Laplacian (host, for
 * tests): out_host[n*(mx+1) + m] for 0 <= m <= mx, 0 <= n <= my. */
int iim_lgf_table(int32_t mx, int32_t my, double* out_host);

/* psi = G src with the context's exterior condition, no immersed bodies
 * (Sec. 4.2, the FFT solution operator).  src_dev: grid field; psi_dev:
 * ring field. */
int iim_poisson(iim_ctx* ctx, const double* src_dev, double* psi_dev);

/* iim_poisson with FP32 FFTs and kernel spectrum (the operator of the inner
 * products of the mixed-precision solve; inputs and output FP64).  Needs a
 * mixed-precision free-space context with FFT sizes >= 256, else
 * IIM_EUNSUPPORTED. */
int iim_poisson_fp32(iim_ctx* ctx, const double* src_dev, double* psi_dev);

/* Velocity reconstruction of one stage (Sec. 4.2): solves the Schur system
 * for gamma and the body constants, recovers psi, fills the ghost values and
 * the velocity (extended to A- at third order with u_b).
 * omega_dev: grid field (values at solid nodes ignored); Gamma_host:
 * [n_circ] circulations of the bounding regions R_k; psi_dev (nullable),
 * u_dev, v_dev: ring fields.  Returns IIM_ENOCONV if the Krylov limit was
 * hit (outputs still written). */
int iim_reconstruct(iim_ctx* ctx, const double* omega_dev, const double* Gamma_host,
                    double* psi_dev, double* u_dev, double* v_dev, iim_step_stats* stats);

/* Right-hand side of the transport equation and of the Kelvin ODE (Sec. 3,
 * Sec. 5.1, Sec. 5.3) for a given (extended) velocity.  u_dev, v_dev: ring
 * fields as written by iim_reconstruct; domega_dev: grid field (zero at
 * solid nodes); dGamma_host: [n_circ]; omega_b_dev (nullable): [n_control]. */
int iim_rhs(iim_ctx* ctx, const double* omega_dev, const double* u_dev, const double* v_dev,
            double* domega_dev, double* dGamma_host, double* omega_b_dev);

/* The same right-hand side with the wall vorticity given instead of computed
 * from the velocity: omega_b_dev [n_control] (device, the order of
 * iim_get_geometry) enters the vorticity extensions E4b and E3b, as in the
 * transport study of Sec. 3, whose body carries the exact solution's
 * boundary data.  Callers that prescribe the velocity too (a uniform stream)
 * pass it on the ring, ghost nodes included.  Synchronises the stream.
 * IIM_EINVAL on null arguments; IIM_EUNSUPPORTED for host-only contexts. */
int iim_rhs_given_wb(iim_ctx* ctx, const double* omega_dev, const double* u_dev, const double* v_dev,
                     const double* omega_b_dev, double* domega_dev, double* dGamma_host);

/* One low-storage RK3 step (Sec. 5.5) of (omega, Gamma) in place.
 * omega_dev: grid field; Gamma_host: [n_circ]; 0 < dt <= the context's
 * limit (iim_dt_limit), else IIM_EINVAL.  The RK update raises a device flag
 * when a new vorticity or circulation value is NaN or Inf; the call reads it
 * at its final synchronisation and returns IIM_ENONFINITE (the state holds
 * the non-finite values), on every solver path, the captured step graph of
 * the dense solver included. */
int iim_rk3_step(iim_ctx* ctx, double* omega_dev, double* Gamma_host, double dt,
                 iim_step_stats* stats);

/* Several RK3 steps with Gamma kept on the device between steps (synchronises
 * once at the end).  Same arguments as iim_rk3_step; stats (nullable) are
 * those of the last step. */
int iim_rk3_steps(iim_ctx* ctx, double* omega_dev, double* Gamma_host, double dt, int32_t n_steps,
                  iim_step_stats* stats);

/* ---- instrumentation (measurement of the kernels above; not part of the method) ----
 * iim_profile: drop collected timings and time every later launch of the
 * kernels whose id bit is set in kernel_mask with a pair of HIP events on the
 * context's stream (ids: 0 row FFT pass, 1 column FFT + kernel-multiply pass,
 * 2 inverse row FFT pass, 3 transport of all nodes + Kelvin + RK update, 4 Arnoldi step).
 * iim_profile_read: summed event time (ms), launch count and summed
 * algorithmic bytes of one kernel id since the last iim_profile.
 * iim_krylov_totals: Schur solves and Krylov matrix-vector products so far. */
int iim_profile(iim_ctx* ctx, int32_t kernel_mask);
int iim_profile_read(iim_ctx* ctx, int32_t kernel_id, double* total_ms, int64_t* launches, double* bytes);
int iim_krylov_totals(const iim_ctx* ctx, int64_t* solves, int64_t* matvecs);
/* FFT tile autotuner: times the full Poisson convolution of a stage (dense
 * source plus the correction sources; reps repeats, three interleaved rounds,
 * the minimum of each shape) with every instantiated number of FFTs per
 * workgroup of the row passes and of the column pass (1, 2, 4; shapes over
 * 1024 threads or 128 KiB of LDS fall back to the default; shapes whose
 * kernels the device cannot launch, or whose launches report an error, are
 * never chosen) and keeps the
 * fastest if it beats the default by at least 3 % (otherwise the default).
 * Outputs (nullable): the chosen counts (0 = default), the default's and the
 * best time per convolution in microseconds.  The shapes change only the
 * work per workgroup, not the arithmetic: results are bitwise the same.
 * No-op (zeros) for the box exterior and FFT sizes below 256. */
int iim_autotune(iim_ctx* ctx, int32_t reps, int32_t* row_per, int32_t* col_per, double* us_default,
                 double* us_best);
/* Set the FFTs per workgroup directly (0 = default), e.g. from another
 * context's autotune of the same FFT size.  IIM_EINVAL when the device
 * cannot launch the shape's kernels (register-limited block size, LDS per
 * block, scratch memory), with the kernel named in iim_last_error. */
int iim_set_fft_shape(iim_ctx* ctx, int32_t row_per, int32_t col_per);
/* All solver counters since create. */
typedef struct {
  int64_t solves;                   /* Schur solves */
  int64_t krylov_iterations;        /* Arnoldi steps (one product each) */
  int64_t fp32_products;            /* of which applied in FP32 (mixed precision) */
  int64_t initial_residual_matvecs; /* FP64 products for initial residuals of warm starts */
  int64_t network_kept, network_rejected;
  int64_t recorded;                 /* solves held by iim_record_solves */
} iim_counters;
int iim_solver_counters(const iim_ctx* ctx, iim_counters* out);
/* Repeat the largest launch of kernel id 0, 1 or 2 (the FFT passes; made
 * while it was timed) reps times back to back between one pair of HIP events
 * on the context's stream: average duration (ms) and algorithmic bytes of
 * that launch.  The repeats overwrite only the context's spectrum and
 * stream-function workspaces, which every reconstruction rebuilds before
 * reading them.  Per-launch event pairs also time the dispatch latency that
 * back-to-back launches hide; this is the duration a kernel profiler
 * reports. */
int iim_profile_replay(iim_ctx* ctx, int32_t kernel_id, int32_t reps, double* avg_ms, double* bytes);

/* ---- learned initial guess ----
 * A stack of circular 1D convolutions (kernel 5) with tanh-approximated GELU
 * between layers; the last layer has one output channel.  Layer l maps
 * lin[l] -> lout[l] channels with weights W_l[(tap*lin + ci)*lout + co] and
 * bias b_l[co]; output position p reads input positions (p + tap - 2) mod L
 * of its own sequence.  The flat parameter array is W_0, b_0, W_1, b_1, ...
 * Products run on the matrix cores with BF16 operands and FP32 accumulation
 * (bf16 = 1) or with FP32 operands (bf16 = 0).
 *
 * Ragged sequence batches: x_dev is float [batch][P][in_channels]; seq_dev is
 * int32 [3][P] on the device: for position p, the start of its sequence, the
 * sequence length and p's index inside it.  Outputs are float [batch][P]. */
typedef struct iim_net iim_net;
#define IIM_NET_FEATURES 10   /* input channels of the initial-guess network */
typedef struct {
  int32_t in_channels;    /* IIM_NET_FEATURES for use with iim_set_warm_start */
  int32_t width;          /* hidden channels */
  int32_t layers;         /* number of convolutions (>= 1) */
  int32_t bf16;           /* 1: BF16 operands, FP32 accumulation; 0: FP32 operands */
  uint64_t seed;          /* He-uniform initialisation of the weights, zero biases */
} iim_net_desc;

/* Create / destroy a network; work is enqueued on hip_stream. */
int iim_net_create(const iim_net_desc* desc, void* hip_stream, iim_net** out);
int iim_net_destroy(iim_net* net);
int64_t iim_net_num_params(const iim_net* net);
/* which = 0: parameters, 1: gradients of the last iim_net_grad_mse; n must
 * equal iim_net_num_params.  Synchronises the network's stream. */
int iim_net_get_params(const iim_net* net, int32_t which, float* host, int64_t n);
/* Replace the parameters (and reset the Adam moments). */
int iim_net_set_params(iim_net* net, const float* host, int64_t n);
int iim_net_forward(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                    float* y_dev);
/* iim_net_forward without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  iim_net_forward grows the network's activation
 * buffers with hipMalloc when batch * P exceeds what it holds; this call
 * keeps the hidden activations (16 MiB) and the partial sums of split
 * one-sample products (4 MiB) in a 20 MiB device array of the library
 * instead (one per GPU, held until the process ends) and writes the last
 * layer straight into y_dev, with the same kernels and the same splits: its
 * outputs are identical.  Limit: batch * P <= 2^21 / max hidden width (16384 positions
 * at width 128), else IIM_EINVAL naming the limit.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (two streams, or
 * two threads) race and must be serialised by the caller.  IIM_EINVAL as
 * iim_net_forward; IIM_EDEVICE if the array's address cannot be had. */
int iim_net_forward_noalloc(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                            float* y_dev);
/* Gradients of mean((y - target)^2) over batch*P outputs; loss_host
 * (nullable) receives the loss. */
int iim_net_grad_mse(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                     const float* target_dev, float* loss_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * current gradients. */
int iim_net_adam_step(iim_net* net, float lr);
/* One training step on a batch: iim_net_grad_mse followed by
 * iim_net_adam_step with learning rate lr (> 0), on the network's stream;
 * loss_host (nullable) receives the batch loss before the update.
 * IIM_EINVAL as either call. */
int iim_net_train_step(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                       const float* target_dev, float lr, float* loss_host);
int iim_net_save(const iim_net* net, const char* path);
int iim_net_load(iim_net* net, const char* path);

/* Select the initial guess (IIM_GUESS_*) of the context's Krylov solves;
 * net is required for IIM_GUESS_NETWORK (in_channels IIM_NET_FEATURES, one
 * output channel) and must outlive its use.  Not owned. */
int iim_set_warm_start(iim_ctx* ctx, int32_t guess, iim_net* net);
/* Record the right-hand side and the solution of every solve made inside an
 * RK step (up to capacity solves, device memory 2 * capacity * (|A| + n_circ)
 * doubles); capacity 0 stops recording.  Restarts the record. */
int iim_record_solves(iim_ctx* ctx, int32_t capacity);
/* Train net on the recorded solves: each sample is a recorded solve with
 * three predecessors of the same run; the loss is the mean square, over the
 * affected points, of the network output minus (x - x_base) / s_r, where x
 * is the recorded solution, x_base the extrapolated guess and s_r the RMS of
 * its residual over the corrections.  iters Adam steps with `batch` samples
 * drawn with the seed; loss_host (nullable, [iters]) receives the loss of
 * every step.  Errors: IIM_EINVAL when no recorded solve qualifies. */
int iim_warm_start_train(iim_ctx* ctx, iim_net* net, int32_t iters, int32_t batch, float lr, uint64_t seed,
                         float* loss_host);
/* The same over the records of n_ctx contexts (runs of different geometry or
 * viscosity; one network for all): each step draws its batch from one
 * context, chosen with probability proportional to its qualifying records,
 * so that every qualifying record is equally likely.  Works on the stream of
 * ctxs[0] after synchronizing every context's stream.  Errors: IIM_EINVAL
 * when no record of any context qualifies (message on ctxs[0]). */
int iim_warm_start_train_multi(iim_ctx* const* ctxs, int32_t n_ctx, iim_net* net, int32_t iters, int32_t batch,
                               float lr, uint64_t seed, float* loss_host);
/* The training loss of iim_warm_start_train over every qualifying record of
 * ctx (forward passes only, `batch` records per pass): *loss its mean,
 * *samples (nullable) the number of records.  For held-out validation. */
int iim_warm_start_loss(iim_ctx* ctx, iim_net* net, int32_t batch, double* loss, int64_t* samples);
/* Start a new run: the next solves do not extrapolate from, and recorded
 * samples do not reach back to, the solves made so far (call when the state
 * is replaced by one that does not continue the previous steps). */
int iim_reset_history(iim_ctx* ctx);
/* Counters: solves recorded; network guesses kept and rejected; matrix-vector
 * products spent on initial residuals (not counted as Krylov iterations). */
int iim_warm_start_stats(const iim_ctx* ctx, int64_t* recorded, int64_t* net_used, int64_t* net_rejected,
                         int64_t* extra_matvecs);
/* The network's input ordering for this context: P positions, perm_host[P]
 * (affected index of each position), seq_host[3][P] (as seq_dev above) and
 * geo_host[P][4] (ghost flag, boundary tangent x, y, signed distance / h).
 * Any output pointer may be NULL. */
int iim_warm_start_sequences(iim_ctx* ctx, int32_t* P, int32_t* perm_host, int32_t* seq_host, float* geo_host);

/* ---- batched serving ----
 * Many independent simulations (each a grid with its own bodies, as for
 * iim_create) advanced together: every simulation uses the dense Schur
 * solver in FP64 (opts->solver and opts->precision are overridden), and one
 * batch step is one HIP graph holding the RK3 steps of all simulations,
 * spread over parallel branches.  At create, the FFT tile autotuner runs
 * once per FFT size and the number of branches (1, 2, 4, 8) is chosen by
 * timing batch steps on scratch states; iim_batch_info reports both. */
typedef struct iim_batch iim_batch;
typedef struct {
  int32_t fft_mx, fft_my;   /* FFT size this choice applies to */
  int32_t tuned_on;         /* simulation it was timed on */
  int32_t row_per, col_per; /* FFTs per workgroup (0 = default) */
  double us_default, us_best; /* one full convolution, microseconds */
} iim_batch_tuning;
typedef struct {
  int32_t steps;
  int64_t cells_per_step;   /* grid nodes of all simulations */
  double ms_total;          /* sum of the batch-step times */
  double ms_p50, ms_p99, ms_max; /* batch-step time percentiles (HIP events around every graph launch) */
} iim_batch_stats;

/* grids[n_sims]; n_bodies[n_sims]; bodies[s] = the n_bodies[s] bodies of
 * simulation s.  Errors as iim_create (the message, from
 * iim_batch_last_error(NULL), names the simulation and ends with the free and
 * total device memory, the memory the simulations hold and the node count of
 * the last captured batch graph).  A branch count whose graph fails is
 * skipped (its time reads -1 in iim_batch_info, its error stays readable with
 * iim_batch_last_error(batch)); one branch must work. */
int iim_batch_create(int32_t n_sims, const iim_grid_desc* grids, const int32_t* n_bodies,
                     const iim_body_desc* const* bodies, const iim_solver_opts* opts, void* hip_stream,
                     iim_batch** out);
int iim_batch_destroy(iim_batch* batch);
const char* iim_batch_last_error(const iim_batch* batch);
/* n_steps RK3 steps of every simulation: omega_dev[s] grid field of
 * simulation s (in place), Gamma_host[s] its circulations (in place), dt[s]
 * its step.  The graph is captured on the first call and again whenever a
 * pointer or a dt changes.  stats (nullable).  IIM_EINVAL (nothing run) when
 * a dt exceeds its simulation's limit (iim_dt_limit); IIM_ENONFINITE when a
 * simulation's new state holds a NaN or Inf (named in iim_batch_last_error). */
int iim_batch_step(iim_batch* batch, double* const* omega_dev, double* const* Gamma_host, const double* dt,
                   int32_t n_steps, iim_batch_stats* stats);
/* Chosen branch count; the autotuner's choices (tunings: room for n_sims
 * entries, nullable) and their count; batch-step time (ms) of each branch
 * count tried, 1, 2, 4, 8 in that order (branch_ms: room for 4, nullable). */
int iim_batch_info(const iim_batch* batch, int32_t* n_branches, int32_t* n_tunings, iim_batch_tuning* tunings,
                   double* branch_ms);

#ifdef __cplusplus
}
#endif
#endif /* IIM_H */
