// Many independent simulations advanced together (batched serving).
//
// Every simulation is a context with the dense Schur solver (its bodies are
// fixed), so one RK3 step is a fixed sequence of kernels without host
// synchronisation.  A batch step captures the steps of all simulations into
// one HIP graph: the simulations are spread over parallel branches (streams
// forked from and joined into the capture stream), so the small kernels of
// different simulations run side by side on the 256 compute units, and one
// graph launch advances the whole batch.  At create, the FFT tile autotuner
// runs once per FFT size (its choice is applied to every simulation of that
// size) and the number of branches is picked by timing batch steps on
// scratch states.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace iim;

namespace {
thread_local std::string g_batch_error;
}

struct iim_batch {
  std::string err;
  std::vector<iim_ctx*> sims;
  std::vector<long> cells;
  hipStream_t stream = nullptr;            // caller's stream: graph launches, copies
  hipStream_t cap = nullptr;               // capture origin
  std::vector<hipStream_t> branches;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  int n_branches = 1;
  hipGraphExec_t exec = nullptr;
  std::vector<double*> g_omega;
  std::vector<double> g_dt;
  std::vector<iim_batch_tuning> tunes;
  std::vector<double> branch_ms;           // batch-step time of each branch count tried (-1: failed)
  std::vector<std::string> branch_err;     // why a branch count failed
  size_t graph_nodes = 0;                  // nodes of the last captured batch-step graph
  double setup_s = 0.0;
  ~iim_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (auto s : branches) (void)hipStreamDestroy(s);
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto c : sims) iim_destroy(c);
  }
};

namespace {

// Simulations to branches: largest first onto the least loaded branch.
std::vector<int> assign(const iim_batch* b, int nbr) {
  std::vector<int> order(b->sims.size()), out(b->sims.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->cells[x] > b->cells[y]; });
  std::vector<long> load(nbr, 0);
  for (int s : order) {
    const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    out[s] = br;
    load[br] += b->cells[s];
  }
  return out;
}

hipGraphExec_t capture(iim_batch* b, const std::vector<double*>& omega, const std::vector<double>& dt, int nbr) {
  HIPCHK(hipStreamSynchronize(b->stream));
  const std::vector<int> br = assign(b, nbr);
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  int rc = IIM_OK;
  try {
    HIPCHK(hipEventRecord(b->fork, b->cap));
    for (int q = 0; q < nbr; ++q) HIPCHK(hipStreamWaitEvent(b->branches[q], b->fork, 0));
    for (size_t s = 0; s < b->sims.size() && rc == IIM_OK; ++s) {
      iim_ctx* c = b->sims[s];
      hipStream_t user = c->stream;
      c->stream = b->branches[br[s]];
      rc = run_step(c, omega[s], dt[s], nullptr);
      c->stream = user;
    }
    for (int q = 0; q < nbr; ++q) {
      HIPCHK(hipEventRecord(b->join[q], b->branches[q]));
      HIPCHK(hipStreamWaitEvent(b->cap, b->join[q], 0));
    }
  } catch (...) {
    (void)hipStreamEndCapture(b->cap, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIPCHK(hipStreamEndCapture(b->cap, &graph));
  if (rc != IIM_OK) {
    (void)hipGraphDestroy(graph);
    throw HipError("step capture failed", rc);
  }
  size_t nodes = 0;
  if (hipGraphGetNodes(graph, nullptr, &nodes) == hipSuccess) b->graph_nodes = nodes;
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ei);
  return exec;
}

// State of the device and of the batch for error messages: free and total
// device memory, the memory the simulations hold, the last graph's size.
std::string diagnostics(const iim_batch* b) {
  size_t fr = 0, tot = 0;
  const bool mem = hipMemGetInfo(&fr, &tot) == hipSuccess;
  size_t held = 0;
  for (const iim_ctx* c : b->sims) held += c->dev_bytes;
  char buf[256];
  std::snprintf(buf, sizeof buf,
                " [device memory free %.3f of %.3f GiB; %zu simulations hold %.3f GiB; last batch graph %zu nodes]",
                mem ? fr / 1073741824.0 : -1.0, mem ? tot / 1073741824.0 : -1.0, b->sims.size(),
                held / 1073741824.0, b->graph_nodes);
  return buf;
}

// One batch step with nbr branches, captured, launched once to warm up and
// twice between events: its time in ms.
double time_branches(iim_batch* b, const std::vector<double*>& omega, const std::vector<double>& dt, int nbr,
                     hipEvent_t t0, hipEvent_t t1) {
  hipGraphExec_t ex = capture(b, omega, dt, nbr);
  try {
    HIPCHK(hipGraphLaunch(ex, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipEventRecord(t0, b->stream));
    HIPCHK(hipGraphLaunch(ex, b->stream));
    HIPCHK(hipGraphLaunch(ex, b->stream));
    HIPCHK(hipEventRecord(t1, b->stream));
    HIPCHK(hipEventSynchronize(t1));
  } catch (...) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(ex);
    throw;
  }
  float ms = 0.f;
  const hipError_t e = hipEventElapsedTime(&ms, t0, t1);
  (void)hipGraphExecDestroy(ex);
  HIPCHK(e);
  return ms / 2;
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p * (v.size() - 1);
  const size_t lo = (size_t)std::floor(pos), hi = std::min(v.size() - 1, lo + 1);
  return v[lo] + (pos - lo) * (v[hi] - v[lo]);
}

}  // namespace

extern "C" {

int iim_batch_create(int32_t n_sims, const iim_grid_desc* grids, const int32_t* n_bodies,
                     const iim_body_desc* const* bodies, const iim_solver_opts* opts, void* hip_stream,
                     iim_batch** out) {
  if (!out) return IIM_EINVAL;
  *out = nullptr;
  if (n_sims < 1 || !grids || !n_bodies || !bodies) return IIM_EINVAL;
  iim_batch* b = new (std::nothrow) iim_batch();
  if (!b) return IIM_ENOMEM;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<double*> scratch;
  auto release = [&]() {
    for (double* p : scratch)
      if (p) (void)hipFree(p);
    scratch.clear();
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    t0 = t1 = nullptr;
  };
  try {
    b->stream = (hipStream_t)hip_stream;
    iim_solver_opts o{};
    if (opts) o = *opts;
    o.solver = IIM_SOLVER_DIRECT;
    o.precision = IIM_PREC_FP64;
    o.host_only = 0;
    for (int s = 0; s < n_sims; ++s) {
      iim_ctx* c = nullptr;
      const int rc = iim_create(&grids[s], n_bodies[s], bodies[s], &o, hip_stream, &c);
      if (rc != IIM_OK) {
        g_batch_error = "simulation " + std::to_string(s) + ": " + iim_last_error(nullptr) + diagnostics(b);
        delete b;
        return rc;
      }
      c->use_graph = false;
      b->sims.push_back(c);
      b->cells.push_back((long)grids[s].nx * grids[s].ny);
    }
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    // FFT tiles: tune once per FFT size, apply to every simulation of that size
    std::map<std::pair<int, int>, iim_batch_tuning> by_size;
    for (int s = 0; s < n_sims; ++s) {
      iim_ctx* c = b->sims[s];
      if (c->box) continue;
      const std::pair<int, int> key{c->df.mx, c->df.my};
      auto it = by_size.find(key);
      if (it == by_size.end()) {
        iim_batch_tuning t{};
        t.fft_mx = c->df.mx;
        t.fft_my = c->df.my;
        t.tuned_on = s;
        const int rc = iim_autotune(c, 5, &t.row_per, &t.col_per, &t.us_default, &t.us_best);
        if (rc != IIM_OK) throw HipError("autotune of simulation " + std::to_string(s) + ": " + iim_last_error(c), rc);
        it = by_size.emplace(key, t).first;
        b->tunes.push_back(t);
      }
      const int rc = iim_set_fft_shape(c, it->second.row_per, it->second.col_per);
      if (rc != IIM_OK) throw HipError("tile shape of simulation " + std::to_string(s) + ": " + iim_last_error(c), rc);
    }
    // branches: time one batch step (after a warm-up step) of scratch states
    // for 1, 2, 4 and 8 branches and keep the fastest; a branch count whose
    // graph fails is recorded and skipped (one branch must work)
    HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    const int max_br = std::min(8, n_sims);
    for (int q = 0; q < max_br; ++q) {
      hipStream_t st;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->branches.push_back(st);
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->join.push_back(e);
    }
    scratch.assign(n_sims, nullptr);
    std::vector<double> dts(n_sims);
    for (int s = 0; s < n_sims; ++s) {
      HIPCHK(hipMalloc(&scratch[s], b->cells[s] * sizeof(double)));
      launch_fill(scratch[s], 0.0, b->cells[s], b->stream);
      dts[s] = 1e-3 * grids[s].h;
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipGetLastError());
    double best = 1e300;
    for (int nbr = 1; nbr <= max_br; nbr *= 2) {
      double ms = -1.0;
      try {
        ms = time_branches(b, scratch, dts, nbr, t0, t1);
      } catch (const HipError& e) {
        if (nbr == 1) throw;
        b->branch_err.push_back(std::to_string(nbr) + " branches: " + e.what());
        (void)hipGetLastError();
      }
      b->branch_ms.push_back(ms);
      if (ms >= 0 && ms < best) best = ms, b->n_branches = nbr;
    }
    for (iim_ctx* c : b->sims)
      if (take_nonfinite(c)) throw HipError("non-finite state in the branch timing of the scratch states", IIM_ENONFINITE);
    // failed branch counts stay readable through iim_batch_last_error(batch)
    for (const std::string& e : b->branch_err) b->err += e + "; ";
    release();
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    g_batch_error = e.what() + diagnostics(b);
    const int code = e.code;
    (void)hipStreamSynchronize(b->stream);
    release();
    delete b;
    return code;
  }
  *out = b;
  return IIM_OK;
}

int iim_batch_destroy(iim_batch* b) {
  if (!b) return IIM_EINVAL;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  delete b;
  return IIM_OK;
}

const char* iim_batch_last_error(const iim_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

int iim_batch_info(const iim_batch* b, int32_t* n_branches, int32_t* n_tunings, iim_batch_tuning* tunings,
                   double* branch_ms) {
  if (!b) return IIM_EINVAL;
  if (n_branches) *n_branches = b->n_branches;
  if (n_tunings) *n_tunings = (int32_t)b->tunes.size();
  if (tunings) std::copy(b->tunes.begin(), b->tunes.end(), tunings);
  if (branch_ms) std::copy(b->branch_ms.begin(), b->branch_ms.end(), branch_ms);
  return IIM_OK;
}

int iim_batch_step(iim_batch* b, double* const* omega_dev, double* const* Gamma_host, const double* dt,
                   int32_t n_steps, iim_batch_stats* stats) {
  if (!b || !omega_dev || !Gamma_host || !dt || n_steps < 0) return IIM_EINVAL;
  const size_t n = b->sims.size();
  for (size_t s = 0; s < n; ++s)
    if (!omega_dev[s] || !(dt[s] > 0) || (b->sims[s]->geo.nbc() > 0 && !Gamma_host[s])) return IIM_EINVAL;
  for (size_t s = 0; s < n; ++s) {
    const double lim = dt_limit(b->sims[s], b->sims[s]->a_max);
    if (dt[s] > lim * (1.0 + 1e-12)) {
      b->err = "simulation " + std::to_string(s) + ": dt = " + std::to_string(dt[s]) +
               " exceeds the RK3 stability limit " + std::to_string(lim);
      return IIM_EINVAL;
    }
  }
  std::vector<hipEvent_t> ev;
  try {
    for (size_t s = 0; s < n; ++s) {
      const int nb = b->sims[s]->geo.nbc();
      if (nb)
        HIPCHK(hipMemcpyAsync(b->sims[s]->Gd, Gamma_host[s], nb * sizeof(double), hipMemcpyHostToDevice, b->stream));
    }
    std::vector<double*> om(omega_dev, omega_dev + n);
    std::vector<double> d(dt, dt + n);
    if (!b->exec || om != b->g_omega || d != b->g_dt) {
      if (b->exec) {
        HIPCHK(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
      }
      b->exec = capture(b, om, d, b->n_branches);
      b->g_omega = om;
      b->g_dt = d;
    }
    ev.resize(n_steps + 1);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(ev[0], b->stream));
    for (int k = 0; k < n_steps; ++k) {
      HIPCHK(hipGraphLaunch(b->exec, b->stream));
      HIPCHK(hipEventRecord(ev[k + 1], b->stream));
    }
    for (size_t s = 0; s < n; ++s) {
      const int nb = b->sims[s]->geo.nbc();
      if (nb)
        HIPCHK(hipMemcpyAsync(Gamma_host[s], b->sims[s]->Gd, nb * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipGetLastError());
    for (size_t s = 0; s < n && n_steps > 0; ++s)
      if (take_nonfinite(b->sims[s])) {
        for (auto e2 : ev)
          if (e2) (void)hipEventDestroy(e2);
        b->err = "simulation " + std::to_string(s) + ": non-finite vorticity or circulation";
        return IIM_ENONFINITE;
      }
    std::vector<double> ms(n_steps);
    for (int k = 0; k < n_steps; ++k) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      ms[k] = t;
    }
    if (stats) {
      *stats = iim_batch_stats{};
      stats->steps = n_steps;
      stats->cells_per_step = std::accumulate(b->cells.begin(), b->cells.end(), 0L);
      stats->ms_total = std::accumulate(ms.begin(), ms.end(), 0.0);
      stats->ms_p50 = percentile(ms, 0.50);
      stats->ms_p99 = percentile(ms, 0.99);
      stats->ms_max = ms.empty() ? 0.0 : *std::max_element(ms.begin(), ms.end());
    }
  } catch (const HipError& e) {
    for (auto e2 : ev)
      if (e2) (void)hipEventDestroy(e2);
    b->err = e.what();
    return e.code;
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  return IIM_OK;
}

}  // extern "C"
