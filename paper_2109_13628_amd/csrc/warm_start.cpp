// Initial guesses of the Schur solve and the network that improves them.
//
// Consecutive RK stages solve S x = b with slowly changing b.  Besides the
// previous solution, the solve history gives x_base = x_1 + a (x_1 - x_2),
// the straight line through the last two solutions extended to the current
// stage time (a from the stage times t + c dt, c = 0, 1/3, 3/4).  Because S
// is fixed, the residual of x_base follows from the history alone:
// b - S x_base = b_0 - (1 + a) b_1 + a b_2 (up to the previous solves'
// tolerance).  The network reads that residual, the last two solution
// increments and the local geometry along each body, and predicts the error
// x - x_base of the corrections, in units of the residual's RMS (trained on
// recorded solves by least squares on that error: a loss on the residual
// norm instead lowers the initial residual but not the GMRES iterations,
// which depend on the error in the slowly converging directions).  Its guess
// is kept only when its true residual is below the previous-stage residual
// |b_0 - b_1|.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace iim;

// Scratch of the allocation-free forward pass (iim_net_forward_noalloc): the
// hidden layers' outputs alternate between the two halves of the first
// NET_SCRATCH_FLOATS floats, and the split products' partial sums use the
// CONV_FWD_PART_MAX floats after them; every GPU the library runs on holds
// this file-scope array for the life of the process.
constexpr size_t NET_SCRATCH_FLOATS = (size_t)4 << 20;   // 16 MiB of activations
static __device__ __align__(256) float scratch[NET_SCRATCH_FLOATS + CONV_FWD_PART_MAX];

namespace {

// Device address of the current GPU's scratch array, resolved once per device
// with that device current (the array's name is not a device address in host
// code); a fixed table, so that no call allocates.
constexpr int MAX_DEVICES = 256;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_address(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return IIM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IIM_EDEVICE;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return IIM_OK;
}

}  // namespace

iim_net::~iim_net() {
  for (void* p : act_allocs) (void)hipFree(p);
  for (void* p : allocs) (void)hipFree(p);
}

namespace {

template <class T>
T* net_alloc(std::vector<void*>& list, size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, n * sizeof(T)));
  list.push_back(p);
  return (T*)p;
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

void ensure_rows(iim_net* net, size_t rows) {
  if (rows <= net->cap_rows) return;
  for (void* p : net->act_allocs) (void)hipFree(p);
  net->act_allocs.clear();
  size_t cap = std::max(rows, (size_t)1024);
  const int L = net->layers;
  net->Z.assign(L, nullptr);
  net->H.assign(L, nullptr);
  int wmax = 1;
  for (int l = 0; l < L; ++l) {
    net->Z[l] = net_alloc<float>(net->act_allocs, cap * net->lout[l]);
    net->H[l] = net_alloc<float>(net->act_allocs, cap * net->lout[l]);
    wmax = std::max(wmax, std::max(net->lout[l], net->lin[l]));
  }
  net->dA = net_alloc<float>(net->act_allocs, cap * wmax);
  net->dB = net_alloc<float>(net->act_allocs, cap * wmax);
  net->dY = net_alloc<float>(net->act_allocs, cap);
  net->fwd_part = net_alloc<float>(net->act_allocs, CONV_FWD_PART_MAX);
  size_t kn = 0;
  for (int l = 0; l < L; ++l) kn = std::max(kn, (size_t)NET_TAPS * net->lin[l] * net->lout[l]);
  net->part_cap = (size_t)conv_bwd_w_splits((int)std::min(cap, (size_t)1 << 30)) * kn;
  net->part = net_alloc<float>(net->act_allocs, net->part_cap);
  net->cap_rows = cap;
}

void net_backward(iim_net* net, const Seq& s, int B, const float* X, const float* dY, hipStream_t st) {
  const int L = net->layers;
  const int rows = B * s.P;
  const int splits = conv_bwd_w_splits(rows);
  const float* dcur = dY;
  for (int l = L - 1; l >= 0; --l) {
    const float* Hin = l == 0 ? X : net->H[l - 1];
    launch_conv_bwd_w(net->bf16, s, B, Hin, net->lin[l], dcur, net->lout[l], net->part, splits,
                      net->grads + net->offW[l], net->grads + net->offb[l], st);
    if (l > 0) {
      float* dn = (dcur == net->dA) ? net->dB : net->dA;
      launch_conv_bwd_data(net->bf16, s, B, dcur, net->lout[l], net->params + net->offW[l], net->lin[l],
                           net->Z[l - 1], dn, st);
      dcur = dn;
    }
  }
}

void adam(iim_net* net, float lr, hipStream_t st) {
  net->t += 1;
  launch_adam(net->params, net->grads, net->m, net->v, net->nparam, lr, net->beta1, net->beta2, net->eps, net->t, st);
}

// ---------------------------------------------------------------- IIM side
// Affected points of every body ordered along its boundary: by the nearest
// input boundary point, then by signed distance (ghosts negative).
void ensure_sequences(iim_ctx* c) {
  if (c->perm) return;
  const Geometry& g = c->geo;
  const double h = g.grid.h;
  std::vector<int> perm, seg0, segl, pos;
  std::vector<float> geo;
  for (size_t k = 0; k < g.bodies.size(); ++k) {
    const auto& xy = g.bodies[k].xy;
    const int np = (int)xy.size() / 2;
    struct Item { int a, idx; double sd; };
    std::vector<Item> items;
    for (int a = 0; a < g.na; ++a) {
      if (g.a_body[a] != (int)k) continue;
      const double x = g.grid.x0 + h * g.a_i[a], y = g.grid.y0 + h * g.a_j[a];
      int best = 0;
      double bd = 1e300;
      for (int q = 0; q < np; ++q) {
        const double dx = xy[2 * q] - x, dy = xy[2 * q + 1] - y, d = dx * dx + dy * dy;
        if (d < bd) bd = d, best = q;
      }
      items.push_back({a, best, (g.a_ghost[a] ? -1.0 : 1.0) * std::sqrt(bd) / h});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& u, const Item& v) {
      return u.idx != v.idx ? u.idx < v.idx : u.sd < v.sd;
    });
    const int start = (int)perm.size(), L = (int)items.size();
    for (int q = 0; q < L; ++q) {
      const Item& it = items[q];
      perm.push_back(it.a);
      seg0.push_back(start);
      segl.push_back(L);
      pos.push_back(q);
      const int qa = (it.idx + 1) % np, qb = (it.idx + np - 1) % np;
      double tx = xy[2 * qa] - xy[2 * qb], ty = xy[2 * qa + 1] - xy[2 * qb + 1];
      const double tn = std::hypot(tx, ty);
      tx /= tn > 0 ? tn : 1.0;
      ty /= tn > 0 ? tn : 1.0;
      geo.push_back(g.a_ghost[it.a] ? 1.f : 0.f);
      geo.push_back((float)tx);
      geo.push_back((float)ty);
      geo.push_back((float)it.sd);
    }
  }
  c->seq_P = (int)perm.size();
  std::vector<int> seq(seg0);
  seq.insert(seq.end(), segl.begin(), segl.end());
  seq.insert(seq.end(), pos.begin(), pos.end());
  c->perm = c->upload(perm);
  c->seq = c->upload(seq);
  c->seq_geo = c->upload(geo);
}

Seq ctx_seq(const iim_ctx* c) {
  return Seq{c->seq, c->seq + c->seq_P, c->seq + 2 * c->seq_P, c->seq_P};
}

bool history_on(const iim_ctx* c) {
  return c->guess == IIM_GUESS_EXTRAPOLATE || c->guess == IIM_GUESS_NETWORK || c->rec_cap > 0;
}

void ensure_history(iim_ctx* c) {
  if (c->hb) return;
  const int n = c->dk.n;
  c->hb = c->dalloc<double>((size_t)4 * n);
  c->hx = c->dalloc<double>((size_t)4 * n);
  std::vector<int> tab(3 * 4 * 8);
  for (int s = 0; s < 3; ++s)
    for (int q = 0; q < 4; ++q) {
      int* t = &tab[(4 * s + q) * 8];
      t[0] = q;
      t[1] = (q + 3) % 4;
      t[2] = (q + 2) % 4;
      t[3] = (q + 3) % 4;
      t[4] = (q + 2) % 4;
      t[5] = (q + 1) % 4;
      t[6] = s;
      t[7] = 0;
    }
  c->hs_ring = c->upload(tab);
  ensure_sequences(c);
  c->inf_F = c->dalloc<float>((size_t)std::max(1, c->seq_P) * NET_FEATURES);
  c->inf_scale = c->dalloc<float>(1);
}

int check_net(const iim_net* net) {
  if (!net) return IIM_EINVAL;
  if (net->cin != NET_FEATURES || net->lout.back() != 1) return IIM_EINVAL;
  return IIM_OK;
}

}  // namespace

// ------------------------------------------------------------------ hooks
void iim::net_forward(iim_net* net, const Seq& s, int B, const float* X, bool keep_pre, hipStream_t st) {
  ensure_rows(net, (size_t)B * s.P);
  const float* in = X;
  for (int l = 0; l < net->layers; ++l) {
    const bool last = l == net->layers - 1;
    launch_conv_fwd(net->bf16, s, B, in, net->lin[l], net->params + net->offW[l], net->params + net->offb[l],
                    net->lout[l], (keep_pre && !last) ? net->Z[l] : nullptr, net->H[l], last ? 0 : 1, net->fwd_part,
                    st);
    in = net->H[l];
  }
}

int iim::prepare_guess(iim_ctx* c) {
  const int want = c->guess;
  if (want == IIM_GUESS_ZERO || !c->have_prev) return IIM_GUESS_ZERO;
  if (want == IIM_GUESS_PREVIOUS || c->cur_stage < 0) return IIM_GUESS_PREVIOUS;
  const int need = want == IIM_GUESS_NETWORK ? 3 : 2;
  if (c->hist_count < need || (want == IIM_GUESS_NETWORK && !c->net)) return IIM_GUESS_PREVIOUS;
  ensure_history(c);
  const DKrylov& k = c->dk;
  const int slot = (int)(c->hist_next % 4);
  HIPCHK(hipMemcpyAsync(c->hb + (size_t)slot * k.n, k.b, k.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  NetPrep p{};
  p.bh = c->hb;
  p.xh = c->hx;
  p.hs = c->hs_ring + 8 * (4 * c->cur_stage + slot);
  p.perm = c->perm;
  p.geo = c->seq_geo;
  p.n = k.n;
  p.na = c->dg.na;
  p.P = c->seq_P;
  p.F = c->inf_F;
  p.tgt = nullptr;
  p.scale = c->inf_scale;
  p.xbase = k.x;
  p.prevres = k.st + KS_PREVRES;
  launch_net_prep(p, 1, c->stream);
  if (want == IIM_GUESS_NETWORK) {
    net_forward(c->net, ctx_seq(c), 1, c->inf_F, false, c->stream);
    launch_net_apply(c->perm, c->seq_P, c->net->H.back(), c->inf_scale, k.x, c->stream);
  }
  return want;
}

void iim::push_history(iim_ctx* c) {
  if (!history_on(c)) return;
  if (c->solver == IIM_SOLVER_DIRECT && c->rec_cap == 0) return;  // no guesses to prepare
  if (c->cur_stage < 0) {     // a solve outside an RK step breaks the sequence
    c->hist_count = 0;
    ++c->run_id;
    return;
  }
  ensure_history(c);
  const DKrylov& k = c->dk;
  const int slot = (int)(c->hist_next % 4);
  HIPCHK(hipMemcpyAsync(c->hb + (size_t)slot * k.n, k.b, k.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->hx + (size_t)slot * k.n, k.x, k.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->hist_next += 1;
  c->hist_count = std::min(c->hist_count + 1, 4);
  if (c->rec_cap > 0 && c->rec_count < c->rec_cap) {
    const size_t off = (size_t)c->rec_count * k.n;
    HIPCHK(hipMemcpyAsync(c->rb + off, k.b, k.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->rx + off, k.x, k.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    c->rec_stage.push_back(c->cur_stage);
    c->rec_run.push_back(c->run_id);
    c->rec_count += 1;
  }
}

void iim::restore_previous(iim_ctx* c) {
  const DKrylov& k = c->dk;
  const int slot = (int)((c->hist_next + 3) % 4);
  HIPCHK(hipMemcpyAsync(k.x, c->hx + (size_t)slot * k.n, k.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
}

// ================================================================== ABI
extern "C" {

int iim_net_create(const iim_net_desc* d, void* hip_stream, iim_net** out) {
  if (!out) return IIM_EINVAL;
  *out = nullptr;
  if (!d || d->in_channels < 1 || d->width < 1 || d->layers < 1 || d->in_channels > 4096 || d->width > 4096 ||
      d->layers > 64)
    return IIM_EINVAL;
  iim_net* net = new (std::nothrow) iim_net();
  if (!net) return IIM_ENOMEM;
  try {
    net->cin = d->in_channels;
    net->width = d->width;
    net->layers = d->layers;
    net->bf16 = d->bf16 != 0;
    net->stream = (hipStream_t)hip_stream;
    for (int l = 0; l < net->layers; ++l) {
      net->lin.push_back(l == 0 ? net->cin : net->width);
      net->lout.push_back(l == net->layers - 1 ? 1 : net->width);
    }
    size_t off = 0;
    for (int l = 0; l < net->layers; ++l) {
      net->offW.push_back(off);
      off += (size_t)NET_TAPS * net->lin[l] * net->lout[l];
      net->offb.push_back(off);
      off += net->lout[l];
    }
    net->nparam = off;
    net->params = net_alloc<float>(net->allocs, off);
    net->grads = net_alloc<float>(net->allocs, off);
    net->m = net_alloc<float>(net->allocs, off);
    net->v = net_alloc<float>(net->allocs, off);
    net->lossbuf = net_alloc<float>(net->allocs, 1);
    // He-style uniform weights, zero biases
    std::vector<float> p(off, 0.f);
    uint64_t s = d->seed;
    for (int l = 0; l < net->layers; ++l) {
      const double lim = std::sqrt(6.0 / (NET_TAPS * net->lin[l]));
      for (size_t i = net->offW[l]; i < net->offb[l]; ++i) p[i] = (float)((2.0 * uniform01(s) - 1.0) * lim);
    }
    HIPCHK(hipMemcpy(net->params, p.data(), off * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(net->grads, 0, off * sizeof(float)));
    HIPCHK(hipMemset(net->m, 0, off * sizeof(float)));
    HIPCHK(hipMemset(net->v, 0, off * sizeof(float)));
    // the allocation-free forward pass's scratch on this device, resolved at
    // set-up (a later first call on another device resolves that one)
    float* sp = nullptr;
    if (scratch_address(&sp) != IIM_OK) throw HipError("scratch array address unavailable", IIM_EDEVICE);
  } catch (const HipError& e) {
    const int code = e.code;
    delete net;
    return code;
  }
  *out = net;
  return IIM_OK;
}

int iim_net_destroy(iim_net* net) {
  if (!net) return IIM_EINVAL;
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  delete net;
  return IIM_OK;
}

int64_t iim_net_num_params(const iim_net* net) { return net ? (int64_t)net->nparam : -1; }

int iim_net_get_params(const iim_net* net, int32_t which, float* host, int64_t n) {
  if (!net || !host || n != (int64_t)net->nparam || which < 0 || which > 1) return IIM_EINVAL;
  if (hipStreamSynchronize(net->stream) != hipSuccess) return IIM_EDEVICE;
  if (hipMemcpy(host, which == 0 ? net->params : net->grads, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return IIM_EDEVICE;
  return IIM_OK;
}

int iim_net_set_params(iim_net* net, const float* host, int64_t n) {
  if (!net || !host || n != (int64_t)net->nparam) return IIM_EINVAL;
  if (hipStreamSynchronize(net->stream) != hipSuccess) return IIM_EDEVICE;
  if (hipMemcpy(net->params, host, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return IIM_EDEVICE;
  // a new parameter set restarts Adam
  net->t = 0;
  if (hipMemset(net->m, 0, n * sizeof(float)) != hipSuccess) return IIM_EDEVICE;
  if (hipMemset(net->v, 0, n * sizeof(float)) != hipSuccess) return IIM_EDEVICE;
  return IIM_OK;
}

int iim_net_forward(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                    float* y_dev) {
  if (!net || !x_dev || !seq_dev || !y_dev || batch < 1 || P < 1) return IIM_EINVAL;
  if (net->lout.back() != 1) return IIM_EINVAL;
  try {
    const Seq s{seq_dev, seq_dev + P, seq_dev + 2 * P, P};
    net_forward(net, s, batch, x_dev, false, net->stream);
    HIPCHK(hipMemcpyAsync(y_dev, net->H.back(), (size_t)batch * P * sizeof(float), hipMemcpyDeviceToDevice,
                          net->stream));
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    net->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

int iim_net_forward_noalloc(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                            float* y_dev) {
  if (!net || !x_dev || !seq_dev || !y_dev || batch < 1 || P < 1) return IIM_EINVAL;
  if (net->lout.back() != 1) return IIM_EINVAL;
  size_t wmax = 1;
  for (int l = 0; l + 1 < net->layers; ++l) wmax = std::max(wmax, (size_t)net->lout[l]);
  const size_t rows = (size_t)batch * P;
  if (rows > NET_SCRATCH_FLOATS / (2 * wmax)) {
    net->err = "iim_net_forward_noalloc: batch * P = " + std::to_string(rows) + " exceeds the scratch limit of " +
               std::to_string(NET_SCRATCH_FLOATS / (2 * wmax)) + " positions for hidden width " + std::to_string(wmax);
    return IIM_EINVAL;
  }
  float* buf = nullptr;
  if (scratch_address(&buf) != IIM_OK) {
    net->err = "iim_net_forward_noalloc: scratch array address unavailable";
    return IIM_EDEVICE;
  }
  try {
    const Seq s{seq_dev, seq_dev + P, seq_dev + 2 * P, P};
    const float* in = x_dev;
    for (int l = 0; l < net->layers; ++l) {
      const bool last = l == net->layers - 1;
      // hidden layers alternate between the scratch halves; the last writes y
      float* out = last ? y_dev : buf + (size_t)(l & 1) * rows * wmax;
      launch_conv_fwd(net->bf16, s, batch, in, net->lin[l], net->params + net->offW[l], net->params + net->offb[l],
                      net->lout[l], nullptr, out, last ? 0 : 1, buf + NET_SCRATCH_FLOATS, net->stream);
      in = out;
    }
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    net->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

int iim_net_grad_mse(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                     const float* target_dev, float* loss_host) {
  if (!net || !x_dev || !seq_dev || !target_dev || batch < 1 || P < 1) return IIM_EINVAL;
  if (net->lout.back() != 1) return IIM_EINVAL;
  try {
    const Seq s{seq_dev, seq_dev + P, seq_dev + 2 * P, P};
    net_forward(net, s, batch, x_dev, true, net->stream);
    const size_t cnt = (size_t)batch * P;
    launch_mse(net->H.back(), target_dev, cnt, net->dY, net->lossbuf, net->stream);
    net_backward(net, s, batch, x_dev, net->dY, net->stream);
    if (loss_host) {
      float l = 0.f;
      HIPCHK(hipMemcpyAsync(&l, net->lossbuf, sizeof(float), hipMemcpyDeviceToHost, net->stream));
      HIPCHK(hipStreamSynchronize(net->stream));
      *loss_host = l;
    }
    HIPCHK(hipGetLastError());
  } catch (const HipError& e) {
    net->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

int iim_net_adam_step(iim_net* net, float lr) {
  if (!net || !(lr > 0.f)) return IIM_EINVAL;
  adam(net, lr, net->stream);
  return hipGetLastError() == hipSuccess ? IIM_OK : IIM_EDEVICE;
}

int iim_net_train_step(iim_net* net, const float* x_dev, int32_t batch, int32_t P, const int32_t* seq_dev,
                       const float* target_dev, float lr, float* loss_host) {
  if (!(lr > 0.f)) return IIM_EINVAL;
  const int rc = iim_net_grad_mse(net, x_dev, batch, P, seq_dev, target_dev, loss_host);
  if (rc != IIM_OK) return rc;
  return iim_net_adam_step(net, lr);
}

int iim_net_save(const iim_net* net, const char* path) {
  if (!net || !path) return IIM_EINVAL;
  std::vector<float> p(net->nparam);
  const int rc = iim_net_get_params(net, 0, p.data(), (int64_t)p.size());
  if (rc != IIM_OK) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return IIM_EINVAL;
  const char magic[8] = {'I', 'I', 'M', 'N', 'E', 'T', '0', '1'};
  const int32_t dims[4] = {net->cin, net->width, net->layers, net->bf16 ? 1 : 0};
  const int64_t np = (int64_t)net->nparam;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(dims, sizeof(int32_t), 4, f) == 4 &&
            std::fwrite(&np, sizeof(np), 1, f) == 1 && std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? IIM_OK : IIM_EINVAL;
}

int iim_net_load(iim_net* net, const char* path) {
  if (!net || !path) return IIM_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return IIM_EINVAL;
  char magic[8];
  int32_t dims[4];
  int64_t np = 0;
  std::vector<float> p(net->nparam);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "IIMNET01", 8) == 0 &&
            std::fread(dims, sizeof(int32_t), 4, f) == 4 && std::fread(&np, sizeof(np), 1, f) == 1 &&
            dims[0] == net->cin && dims[1] == net->width && dims[2] == net->layers && np == (int64_t)net->nparam &&
            std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  if (!ok) {
    net->err = "not a network file of this shape";
    return IIM_EINVAL;
  }
  return iim_net_set_params(net, p.data(), np);
}

int iim_set_warm_start(iim_ctx* c, int32_t guess, iim_net* net) {
  if (!c) return IIM_EINVAL;
  if (guess < IIM_GUESS_ZERO || guess > IIM_GUESS_NETWORK) return IIM_EINVAL;
  if (guess == IIM_GUESS_NETWORK && check_net(net) != IIM_OK) {
    c->err = "the network must take the initial-guess features and have one output channel";
    return IIM_EINVAL;
  }
  c->guess = guess;
  c->net = guess == IIM_GUESS_NETWORK ? net : nullptr;
  return IIM_OK;
}

int iim_record_solves(iim_ctx* c, int32_t capacity) {
  if (!c || capacity < 0) return IIM_EINVAL;
  if (c->host_only) return IIM_EUNSUPPORTED;
  try {
    if (capacity > c->rec_cap) {
      const size_t n = c->dk.n;
      c->rb = c->dalloc<double>((size_t)capacity * n);
      c->rx = c->dalloc<double>((size_t)capacity * n);
    }
    c->rec_cap = capacity;
    c->rec_count = 0;
    c->rec_stage.clear();
    c->rec_run.clear();
    c->hist_count = 0;
    ++c->run_id;
    // recording needs the eager step (the graph would replay fixed slots)
    if (c->gexec) {
      HIPCHK(hipGraphExecDestroy(c->gexec));
      c->gexec = nullptr;
    }
  } catch (const HipError& e) {
    c->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

int iim_reset_history(iim_ctx* c) {
  if (!c) return IIM_EINVAL;
  c->hist_count = 0;
  c->have_prev = false;
  ++c->run_id;
  return IIM_OK;
}

int iim_warm_start_stats(const iim_ctx* c, int64_t* recorded, int64_t* net_used, int64_t* net_rejected,
                         int64_t* extra_matvecs) {
  if (!c) return IIM_EINVAL;
  if (recorded) *recorded = c->rec_count;
  if (net_used) *net_used = c->n_net_used;
  if (net_rejected) *net_rejected = c->n_net_rejected;
  if (extra_matvecs) *extra_matvecs = c->n_extra_matvecs;
  return IIM_OK;
}

int iim_warm_start_train(iim_ctx* c, iim_net* net, int32_t iters, int32_t batch, float lr, uint64_t seed,
                         float* loss_host) {
  return iim_warm_start_train_multi(&c, 1, net, iters, batch, lr, seed, loss_host);
}

int iim_warm_start_train_multi(iim_ctx* const* ctxs, int32_t n_ctx, iim_net* net, int32_t iters, int32_t batch,
                               float lr, uint64_t seed, float* loss_host) {
  if (!ctxs || n_ctx < 1) return IIM_EINVAL;
  for (int q = 0; q < n_ctx; ++q)
    if (!ctxs[q]) return IIM_EINVAL;
  iim_ctx* c0 = ctxs[0];
  if (check_net(net) != IIM_OK || iters < 1 || batch < 1 || !(lr > 0.f)) return IIM_EINVAL;
  for (int q = 0; q < n_ctx; ++q)
    if (ctxs[q]->host_only) return IIM_EUNSUPPORTED;
  // the usable records of every context: three predecessors in the same run
  std::vector<std::vector<int>> valid(n_ctx);
  size_t total = 0;
  for (int q = 0; q < n_ctx; ++q) {
    const iim_ctx* c = ctxs[q];
    for (int m = 3; m < c->rec_count; ++m)
      if (c->rec_run[m - 3] == c->rec_run[m]) valid[q].push_back(m);
    total += valid[q].size();
  }
  if (total == 0) {
    c0->err = "no recorded solve has three predecessors in the same run";
    return IIM_EINVAL;
  }
  iim_ctx* failed = c0;
  try {
    // every context's records are complete before the training stream reads them
    for (int q = 0; q < n_ctx; ++q) {
      failed = ctxs[q];
      HIPCHK(hipStreamSynchronize(ctxs[q]->stream));
      ensure_sequences(ctxs[q]);
    }
    failed = c0;
    hipStream_t st = c0->stream;
    int Pmax = 1;
    for (int q = 0; q < n_ctx; ++q) Pmax = std::max(Pmax, ctxs[q]->seq_P);
    std::vector<void*> tmp;
    struct Free {
      std::vector<void*>& l;
      ~Free() {
        for (void* p : l) (void)hipFree(p);
      }
    } fr{tmp};
    float* F = net_alloc<float>(tmp, (size_t)batch * Pmax * NET_FEATURES);
    float* tgt = net_alloc<float>(tmp, (size_t)batch * Pmax);
    float* scale = net_alloc<float>(tmp, batch);
    float* losses = net_alloc<float>(tmp, iters);
    int* hs = net_alloc<int>(tmp, (size_t)iters * batch * 8);
    // each iteration draws its batch from one context (one boundary
    // sequence), the context chosen in proportion to its usable records
    std::vector<int> h_hs((size_t)iters * batch * 8), which(iters);
    uint64_t s = seed;
    for (int it = 0; it < iters; ++it) {
      size_t pick = (size_t)(uniform01(s) * total) % total;
      int q = 0;
      while (pick >= valid[q].size()) pick -= valid[q++].size();
      which[it] = q;
      const std::vector<int>& vq = valid[q];
      for (int e = 0; e < batch; ++e) {
        const int m = vq[(size_t)(uniform01(s) * vq.size()) % vq.size()];
        int* t = &h_hs[8 * ((size_t)it * batch + e)];
        t[0] = m;
        t[1] = m - 1;
        t[2] = m - 2;
        t[3] = m - 1;
        t[4] = m - 2;
        t[5] = m - 3;
        t[6] = ctxs[q]->rec_stage[m];
        t[7] = m;
      }
    }
    HIPCHK(hipMemcpy(hs, h_hs.data(), h_hs.size() * sizeof(int), hipMemcpyHostToDevice));
    ensure_rows(net, (size_t)batch * Pmax);   // no regrowth (and free) between queued launches
    for (int it = 0; it < iters; ++it) {
      const iim_ctx* c = ctxs[which[it]];
      const Seq sq = ctx_seq(c);
      NetPrep p{};
      p.bh = c->rb;
      p.xh = c->rx;
      p.hs = hs + (size_t)it * batch * 8;
      p.perm = c->perm;
      p.geo = c->seq_geo;
      p.n = c->dk.n;
      p.na = c->dg.na;
      p.P = c->seq_P;
      p.F = F;
      p.tgt = tgt;
      p.scale = scale;
      launch_net_prep(p, batch, st);
      net_forward(net, sq, batch, F, true, st);
      launch_mse(net->H.back(), tgt, (size_t)batch * c->seq_P, net->dY, losses + it, st);
      net_backward(net, sq, batch, F, net->dY, st);
      adam(net, lr, st);
    }
    std::vector<float> hl(iters);
    HIPCHK(hipMemcpyAsync(hl.data(), losses, iters * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    if (loss_host) std::copy(hl.begin(), hl.end(), loss_host);
  } catch (const HipError& e) {
    failed->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

int iim_warm_start_loss(iim_ctx* c, iim_net* net, int32_t batch, double* loss, int64_t* samples) {
  if (!c || check_net(net) != IIM_OK || batch < 1 || !loss) return IIM_EINVAL;
  if (c->host_only) return IIM_EUNSUPPORTED;
  std::vector<int> valid;
  for (int m = 3; m < c->rec_count; ++m)
    if (c->rec_run[m - 3] == c->rec_run[m]) valid.push_back(m);
  if (valid.empty()) {
    c->err = "no recorded solve has three predecessors in the same run";
    return IIM_EINVAL;
  }
  try {
    hipStream_t st = c->stream;
    ensure_sequences(c);
    const int P = c->seq_P;
    const int nb = (int)((valid.size() + batch - 1) / batch);
    std::vector<void*> tmp;
    struct Free {
      std::vector<void*>& l;
      ~Free() {
        for (void* p : l) (void)hipFree(p);
      }
    } fr{tmp};
    float* F = net_alloc<float>(tmp, (size_t)batch * P * NET_FEATURES);
    float* tgt = net_alloc<float>(tmp, (size_t)batch * P);
    float* scale = net_alloc<float>(tmp, batch);
    float* losses = net_alloc<float>(tmp, nb);
    int* hs = net_alloc<int>(tmp, (size_t)nb * batch * 8);
    std::vector<int> h_hs((size_t)nb * batch * 8), count(nb);
    for (int bq = 0; bq < nb; ++bq) {
      count[bq] = (int)std::min<size_t>(batch, valid.size() - (size_t)bq * batch);
      for (int e = 0; e < count[bq]; ++e) {
        const int m = valid[(size_t)bq * batch + e];
        int* t = &h_hs[8 * ((size_t)bq * batch + e)];
        t[0] = m;
        t[1] = m - 1;
        t[2] = m - 2;
        t[3] = m - 1;
        t[4] = m - 2;
        t[5] = m - 3;
        t[6] = c->rec_stage[m];
        t[7] = m;
      }
    }
    HIPCHK(hipMemcpy(hs, h_hs.data(), h_hs.size() * sizeof(int), hipMemcpyHostToDevice));
    ensure_rows(net, (size_t)batch * P);
    const Seq sq = ctx_seq(c);
    for (int bq = 0; bq < nb; ++bq) {
      NetPrep p{};
      p.bh = c->rb;
      p.xh = c->rx;
      p.hs = hs + (size_t)bq * batch * 8;
      p.perm = c->perm;
      p.geo = c->seq_geo;
      p.n = c->dk.n;
      p.na = c->dg.na;
      p.P = P;
      p.F = F;
      p.tgt = tgt;
      p.scale = scale;
      launch_net_prep(p, count[bq], st);
      net_forward(net, sq, count[bq], F, false, st);
      launch_mse(net->H.back(), tgt, (size_t)count[bq] * P, net->dY, losses + bq, st);
    }
    std::vector<float> hl(nb);
    HIPCHK(hipMemcpyAsync(hl.data(), losses, nb * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    double acc = 0.0;
    for (int bq = 0; bq < nb; ++bq) acc += (double)hl[bq] * count[bq];
    *loss = acc / (double)valid.size();
    if (samples) *samples = (int64_t)valid.size();
  } catch (const HipError& e) {
    c->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

int iim_warm_start_sequences(iim_ctx* c, int32_t* P, int32_t* perm_host, int32_t* seq_host, float* geo_host) {
  if (!c || !P) return IIM_EINVAL;
  if (c->host_only) return IIM_EUNSUPPORTED;
  try {
    ensure_sequences(c);
    *P = c->seq_P;
    const size_t Pn = c->seq_P;
    if (perm_host) HIPCHK(hipMemcpy(perm_host, c->perm, Pn * sizeof(int), hipMemcpyDeviceToHost));
    if (seq_host) HIPCHK(hipMemcpy(seq_host, c->seq, 3 * Pn * sizeof(int), hipMemcpyDeviceToHost));
    if (geo_host) HIPCHK(hipMemcpy(geo_host, c->seq_geo, 4 * Pn * sizeof(float), hipMemcpyDeviceToHost));
  } catch (const HipError& e) {
    c->err = e.what();
    return e.code;
  }
  return IIM_OK;
}

}  // extern "C"
