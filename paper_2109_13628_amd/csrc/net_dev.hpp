// Device side of the initial-guess network: circular 1D convolutions over the
// affected points of each body, ordered around it (kernel 5, GELU between
// layers), as GEMMs on the matrix cores (BF16 operands, FP32 accumulation),
// with an FP32-operand variant of the same kernels for gradient checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace iim {

constexpr int NET_TAPS = 5;

// Ragged batch of circular sequences: position p (0 <= p < P) belongs to the
// sequence starting at seg0[p] with length segl[p] and sits at index pos[p]
// inside it.  A batch of B samples holds B * P rows (sample-major).
struct Seq {
  const int* seg0;
  const int* segl;
  const int* pos;
  int P;
};

// forward: Z = conv(X) + bias; H = gelu(Z) (act = 1) or H = Z (act = 0).
// Small products (few output tiles, e.g. one sample at inference) split the
// k range over conv_fwd_splits(...) workgroups whose partial sums go to
// `part` (conv_fwd_splits * rows * cout floats) and are added in a fixed
// order by a second kernel; part may be null when the count is 1.
int conv_fwd_splits(int rows, int cin, int cout);
constexpr size_t CONV_FWD_PART_MAX = (size_t)1 << 20;   // floats: the largest split workspace used
void launch_conv_fwd(bool bf16, const Seq& s, int B, const float* X, int cin, const float* W, const float* bias,
                     int cout, float* Z, float* H, int act, float* part, hipStream_t st);
// backward data: dX = conv^T(dZ); written as dX * gelu'(Zprev) when Zprev != null
void launch_conv_bwd_data(bool bf16, const Seq& s, int B, const float* dZ, int cout, const float* W, int cin,
                          const float* Zprev, float* dXout, hipStream_t st);
// backward weights and bias: gW[(tap*cin + ci)*cout + co], gb[co]; part is a
// workspace of splits * 5*cin*cout floats
void launch_conv_bwd_w(bool bf16, const Seq& s, int B, const float* H, int cin, const float* dZ, int cout,
                       float* part, int splits, float* gW, float* gb, hipStream_t st);
int conv_bwd_w_splits(int rows);

// loss[0] = mean((Y - T)^2), dY = 2 (Y - T) / n
void launch_mse(const float* Y, const float* T, size_t n, float* dY, float* loss, hipStream_t st);

void launch_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                 int t, hipStream_t st);
void launch_fillf(float* p, float v, size_t n, hipStream_t st);

// Initial-guess features.  For every sample, hs[8*b .. 8*b+7] = slots of
// (b_0, b_1, b_2, x_1, x_2, x_3) in the history arrays bh, xh ([slots][n]),
// the RK stage of the solve, and the slot of its solution x_0 (training).
// With a = the stage's time-extrapolation ratio, r = b_0 - (1+a) b_1 + a b_2
// is the residual of x_base = x_1 + a (x_1 - x_2); features per position p
// (affected index perm[p]): r / s_r, (x_1 - x_2) / s_d, (x_2 - x_3) / s_d,
// stage one-hot (3), geo[p][4].  s_r, s_d are the RMS of r and x_1 - x_2
// over the corrections.  Outputs: scale[b] = s_r; optional tgt[b][p] =
// (x_0 - x_base) / s_r at perm[p] (training target), xbase (sample 0) and
// prevres = |b_0 - b_1| (sample 0).
struct NetPrep {
  const double* bh;
  const double* xh;
  const int* hs;
  const int* perm;
  const float* geo;
  int n, na, P;
  float* F;                    // [B][P][10]
  float* tgt;                  // nullable, [B][P]
  float* scale;                // [B]
  double* xbase;               // nullable
  double* prevres;             // nullable
};
constexpr int NET_FEATURES = 10;
void launch_net_prep(const NetPrep& p, int B, hipStream_t st);
// x[perm[p]] += scale[0] * y[p]
void launch_net_apply(const int* perm, int P, const float* y, const float* scale, double* x, hipStream_t st);

}  // namespace iim
