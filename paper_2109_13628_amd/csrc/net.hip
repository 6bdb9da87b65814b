// Kernels of the initial-guess network (declared in net_dev.hpp).
//
// Every convolution is one GEMM on the matrix cores.  A workgroup of four
// 64-wide waves owns a 64 x 64 output tile; each wave computes 32 x 32 of it
// as 2 x 2 blocks of 16 x 16 MFMA results.  The operands are gathered from
// global memory through accessors (im2col over the circular sequences,
// transposed weights, ...).  BF16 operands: each 32-deep slice of the A and B
// tiles is gathered once per workgroup (coalesced, rounded to BF16), staged
// in LDS (double-buffered: the next slice's loads are in flight while the
// current one is multiplied) and read back as 16-byte fragments for the
// gfx950 16x16x32 BF16 MFMA.  FP32 operands: fragments gathered straight from
// global memory (the 16x16x4 FP32 MFMA).
//
// Matrix-core lane layouts (64 lanes, r = lane % 16, g = lane / 16):
//   16x16x32 bf16: lane holds A[r][8g + q] and B[8g + q][r], q = 0..7
//   16x16x4  f32 : lane holds A[r][g] and B[g][r]
//   result       : lane holds D[4g + q][r], q = 0..3
// (a GEMM only needs the A and B slots of a lane to hold the same k values;
// the result layout fixes where D lands)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "net_dev.hpp"

namespace iim {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ short to_bf16(float f) {
  // round to nearest even (finite inputs)
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

constexpr float GELU_C = 0.7978845608028654f;  // sqrt(2 / pi)
constexpr float GELU_A = 0.044715f;

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + tanhf(GELU_C * (z + GELU_A * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float t = tanhf(GELU_C * (z + GELU_A * z * z * z));
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * GELU_C * (1.0f + 3.0f * GELU_A * z * z);
}

__device__ __forceinline__ int seq_src(const Seq& s, int p, int off) {
  const int L = s.segl[p];
  int q = (s.pos[p] + off) % L;
  if (q < 0) q += L;
  return s.seg0[p] + q;
}

// ---- operand accessors: A(m, k), B(k, n).  For the A operand, row(m)
// gathers what depends on the row alone (the sequence lookups of the
// circular convolution) once, and at(row, m, k) forms an element from it.
struct RowIdx {
  int m;
};
struct AConv {               // im2col: A(row, tap*C + c) = X[row shifted by sgn*(tap-2) in its sequence][c]
  const float* X;
  int C;
  Seq s;
  int sgn;
  struct Row {               // the row's sequence: first row, length, position
    int first, len, pos;
  };
  __device__ float operator()(int m, int k) const {
    const int b = m / s.P, p = m - b * s.P;
    const int tap = k / C, c = k - tap * C;
    return X[((size_t)b * s.P + seq_src(s, p, sgn * (tap - 2))) * C + c];
  }
  __device__ Row row(int m) const {
    const int b = m / s.P, p = m - b * s.P;
    return Row{b * s.P + s.seg0[p], s.segl[p], s.pos[p]};
  }
  // arithmetic only (a table of the five source rows would be indexed by the
  // tap at run time, which the compiler places in private memory)
  __device__ float at(const Row& r, int, int k) const {
    const int tap = k / C, c = k - tap * C;
    int q = r.pos + sgn * (tap - 2);            // |shift| <= 2: two corrections reach [0, len)
    q += q < 0 ? r.len : 0;
    q += q < 0 ? r.len : 0;
    q -= q >= r.len ? r.len : 0;
    q -= q >= r.len ? r.len : 0;
    return X[(size_t)(r.first + q) * C + c];
  }
};
struct AConvT {              // A(tap*C + c, row) = X[row shifted by (tap-2)][c]  (weight gradient)
  const float* X;
  int C;
  Seq s;
  using Row = RowIdx;
  __device__ float operator()(int m, int k) const {
    const int tap = m / C, c = m - tap * C;
    const int b = k / s.P, p = k - b * s.P;
    return X[((size_t)b * s.P + seq_src(s, p, tap - 2)) * C + c];
  }
  __device__ Row row(int m) const { return Row{m}; }
  __device__ float at(const Row&, int m, int k) const { return (*this)(m, k); }
};
struct BRow {                // B(k, n) = P[k*ld + n]
  const float* P;
  int ld;
  __device__ float operator()(int k, int n) const { return P[(size_t)k * ld + n]; }
};
struct BWt {                 // B(tap*cout + co, ci) = W[(tap*cin + ci)*cout + co]
  const float* W;
  int cin, cout;
  __device__ float operator()(int k, int n) const {
    const int tap = k / cout, co = k - tap * cout;
    return W[((size_t)tap * cin + n) * cout + co];
  }
};

// ---- epilogues E(m, n, value, split)
struct EFwd {
  const float* bias;
  float* Z;
  float* H;
  int N, act;
  __device__ void operator()(int m, int n, float v, int) const {
    const float z = v + bias[n];
    const size_t i = (size_t)m * N + n;
    if (Z) Z[i] = z;
    H[i] = act ? gelu(z) : z;
  }
};
struct EBwd {
  const float* Zp;
  float* out;
  int N;
  __device__ void operator()(int m, int n, float v, int) const {
    const size_t i = (size_t)m * N + n;
    out[i] = Zp ? v * gelu_grad(Zp[i]) : v;
  }
};
struct EPart {
  float* part;
  size_t MN;
  int N;
  __device__ void operator()(int m, int n, float v, int z) const { part[z * MN + (size_t)m * N + n] = v; }
};

// Round eight FP32 values to BF16 (nearest even) and pack them.
__device__ __forceinline__ uint4 pack_bf16x8(const float (&f)[8]) {
  unsigned h[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) h[q] = (unsigned short)to_bf16(f[q]);
  return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

constexpr int MM_KT = 32;               // k depth of one staged slice (one 16x16x32 MFMA)
constexpr int MM_LD = MM_KT + 8;        // LDS row length in BF16 (16-byte pad against bank conflicts)

// C(M x N) = sum_k A(m, k) B(k, n) over k in [z*kper, min(K, (z+1)*kper)),
// z = blockIdx.z; BF16 operands staged in LDS, FP32 accumulation.
//
// Slice i is gathered into register set i mod MM_D at iteration i - MM_D,
// staged into LDS buffer i mod 2 at the end of iteration i - 1 and
// multiplied at iteration i: MM_D - 1 iterations of products hide each
// gather's latency (with one slice in flight the loop waited a full global
// round trip per slice, which dominated the small inference products).
constexpr int MM_D = 3;
template <class AF, class BF, class EF>
__global__ void __launch_bounds__(256) k_mm_bf16(int M, int N, int K, int kper, AF A, BF B, EF E) {
  // slices: A as [m][k], B transposed as [n][k], both k-contiguous
  __shared__ __align__(16) unsigned short As[2][64 * MM_LD];
  __shared__ __align__(16) unsigned short Bs[2][64 * MM_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int mw = (wave & 1) * 32, nw = (wave >> 1) * 32;
  const int kb = blockIdx.z * kper;
  const int ke = min(K, kb + kper);
  const int ns = ke > kb ? (ke - kb + MM_KT - 1) / MM_KT : 0;   // slices of this block
  // gather roles: A row am, k offset ak (8 consecutive k); B column bn, k offset bk
  const int am = tid >> 2, ak = (tid & 3) * 8;
  const int bn = tid & 63, bk = (tid >> 6) * 8;
  float fa[MM_D][8], fb[MM_D][8];
  const int ma = min(m0 + am, M - 1);
  const typename AF::Row arow = A.row(ma);   // the row's lookups, once
  if (ns == 0) {                             // nothing to multiply: zero result, no loads
#pragma unroll
    for (int d = 0; d < MM_D; ++d) {
#pragma unroll
      for (int q = 0; q < 8; ++q) fa[d][q] = fb[d][q] = 0.f;
    }
  }
  // Loads without branches: indices outside the operands are clamped to a
  // valid element (kb < ke whenever ns > 0) and the value replaced by zero.
  const int m = m0 + am, n = n0 + bn;
  const int nc = min(n, N - 1);
  // The validity of each loaded value is kept as a bit and applied when the
  // slice is staged: a select right after the load would wait for it.
  unsigned va[MM_D] = {}, vbm[MM_D] = {};
  auto gather = [&](int slot, int i) {
    const int k0 = kb + i * MM_KT;
    const bool live = i < ns;
    unsigned ba = 0, bb = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ka = k0 + ak + q, kbq = k0 + bk + q;
      fa[slot][q] = A.at(arow, ma, min(ka, ke - 1));
      fb[slot][q] = B(min(kbq, ke - 1), nc);
      ba |= (live && m < M && ka < ke) ? (1u << q) : 0u;
      bb |= (live && n < N && kbq < ke) ? (1u << q) : 0u;
    }
    va[slot] = ba;
    vbm[slot] = bb;
  };
  auto stage = [&](int slot, int buf) {
    float xa[8], xb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      xa[q] = (va[slot] >> q) & 1u ? fa[slot][q] : 0.f;
      xb[q] = (vbm[slot] >> q) & 1u ? fb[slot][q] : 0.f;
    }
    *reinterpret_cast<uint4*>(&As[buf][am * MM_LD + ak]) = pack_bf16x8(xa);
    *reinterpret_cast<uint4*>(&Bs[buf][bn * MM_LD + bk]) = pack_bf16x8(xb);
  };
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  if (ns > 0) {
#pragma unroll
    for (int d = 0; d < MM_D; ++d) gather(d, d);
  }
  stage(0, 0);
  __syncthreads();
  for (int i0 = 0; i0 < ns; i0 += MM_D) {
#pragma unroll
    for (int d = 0; d < MM_D; ++d) {
      const int i = i0 + d;             // slice i sits in register set d
      if (i < ns) {                     // uniform over the block
        const int buf = i & 1;
        bf8v a[2], b[2];
#pragma unroll
        for (int u = 0; u < 2; ++u)
          a[u] = *reinterpret_cast<const bf8v*>(&As[buf][(mw + 16 * u + r) * MM_LD + 8 * g]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
          b[u] = *reinterpret_cast<const bf8v*>(&Bs[buf][(nw + 16 * u + r) * MM_LD + 8 * g]);
        gather(d, i + MM_D);            // set d is free: slice i was staged an iteration ago (ns > 0 here)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v)
            acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b[v], acc[u][v], 0, 0, 0);
        if (i + 1 < ns) stage((d + 1) % MM_D, buf ^ 1);   // the other buffer: last read before the barrier
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + mw + 16 * i + 4 * g + q, n = n0 + nw + 16 * j + r;
        if (m < M && n < N) E(m, n, acc[i][j][q], (int)blockIdx.z);
      }
}

// The same product with FP32 operands gathered straight into the 16x16x4
// FP32 MFMA fragments.
template <class AF, class BF, class EF>
__global__ void __launch_bounds__(256) k_mm_f32(int M, int N, int K, int kper, AF A, BF B, EF E) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int mw = blockIdx.x * 64 + (wave & 1) * 32;
  const int nw = blockIdx.y * 64 + (wave >> 1) * 32;
  const int kb = blockIdx.z * kper;
  const int ke = min(K, kb + kper);
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 4) {
    const int k = k0 + g;
    float a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = mw + 16 * i + r;
      a[i] = (m < M && k < ke) ? A(m, k) : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = nw + 16 * j + r;
      b[j] = (n < N && k < ke) ? B(k, n) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = mw + 16 * i + 4 * g + q, n = nw + 16 * j + r;
        if (m < M && n < N) E(m, n, acc[i][j][q], (int)blockIdx.z);
      }
}

// Split-K chunks are multiples of MM_KT rows (the BF16 slice depth; a
// multiple of the FP32 kernel's 4).
int mm_kper(int K, int splits) {
  int kper = (K + splits - 1) / splits;
  kper = ((kper + MM_KT - 1) / MM_KT) * MM_KT;
  return kper == 0 ? MM_KT : kper;
}

template <class AF, class BF, class EF>
void mm(bool bf16, int M, int N, int K, int splits, AF A, BF B, EF E, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const int kper = mm_kper(K, splits);
  const int z = (K + kper - 1) / kper;
  dim3 grid((M + 63) / 64, (N + 63) / 64, z < 1 ? 1 : z);
  if (bf16)
    k_mm_bf16<<<grid, 256, 0, st>>>(M, N, K, kper, A, B, E);
  else
    k_mm_f32<<<grid, 256, 0, st>>>(M, N, K, kper, A, B, E);
}

__global__ void k_reduce_part(const float* __restrict__ part, int splits, size_t MN, float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[z * MN + i];
  out[i] = s;
}

__device__ float block_sumf(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float t = 0.f;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
  __syncthreads();
  return t;
}
__device__ double block_sumd(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
  __syncthreads();
  return t;
}

// gb[n] = sum over rows of dZ[row][n]   (one workgroup per column)
__global__ void __launch_bounds__(256) k_bias_grad(const float* __restrict__ dZ, int rows, int N, float* __restrict__ gb) {
  __shared__ float red[4];
  const int n = blockIdx.x;
  float s = 0.f;
  for (int m = threadIdx.x; m < rows; m += blockDim.x) s += dZ[(size_t)m * N + n];
  s = block_sumf(s, red);
  if (threadIdx.x == 0) gb[n] = s;
}

// Adam (Kingma & Ba) with bias correction at step t >= 1
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_fillf(float* p, float v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// time-extrapolation ratio of the solve at each RK stage: the stages sit at
// t + c dt with c = 0, 1/3, 3/4, and x_base extends the line through the two
// previous solves
__device__ double extrap_ratio(int stage) {
  return stage == 0 ? 0.6 : (stage == 1 ? 4.0 / 3.0 : 1.25);
}

__global__ void __launch_bounds__(1024) k_net_prep(NetPrep p) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const int* hs = p.hs + 8 * b;
  const double* b0 = p.bh + (size_t)hs[0] * p.n;
  const double* b1 = p.bh + (size_t)hs[1] * p.n;
  const double* b2 = p.bh + (size_t)hs[2] * p.n;
  const double* x1 = p.xh + (size_t)hs[3] * p.n;
  const double* x2 = p.xh + (size_t)hs[4] * p.n;
  const double* x3 = p.xh + (size_t)hs[5] * p.n;
  const int stage = hs[6];
  const double a = extrap_ratio(stage);
  double rr = 0.0, dd = 0.0, pp = 0.0;
  for (int i = threadIdx.x; i < p.n; i += blockDim.x) {
    const double r = b0[i] - (1.0 + a) * b1[i] + a * b2[i];
    const double pr = b0[i] - b1[i];
    pp += pr * pr;
    if (i < p.na) {
      const double d = x1[i] - x2[i];
      rr += r * r;
      dd += d * d;
    }
    if (p.xbase && b == 0) p.xbase[i] = x1[i] + a * (x1[i] - x2[i]);
  }
  rr = block_sumd(rr, red);
  dd = block_sumd(dd, red);
  pp = block_sumd(pp, red);
  const double na = p.na > 0 ? (double)p.na : 1.0;
  double sr = sqrt(rr / na), sd = sqrt(dd / na);
  if (!(sr > 0.0)) sr = 1.0;
  if (!(sd > 0.0)) sd = 1.0;
  const double isr = 1.0 / sr, isd = 1.0 / sd;
  if (threadIdx.x == 0) {
    p.scale[b] = (float)sr;
    if (p.prevres && b == 0) p.prevres[0] = sqrt(pp);
  }
  const double* x0 = p.xh + (size_t)hs[7] * p.n;   // solution of this solve (training only)
  for (int q = threadIdx.x; q < p.P; q += blockDim.x) {
    const int i = p.perm[q];
    float* f = p.F + ((size_t)b * p.P + q) * NET_FEATURES;
    f[0] = (float)((b0[i] - (1.0 + a) * b1[i] + a * b2[i]) * isr);
    f[1] = (float)((x1[i] - x2[i]) * isd);
    f[2] = (float)((x2[i] - x3[i]) * isd);
    f[3] = stage == 0 ? 1.f : 0.f;
    f[4] = stage == 1 ? 1.f : 0.f;
    f[5] = stage == 2 ? 1.f : 0.f;
    for (int c = 0; c < 4; ++c) f[6 + c] = p.geo[4 * q + c];
    if (p.tgt) p.tgt[(size_t)b * p.P + q] = (float)((x0[i] - x1[i] - a * (x1[i] - x2[i])) * isr);
  }
}

__global__ void k_net_apply(const int* __restrict__ perm, int P, const float* __restrict__ y,
                            const float* __restrict__ scale, double* __restrict__ x) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) x[perm[q]] += (double)scale[0] * (double)y[q];
}

// loss = mean((Y - T)^2), dY = 2 (Y - T) / n   (one workgroup)
__global__ void __launch_bounds__(1024) k_mse(const float* __restrict__ Y, const float* __restrict__ T, size_t n,
                                              float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ double red[16];
  const float sc = 2.0f / (float)n;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = sc * d;
    s += (double)d * d;
  }
  s = block_sumd(s, red);
  if (threadIdx.x == 0) loss[0] = (float)(s / (double)n);
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_mse(const float* Y, const float* T, size_t n, float* dY, float* loss, hipStream_t st) {
  k_mse<<<1, 1024, 0, st>>>(Y, T, n, dY, loss);
}

// Split count of a forward product: enough workgroups to occupy the device
// when the output has few 64 x 64 tiles (the k chain of one workgroup, not
// bandwidth, sets the time of a one-sample product), at least two 32-deep
// slices per split, and the workspace within CONV_FWD_PART_MAX floats.
int conv_fwd_splits(int rows, int cin, int cout) {
  const int tiles = ((rows + 63) / 64) * ((cout + 63) / 64);
  const int slices = (NET_TAPS * cin + MM_KT - 1) / MM_KT;
  int sp = (128 + tiles - 1) / tiles;
  sp = std::min(sp, slices / 2);
  while (sp > 1 && (size_t)sp * rows * cout > CONV_FWD_PART_MAX) --sp;
  if (sp < 1) sp = 1;
  // the count the GEMM really uses (its chunks are whole slices)
  const int K = NET_TAPS * cin;
  const int kper = mm_kper(K, sp);
  return (K + kper - 1) / kper;
}

// out = sum over splits of part (in split order) + bias; Z keeps it, H its GELU
__global__ void k_reduce_fwd(const float* __restrict__ part, int splits, size_t MN, int N,
                             const float* __restrict__ bias, float* __restrict__ Z, float* __restrict__ H, int act) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += part[z * MN + i];
  const float zv = v + bias[i % N];
  if (Z) Z[i] = zv;
  H[i] = act ? gelu(zv) : zv;
}

void launch_conv_fwd(bool bf16, const Seq& s, int B, const float* X, int cin, const float* W, const float* bias,
                     int cout, float* Z, float* H, int act, float* part, hipStream_t st) {
  const int rows = B * s.P;
  const int sp = bf16 && part ? conv_fwd_splits(rows, cin, cout) : 1;
  if (sp <= 1) {
    mm(bf16, rows, cout, NET_TAPS * cin, 1, AConv{X, cin, s, 1}, BRow{W, cout}, EFwd{bias, Z, H, cout, act}, st);
    return;
  }
  const size_t MN = (size_t)rows * cout;
  mm(bf16, rows, cout, NET_TAPS * cin, sp, AConv{X, cin, s, 1}, BRow{W, cout}, EPart{part, MN, cout}, st);
  k_reduce_fwd<<<(unsigned)((MN + 255) / 256), 256, 0, st>>>(part, sp, MN, cout, bias, Z, H, act);
}

void launch_conv_bwd_data(bool bf16, const Seq& s, int B, const float* dZ, int cout, const float* W, int cin,
                          const float* Zprev, float* dXout, hipStream_t st) {
  mm(bf16, B * s.P, cin, NET_TAPS * cout, 1, AConv{dZ, cout, s, -1}, BWt{W, cin, cout}, EBwd{Zprev, dXout, cin},
     st);
}

int conv_bwd_w_splits(int rows) {
  int sp = (rows + 1023) / 1024;
  return sp < 1 ? 1 : (sp > 64 ? 64 : sp);
}

void launch_conv_bwd_w(bool bf16, const Seq& s, int B, const float* H, int cin, const float* dZ, int cout,
                       float* part, int splits, float* gW, float* gb, hipStream_t st) {
  const int rows = B * s.P;
  const int M = NET_TAPS * cin;
  const size_t MN = (size_t)M * cout;
  // the split count the GEMM really uses
  const int kper = mm_kper(rows, splits);
  const int z = (rows + kper - 1) / kper;
  mm(bf16, M, cout, rows, splits, AConvT{H, cin, s}, BRow{dZ, cout}, EPart{part, MN, cout}, st);
  k_reduce_part<<<(unsigned)((MN + 255) / 256), 256, 0, st>>>(part, z, MN, gW);
  k_bias_grad<<<cout, 256, 0, st>>>(dZ, rows, cout, gb);
}


void launch_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                 int t, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  if (n) k_adam<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void launch_fillf(float* p, float v, size_t n, hipStream_t st) {
  if (n) k_fillf<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, v, n);
}

void launch_net_prep(const NetPrep& p, int B, hipStream_t st) {
  if (B > 0) k_net_prep<<<B, 1024, 0, st>>>(p);
}

void launch_net_apply(const int* perm, int P, const float* y, const float* scale, double* x, hipStream_t st) {
  if (P > 0) k_net_apply<<<(P + 255) / 256, 256, 0, st>>>(perm, P, y, scale, x);
}


}  // namespace iim
