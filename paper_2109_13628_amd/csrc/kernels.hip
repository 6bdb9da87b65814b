// HIP kernels of the IIM library (gfx950, wave64).
//
// Poisson operator (Sec. 4.2): zero-padded lattice-Green's-function
// convolution on an mx x my torus in three passes over HBM,
//   rows  : real-to-complex FFT of each dense source row (half-length
//           complex FFT + split), spectrum written column-major spec[kx][j];
//   cols  : per column kx: the dense rows' transforms plus the direct row
//           transforms of the IIM correction sources (a few points per row),
//           FFT, multiply by the (real) kernel spectrum, inverse FFT, reading
//           only the source rows and writing only the requested output rows
//           (pruned in the Krylov loop) into a second buffer, so that the row
//           transforms of omega survive the solve's products;
//   irows : complex-to-real inverse FFT of the requested rows, writing the
//           grid plus the one-node ring.
// FFTs are LDS Stockham radix-4 (one radix-2 stage when log2 N is odd) with
// per-thread register butterflies and a twiddle table in global memory.
//
// Box exterior: dense orthonormal sine transforms (DST-II) as four small
// GEMMs.
//
// IIM sparse kernels (Sec. 2.1-2.2): ghost values, correction rows, boundary
// vorticity (Sec. 5.3) and the vorticity extensions read host-built tables.
// Transport (Sec. 3): a bulk kernel for fluid nodes whose stencils are all
// fluid, and a boundary kernel for the rest; both fuse the RK3 update.
// GMRES (Sec. 4.2): Arnoldi with classical Gram-Schmidt applied twice, Givens
// rotations, all in one workgroup per step, state in device memory.
#include <hip/hip_runtime.h>
#include <string>

#include <type_traits>

#include "iim_dev.hpp"

namespace iim {

#define IIM_LAUNCH_CHECK() (void)0

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// complex type -> its real type; complex from two reals
template <class CX>
struct Real;
template <>
struct Real<double2> { using t = double; };
template <>
struct Real<float2> { using t = float; };
template <class CX, class A, class B>
__device__ __forceinline__ CX mkc(A x, B y) {
  CX r;
  r.x = (typename Real<CX>::t)x;
  r.y = (typename Real<CX>::t)y;
  return r;
}

// Row transform, at frequency kx, of the correction sources of row n: the
// sum over the row's entries of sgn * gam[a] * W^(kx i), W = exp(-2 pi i / mx),
// plus the mirrored source at column 2 nx - 1 - i for the outflow exterior.
// This is what the real row transform of length mx gives for a row that holds
// only these point values; the column pass adds it directly, so the sparse
// sources need no row pass.  tw_xr holds W^k for k <= mx / 2 (mx even).
// W^r for 0 <= r < mx from the table of W^k, k <= mx / 2 (one load, always in range)
// v mod m for v >= 0: a mask when m is a power of two (every LDS-kernel torus),
// a division otherwise (tori with a factor 3 or 5)
__device__ __forceinline__ int torus_mod(int v, int m) { return (m & (m - 1)) == 0 ? (v & (m - 1)) : v % m; }
template <class CX>
__device__ __forceinline__ CX twiddle_r(const CX* __restrict__ tw_xr, int r, int mx) {
  const bool hi = r > mx / 2;
  const CX w = tw_xr[hi ? mx - r : r];
  return hi ? conj2(w) : w;
}

template <class CX>
__device__ __forceinline__ CX sparse_row_dft(const DGeom& g, int mx, bool outflow, const CX* __restrict__ tw_xr,
                                             const double* __restrict__ gam, double sgn, int n, int kx) {
  using S = typename Real<CX>::t;
  CX acc = mkc<CX>(0, 0);
  const int e1 = g.row_ptr[n + 1];
  for (int e0 = g.row_ptr[n]; e0 < e1; e0 += 4) {
    int ii[4];
    double val[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = e0 + u < e1;
      ii[u] = ok ? g.row_i[e0 + u] : 0;
      val[u] = ok ? sgn * gam[g.row_a[e0 + u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const CX w = twiddle_r(tw_xr, torus_mod(kx * ii[u], mx), mx);
      const S v = (S)val[u];
      acc.x += v * w.x;
      acc.y += v * w.y;
      if (outflow) {
        const CX w2 = twiddle_r(tw_xr, torus_mod(kx * (2 * g.nx - 1 - ii[u]), mx), mx);
        acc.x += v * w2.x;
        acc.y += v * w2.y;
      }
    }
  }
  return acc;
}

// ------------------------------------------------------------------ FFT core
template <int N>
struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <>
struct Log2<1> { static constexpr int v = 0; };

// One Stockham stage of radix R on N points by TPF threads.  In place: all
// loads to registers, barrier, all stores, barrier.
template <int N, int TPF, int R, bool INV>
__device__ __forceinline__ void fft_stage(double2* buf, int lt, int Ns, const double2* __restrict__ tw) {
  constexpr int NBF = N / R;                   // butterflies
  constexpr int NB = (NBF + TPF - 1) / TPF;    // per thread
  double2 v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lt + b * TPF;
    if (NBF % TPF == 0 || j < NBF) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * NBF];
      const int k = j & (Ns - 1);
      if (Ns > 1) {
        const int step = N / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = tw[r * k * step];
          if (INV) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      if constexpr (R == 2) {
        const double2 a = v[b][0], c = v[b][1];
        v[b][0] = cadd(a, c);
        v[b][1] = csub(a, c);
      } else {
        const double2 a0 = cadd(v[b][0], v[b][2]);
        const double2 a1 = csub(v[b][0], v[b][2]);
        const double2 a2 = cadd(v[b][1], v[b][3]);
        const double2 d = csub(v[b][1], v[b][3]);
        // forward: -i * d ; inverse: +i * d
        const double2 a3 = INV ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
        v[b][0] = cadd(a0, a2);
        v[b][2] = csub(a0, a2);
        v[b][1] = cadd(a1, a3);
        v[b][3] = csub(a1, a3);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lt + b * TPF;
    if (NBF % TPF == 0 || j < NBF) {
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

// In-place FFT of N complex points in LDS; tw[k] = exp(-2 pi i k / N).
// Forward: X_k = sum x_n e^{-2 pi i k n / N}; inverse: unnormalised, +i.
template <int N, int TPF, bool INV>
__device__ __forceinline__ void fft_lds(double2* buf, int lt, const double2* __restrict__ tw) {
  int Ns = 1;
  if (Log2<N>::v % 2 == 1) {
    fft_stage<N, TPF, 2, INV>(buf, lt, Ns, tw);
    Ns = 2;
  }
#pragma unroll 1
  for (; Ns < N; Ns *= 4) fft_stage<N, TPF, 4, INV>(buf, lt, Ns, tw);
}

template <int N>
struct FftCfg {
  static constexpr int TPF = (N / 4 >= 64) ? 64 : (N / 4 >= 1 ? N / 4 : 1);
  // FFTs per block: keep LDS <= 64 KB and the block <= 256 threads
  static constexpr int PER_LDS = (65536 / (N * 16)) > 0 ? (65536 / (N * 16)) : 1;
  static constexpr int PER_THR = 256 / TPF;
  static constexpr int PER = PER_LDS < PER_THR ? (PER_LDS < 4 ? PER_LDS : 4) : (PER_THR < 4 ? PER_THR : 4);
  static constexpr int THREADS = PER * TPF;
};

// ------------------------------------------------------------------ row pass
// Forward real FFT of length mx = 2*HX of the source rows j in [j0, j0 + count).
template <int HX>
__global__ void __launch_bounds__(FftCfg<HX>::THREADS)
k_rows_fwd(DGeom g, DFft f, const double* __restrict__ omega, int j0, int count, const double* __restrict__ done) {
  using C = FftCfg<HX>;
  if (done && done[KS_DONE] != 0.0) return;
  __shared__ double2 lds[C::PER][HX];
  const int tid = threadIdx.x;
  const int r = tid / C::TPF, lt = tid % C::TPF;
  const int jrow = j0 + blockIdx.x * C::PER + r;
  const bool valid = (jrow < j0 + count) && jrow >= 0 && jrow < g.ny;
  double2* z = lds[r];
  // load z_n = (x_{2n}, x_{2n+1})
  for (int n = lt; n < HX; n += C::TPF) {
    double2 v = make_double2(0.0, 0.0);
    if (valid && omega) {
      const int i0 = 2 * n, i1 = 2 * n + 1;
      if (!f.outflow) {
        if (i0 < g.nx && g.cls[jrow * g.nx + i0] < 2) v.x = omega[jrow * g.nx + i0];
        if (i1 < g.nx && g.cls[jrow * g.nx + i1] < 2) v.y = omega[jrow * g.nx + i1];
      } else {
        const int m0 = i0 < g.nx ? i0 : 2 * g.nx - 1 - i0;
        const int m1 = i1 < g.nx ? i1 : 2 * g.nx - 1 - i1;
        if (m0 >= 0 && m0 < g.nx && g.cls[jrow * g.nx + m0] < 2) v.x = omega[jrow * g.nx + m0];
        if (m1 >= 0 && m1 < g.nx && g.cls[jrow * g.nx + m1] < 2) v.y = omega[jrow * g.nx + m1];
      }
    }
    z[n] = v;
  }
  __syncthreads();
  fft_lds<HX, C::TPF, false>(z, lt, f.tw_x);
  // split: X_k = E_k + W^k O_k, k in [0, HX]; write spec[k][jrow + 1]
  const int nth = C::THREADS;
  for (int t = tid; t < (HX + 1) * C::PER; t += nth) {
    const int rr = t % C::PER, k = t / C::PER;
    const int jj = j0 + blockIdx.x * C::PER + rr;
    if (jj >= j0 + count || jj < 0 || jj >= g.ny) continue;
    const double2 zk = lds[rr][k & (HX - 1)];
    const double2 zc = conj2(lds[rr][(HX - k) & (HX - 1)]);
    const double2 E = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
    const double2 Od = csub(zk, zc);   // 2 i O
    const double2 O = make_double2(0.5 * Od.y, -0.5 * Od.x);
    const double2 X = cadd(E, cmul(f.tw_xr[k], O));
    f.spec[(size_t)k * f.ld + jj + 1] = X;
  }
}

// ---------------------------------------------------------------- column pass
template <int MY>
__global__ void __launch_bounds__(FftCfg<MY>::THREADS)
k_cols(DGeom g, DFft f, bool dense, const double* __restrict__ gam, double sgn, int rj0, int rj1, int oj0, int oj1,
       const double* __restrict__ done) {
  using C = FftCfg<MY>;
  if (done && done[KS_DONE] != 0.0) return;
  __shared__ double2 lds[C::PER][MY];
  const int tid = threadIdx.x;
  const int r = tid / C::TPF, lt = tid % C::TPF;
  const int kx = blockIdx.x * C::PER + r;
  const bool valid = kx <= f.hx;
  double2* z = lds[r];
  const double2* col = f.spec + (size_t)(valid ? kx : 0) * f.ld;
  double2* out = f.spec_out + (size_t)(valid ? kx : 0) * f.ld;
  for (int n = lt; n < MY; n += C::TPF) z[n] = make_double2(0.0, 0.0);
  __syncthreads();
  if (valid && dense)
    for (int j = rj0 + lt; j <= rj1; j += C::TPF) z[j & (MY - 1)] = col[j + 1];
  // the same thread owns row j in both loops
  if (valid && gam)
    for (int j = rj0 + lt; j <= rj1 && j < g.ny; j += C::TPF)
      z[j & (MY - 1)] = cadd(z[j & (MY - 1)], sparse_row_dft<double2>(g, f.mx, f.outflow, f.tw_xr, gam, sgn, j, kx));
  __syncthreads();
  fft_lds<MY, C::TPF, false>(z, lt, f.tw_y);
  if (valid) {
    const double* gh = f.ghat + (size_t)kx * (MY / 2 + 1);
    for (int n = lt; n < MY; n += C::TPF) {
      const double s = gh[n <= MY / 2 ? n : MY - n];
      z[n].x *= s;
      z[n].y *= s;
    }
  }
  __syncthreads();
  fft_lds<MY, C::TPF, true>(z, lt, f.tw_y);
  if (valid)
    for (int j = oj0 + lt; j <= oj1; j += C::TPF) out[j + 1] = z[j & (MY - 1)];
}

// ------------------------------------------------------------ inverse rows
// Output rows jo in [j0, j0 + count) (jo may be -1 .. ny), written to the ring array.
template <int HX>
__global__ void __launch_bounds__(FftCfg<HX>::THREADS)
k_rows_inv(DGeom g, DFft f, int j0, int count, double* __restrict__ psi, const double* __restrict__ done) {
  using C = FftCfg<HX>;
  if (done && done[KS_DONE] != 0.0) return;
  __shared__ double2 lds[C::PER][HX + 1];
  const int tid = threadIdx.x;
  const int nth = C::THREADS;
  // gather X_k, k in [0, HX]
  for (int t = tid; t < (HX + 1) * C::PER; t += nth) {
    const int rr = t % C::PER, k = t / C::PER;
    const int jo = j0 + blockIdx.x * C::PER + rr;
    double2 v = make_double2(0.0, 0.0);
    if (jo < j0 + count) v = f.spec_out[(size_t)k * f.ld + jo + 1];
    lds[rr][k] = v;
  }
  __syncthreads();
  // Z_k = (X_k + conj X_{HX-k}) + i (X_k - conj X_{HX-k}) / W^k, k < HX (in registers, then store)
  const int r = tid / C::TPF, lt = tid % C::TPF;
  double2* z = lds[r];
  constexpr int NPT = (HX + C::TPF - 1) / C::TPF;
  double2 tmp[NPT];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int k = lt + q * C::TPF;
    if (k < HX) {
      const double2 xk = z[k];
      const double2 xc = conj2(z[HX - k]);
      const double2 E = cadd(xk, xc);
      const double2 D = csub(xk, xc);
      const double2 O = cmul(D, conj2(f.tw_xr[k]));   // divide by W^k = multiply by conj
      tmp[q] = make_double2(E.x - O.y, E.y + O.x);      // E + i O
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int k = lt + q * C::TPF;
    if (k < HX) z[k] = tmp[q];
  }
  __syncthreads();
  fft_lds<HX, C::TPF, true>(z, lt, f.tw_x);
  const int nxr = g.nx + 2;
  for (int t = tid; t < (g.nx + 2) * C::PER; t += nth) {
    const int rr = t / (g.nx + 2), ii = t % (g.nx + 2) - 1;   // ii in [-1, nx]
    const int jo = j0 + blockIdx.x * C::PER + rr;
    if (jo >= j0 + count) continue;
    // ring columns -1 and nx: torus positions mx - 1 and nx (nx wraps to 0
    // on the unpadded periodic torus)
    const int i = ii < 0 ? 2 * HX - 1 : (ii >= 2 * HX ? ii - 2 * HX : ii);
    const double2 zz = lds[rr][i >> 1];
    psi[(size_t)(jo + 1) * nxr + (ii + 1)] = (i & 1) ? zz.y : zz.x;
  }
}

template <int HX>
static void rows_fwd_launch(const DGeom& g, const DFft& f, const double* omega, int j0, int count,
                            const double* done, hipStream_t s) {
  using C = FftCfg<HX>;
  const int blocks = (count + C::PER - 1) / C::PER;
  if (blocks > 0) k_rows_fwd<HX><<<blocks, C::THREADS, 0, s>>>(g, f, omega, j0, count, done);
}
template <int MY>
static void cols_launch(const DGeom& g, const DFft& f, bool dense, const double* gam, double sgn, int rj0, int rj1,
                        int oj0, int oj1, const double* done, hipStream_t s) {
  using C = FftCfg<MY>;
  const int blocks = (f.hx + 1 + C::PER - 1) / C::PER;
  k_cols<MY><<<blocks, C::THREADS, 0, s>>>(g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done);
}
template <int HX>
static void rows_inv_launch(const DGeom& g, const DFft& f, int j0, int count, double* psi, const double* done,
                            hipStream_t s) {
  using C = FftCfg<HX>;
  const int blocks = (count + C::PER - 1) / C::PER;
  if (blocks > 0) k_rows_inv<HX><<<blocks, C::THREADS, 0, s>>>(g, f, j0, count, psi, done);
}

#define IIM_POW2_SWITCH(VAL, FN, ...)                     \
  switch (VAL) {                                          \
    case 16: FN<16>(__VA_ARGS__); break;                  \
    case 32: FN<32>(__VA_ARGS__); break;                  \
    case 64: FN<64>(__VA_ARGS__); break;                  \
    case 128: FN<128>(__VA_ARGS__); break;                \
    case 256: FN<256>(__VA_ARGS__); break;                \
    case 512: FN<512>(__VA_ARGS__); break;                \
    case 1024: FN<1024>(__VA_ARGS__); break;              \
    case 2048: FN<2048>(__VA_ARGS__); break;              \
    case 4096: FN<4096>(__VA_ARGS__); break;              \
    default: break;                                       \
  }

void launch_conv_reg(const DGeom& g, const DFft& f, const double* omega, const double* gam, double sgn, int rj0,
                     int rj1, int oj0, int oj1, double* psi_ring, const double* done, hipStream_t s, Prof* prof,
                     bool fp32, bool rows_ready);

void launch_conv(const DGeom& g, const DFft& f, const double* omega, const double* gam, double sgn, int rj0,
                 int rj1, int oj0, int oj1, double* psi_ring, const double* done, hipStream_t s, Prof* prof,
                 bool fp32, bool rows_ready) {
  if (f.use_reg && conv_reg_supported(f.hx, f.my)) {
    launch_conv_reg(g, f, omega, gam, sgn, rj0, rj1, oj0, oj1, psi_ring, done, s, prof, fp32 && f.spec32,
                    rows_ready);
    return;
  }
  const int nin = rj1 - rj0 + 1, nout = oj1 - oj0 + 1;
  const bool dense = omega != nullptr;
  int h = prof ? prof->begin(KID_ROWS_FWD, s) : -1;
  if (dense && !rows_ready) IIM_POW2_SWITCH(f.hx, rows_fwd_launch, g, f, omega, rj0, nin, done, s);
  // algorithmic bytes: source rows read (omega) + half spectrum written
  if (prof) prof->end(h, (dense && !rows_ready) ? (double)nin * (8.0 * g.nx + 16.0 * (f.hx + 1)) : 0.0, s);
  h = prof ? prof->begin(KID_COLS, s) : -1;
  IIM_POW2_SWITCH(f.my, cols_launch, g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done, s);
  if (prof) prof->end(h, (double)(f.hx + 1) * ((dense ? 16.0 * nin : 0.0) + 8.0 * (f.my / 2 + 1) + 16.0 * nout), s);
  h = prof ? prof->begin(KID_ROWS_INV, s) : -1;
  IIM_POW2_SWITCH(f.hx, rows_inv_launch, g, f, oj0, nout, psi_ring, done, s);
  if (prof) prof->end(h, (double)nout * (16.0 * (f.hx + 1) + 8.0 * (g.nx + 2)), s);
}

// ------------------------------------------------------------------ box DST
// C[M][N] (ldc, possibly scaled elementwise by S[M][N]) = A[M][K] * B[K][N]
template <int TS>
__global__ void __launch_bounds__(TS * TS / 4)
k_gemm(int M, int N, int K, const double* __restrict__ A, int lda, bool transA, const double* __restrict__ B,
       int ldb, double* __restrict__ Cm, int ldc, const double* __restrict__ S, const double* __restrict__ done) {
  if (done && done[KS_DONE] != 0.0) return;
  __shared__ double As[TS][TS + 1];
  __shared__ double Bs[TS][TS + 1];
  const int tx = threadIdx.x % TS, ty4 = threadIdx.x / TS;   // each thread: 4 rows
  const int row0 = blockIdx.y * TS, col0 = blockIdx.x * TS;
  double acc[4] = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += TS) {
    for (int q = threadIdx.x; q < TS * TS; q += blockDim.x) {
      const int rr = q / TS, cc = q % TS;
      const int ar = row0 + rr, ak = k0 + cc;
      double av = 0.0;
      if (ar < M && ak < K) av = transA ? A[(size_t)ak * lda + ar] : A[(size_t)ar * lda + ak];
      As[rr][cc] = av;
      const int bk = k0 + rr, bc = col0 + cc;
      Bs[rr][cc] = (bk < K && bc < N) ? B[(size_t)bk * ldb + bc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < TS; ++kk) {
      const double b = Bs[kk][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += As[ty4 * 4 + q][kk] * b;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rr = row0 + ty4 * 4 + q, cc = col0 + tx;
    if (rr < M && cc < N) Cm[(size_t)rr * ldc + cc] = S ? acc[q] * S[(size_t)rr * N + cc] : acc[q];
  }
}

__global__ void k_build_source(DGeom g, const double* __restrict__ omega, const double* __restrict__ gam,
                               double sgn, const int* __restrict__ a_id, double* __restrict__ src,
                               const double* __restrict__ done) {
  if (done && done[KS_DONE] != 0.0) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.nx * g.ny) return;
  double v = (omega && g.cls[q] < 2) ? omega[q] : 0.0;
  if (gam) {
    const int a = a_id[q];
    if (a >= 0) v += sgn * gam[a];
  }
  src[q] = v;
}

__global__ void k_ring_reflect(DGeom g, double* __restrict__ psi, const double* __restrict__ done) {
  if (done && done[KS_DONE] != 0.0) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nxr = g.nx + 2;
  if (t < g.nx) {
    psi[t + 1] = -psi[nxr + t + 1];
    psi[(size_t)(g.ny + 1) * nxr + t + 1] = -psi[(size_t)g.ny * nxr + t + 1];
  }
  if (t < g.ny) {
    psi[(size_t)(t + 1) * nxr] = -psi[(size_t)(t + 1) * nxr + 1];
    psi[(size_t)(t + 1) * nxr + g.nx + 1] = -psi[(size_t)(t + 1) * nxr + g.nx];
  }
  if (t == 0) {
    psi[0] = psi[nxr + 1];
    psi[g.nx + 1] = psi[nxr + g.nx];
    psi[(size_t)(g.ny + 1) * nxr] = psi[(size_t)g.ny * nxr + 1];
    psi[(size_t)(g.ny + 1) * nxr + g.nx + 1] = psi[(size_t)g.ny * nxr + g.nx];
  }
}

// The same product for small boxes: one output per thread (64 columns x 4
// rows per block), the k loop over operands that stay in L2, eight products
// in flight.  A 128 x 128 box gives 64 blocks instead of the tiled kernel's
// 16, and no barrier per k tile: its latency, not its bytes, set the time.
__global__ void __launch_bounds__(256)
k_gemm_small(int M, int N, int K, const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
             double* __restrict__ Cm, int ldc, const double* __restrict__ S, const double* __restrict__ done) {
  if (done && done[KS_DONE] != 0.0) return;
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (r >= M || c >= N) return;
  const double* a = A + (size_t)r * lda;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int k = 0;
  for (; k + 8 <= K; k += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += a[k + u] * B[(size_t)(k + u) * ldb + c];
  }
  for (; k < K; ++k) acc[0] += a[k] * B[(size_t)k * ldb + c];
  const double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  Cm[(size_t)r * ldc + c] = S ? v * S[(size_t)r * N + c] : v;
}

static void gemm(int M, int N, int K, const double* A, int lda, bool tA, const double* B, int ldb, double* Cm,
                 int ldc, const double* S, const double* done, hipStream_t s) {
  if (!tA && (size_t)M * N <= (size_t)512 * 512 && K <= 1024) {
    dim3 grid((N + 63) / 64, (M + 3) / 4);
    k_gemm_small<<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, Cm, ldc, S, done);
    return;
  }
  constexpr int TS = 32;
  dim3 grid((N + TS - 1) / TS, (M + TS - 1) / TS);
  k_gemm<TS><<<grid, TS * TS / 4, 0, s>>>(M, N, K, A, lda, tA, B, ldb, Cm, ldc, S, done);
}

// psi_ring = G src (box): src assembled from omega / gamma, then
// T1 = src phx^T, T2 = (phy T1) .* lam^-1, T1 = T2 phx, psi = phy^T T1.
void launch_dst(const DGeom& g, const DDst& d, const double* omega, const double* gam, double sgn,
                double* psi_ring, const double* done, hipStream_t s) {
  const int nx = g.nx, ny = g.ny, nxr = nx + 2;
  const int n = nx * ny;
  k_build_source<<<(n + 255) / 256, 256, 0, s>>>(g, omega, gam, sgn, g.a_id, d.src, done);
  gemm(ny, nx, nx, d.src, nx, false, d.phxT, nx, d.t1, nx, nullptr, done, s);
  gemm(ny, nx, ny, d.phy, ny, false, d.t1, nx, d.t2, nx, d.lam_inv, done, s);
  gemm(ny, nx, nx, d.t2, nx, false, d.phx, nx, d.t1, nx, nullptr, done, s);
  gemm(ny, nx, ny, d.phyT, ny, false, d.t1, nx, psi_ring + nxr + 1, nxr, nullptr, done, s);
  const int m = nx > ny ? nx : ny;
  k_ring_reflect<<<(m + 255) / 256, 256, 0, s>>>(g, psi_ring, done);
}

}  // namespace iim

namespace iim {

// ============================================================ small helpers
__global__ void k_fill(double* p, double v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void launch_fill(double* p, double v, size_t n, hipStream_t s) {
  if (n) k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}
__global__ void k_fill_int(int* p, int v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void launch_fill_int(int* p, int v, size_t n, hipStream_t s) {
  if (n) k_fill_int<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

// Block-wide sum (blockDim.x a multiple of 64, <= 1024); result valid in all threads.
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double t = 0.0;
  for (int q = 0; q < nw; ++q) t += red[q];
  __syncthreads();
  return t;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ============================================================ Schur system
// y_gamma = v_gamma + A psi - sum_k psibar_k B 1_k ;  y_k = sum_{B_k} v_gamma
// (computed by one workgroup so the circulation rows need no atomics)
__device__ void matvec_finish_block(const DGeom& g, const double* __restrict__ psi, const double* __restrict__ v,
                                    double* __restrict__ out, double* red) {
  double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = threadIdx.x; a < g.na; a += blockDim.x) {
    // the row's indices and weights in flight together, then its psi values
    double acc = 0.0;
    const int e1 = g.aop.ptr[a + 1];
    for (int e0 = g.aop.ptr[a]; e0 < e1; e0 += 8) {
      int ri[8];
      double wv[8], pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = e0 + u < e1;
        ri[u] = ok ? g.aop.ridx[e0 + u] : -1;
        wv[u] = ok ? g.aop.w[e0 + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = ri[u] >= 0 ? psi[ri[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += wv[u] * pv[u];
    }
    double y = v[a] + acc;
    for (int k = 0; k < g.nbc; ++k) y -= g.b1[(size_t)k * g.na + a] * v[g.na + k];
    out[a] = y;
    const int c = g.a_col[a];
    if (c >= 0 && c < 8) part[c] += v[a];
  }
  for (int k = 0; k < g.nbc && k < 8; ++k) {
    const double s = block_sum(part[k], red);
    if (threadIdx.x == 0) out[g.na + k] = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(1024) k_matvec_finish(DGeom g, const double* psi, const double* v, double* out) {
  __shared__ double red[16];
  matvec_finish_block(g, psi, v, out, red);
}
void launch_matvec_finish(const DGeom& g, const DKrylov&, const double* psi_ring, const double* v, double* out,
                          hipStream_t s) {
  k_matvec_finish<<<1, 1024, 0, s>>>(g, psi_ring, v, out);
}

// b_gamma = A (G omega) + B psi_b_tilde ; b_k = sum_{R_k} omega - Gamma_k / h^2
__global__ void __launch_bounds__(1024) k_rhs_vector(DGeom g, const double* __restrict__ psi,
                                                    const double* __restrict__ omega,
                                                    const double* __restrict__ Gamma, double* __restrict__ b) {
  __shared__ double red[16];
  if ((int)blockIdx.x < g.nbc) {
    const int k = blockIdx.x;
    const int i0 = g.rects[4 * k], i1 = g.rects[4 * k + 1], j0 = g.rects[4 * k + 2], j1 = g.rects[4 * k + 3];
    const int w = i1 - i0 + 1, cnt = w * (j1 - j0 + 1);
    double acc = 0.0;
    // four independent loads in flight per thread and iteration
    for (int q0 = threadIdx.x; q0 < cnt; q0 += 4 * blockDim.x) {
      double v[4];
      int8_t cl[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * blockDim.x;
        cl[u] = 3;
        v[u] = 0.0;
        if (q < cnt) {
          const int idx = (j0 + q / w) * g.nx + i0 + q % w;
          cl[u] = g.cls[idx];
          v[u] = omega[idx];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (cl[u] < 2) acc += v[u];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) b[g.na + k] = s - Gamma[k] * g.inv_h * g.inv_h;
    return;
  }
  const int a = (blockIdx.x - g.nbc) * blockDim.x + threadIdx.x;
  if (a >= g.na) return;
  double acc = 0.0;
#pragma unroll 4
  for (int e = g.aop.ptr[a]; e < g.aop.ptr[a + 1]; ++e) acc += g.aop.w[e] * psi[g.aop.ridx[e]];
  b[a] = acc + g.bpsi[a];
}
void launch_rhs_vector(const DGeom& g, const double* psi_ring, const double* omega, const double* Gamma, double* b,
                       hipStream_t s) {
  const int blocks = g.nbc + (g.na + 1023) / 1024;
  if (blocks > 0) k_rhs_vector<<<blocks, 1024, 0, s>>>(g, psi_ring, omega, Gamma, b);
}

// ============================================================ GMRES (device)
// start: r = b - w (or b when x = 0), V0 = r / |r|, g = (|r|, 0, ...)
__global__ void __launch_bounds__(1024) k_krylov_start(DKrylov k, int x_is_zero) {
  __shared__ double red[16];
  const int n = k.n;
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double bi = k.b[i];
    const double ri = x_is_zero ? bi : bi - k.w[i];
    if (x_is_zero) k.x[i] = 0.0;
    k.V[i] = ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  const double beta = sqrt(block_sum(rr, red));
  const double bnorm = sqrt(block_sum(bb, red));
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) k.V[i] *= inv;
  if (threadIdx.x == 0) {
    k.g[0] = beta;
    k.st[KS_BETA] = beta;
    k.st[KS_BNORM] = bnorm;
    const double rel = bnorm > 0.0 ? beta / bnorm : 0.0;
    k.st[KS_RES] = rel;
    if (k.st[KS_RES0] < 0.0) k.st[KS_RES0] = rel;
    k.st[KS_K] = 0.0;
    if (!(beta == beta) || !(bnorm == bnorm)) k.st[KS_NFAIL] = 1.0;
    k.st[KS_DONE] = (beta <= k.st[KS_TOL] * bnorm || !(beta == beta)) ? 1.0 : 0.0;
  }
}
void launch_krylov_start(const DGeom&, const DKrylov& k, bool x_is_zero, hipStream_t s) {
  k_krylov_start<<<1, 1024, 0, s>>>(k, x_is_zero ? 1 : 0);
}

// One Arnoldi step: w = S V_j (psi = G E_a V_j,gamma already in the ring buffer),
// CGS2 against V_0..V_j, new Givens rotation, residual estimate.
__global__ void __launch_bounds__(1024) k_arnoldi(DGeom g, DKrylov k, const double* __restrict__ psi, int j) {
  __shared__ double red[16];
  __shared__ double hcol[72];
  __shared__ double hacc[72];
  __shared__ double lcs[72], lsn[72];
  if (k.st[KS_DONE] != 0.0) return;
  const int n = k.n, m = k.m;
  // previous Givens rotations to LDS now, read by one thread at the end
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    lcs[i] = k.cs[i];
    lsn[i] = k.sn[i];
  }
  const double* vj = k.V + (size_t)j * n;
  double* w = k.V + (size_t)(j + 1) * n;
  matvec_finish_block(g, psi, vj, w, red);   // ends with a barrier; w visible block-wide
  for (int i = threadIdx.x; i <= j; i += blockDim.x) hacc[i] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // One workgroup does the whole step, so its loads must overlap: the loops
  // below issue groups of independent loads before using any of them.
  constexpr int G = 8;
  for (int pass = 0; pass < 2; ++pass) {
    // dots: wave wid handles basis vectors i = wid, wid + nw, ...
    for (int i = wid; i <= j; i += nw) {
      const double* vi = k.V + (size_t)i * n;
      double acc = 0.0;
      for (int e0 = lane; e0 < n; e0 += 64 * G) {
        double a[G], b[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int e = e0 + 64 * u;
          a[u] = e < n ? vi[e] : 0.0;
          b[u] = e < n ? w[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < G; ++u) acc += a[u] * b[u];
      }
      acc = wave_sum(acc);
      if (lane == 0) hcol[i] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      double we = w[e];
      for (int i0 = 0; i0 <= j; i0 += G) {
        double vv[G];
#pragma unroll
        for (int u = 0; u < G; ++u) vv[u] = i0 + u <= j ? k.V[(size_t)(i0 + u) * n + e] : 0.0;
#pragma unroll
        for (int u = 0; u < G; ++u)
          if (i0 + u <= j) we -= hcol[i0 + u] * vv[u];
      }
      w[e] = we;
    }
    for (int i = threadIdx.x; i <= j; i += blockDim.x) hacc[i] += hcol[i];
    __syncthreads();
  }
  double nn = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) nn += w[e] * w[e];
  const double hn = sqrt(block_sum(nn, red));
  const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) w[e] *= inv;
  // the new column of H, rotated in LDS by one thread, then written out
  if (threadIdx.x == 0) {
    hacc[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t = lcs[i] * hacc[i] + lsn[i] * hacc[i + 1];
      hacc[i + 1] = -lsn[i] * hacc[i] + lcs[i] * hacc[i + 1];
      hacc[i] = t;
    }
    const double den = hypot(hacc[j], hacc[j + 1]);
    const double c = den > 0.0 ? hacc[j] / den : 1.0, s = den > 0.0 ? hacc[j + 1] / den : 0.0;
    k.cs[j] = c;
    k.sn[j] = s;
    hacc[j] = den;
    hacc[j + 1] = 0.0;
    k.g[j + 1] = -s * k.g[j];
    k.g[j] = c * k.g[j];
    k.st[KS_K] = (double)(j + 1);
    k.st[KS_ITERS] += 1.0;
    const double bnorm = k.st[KS_BNORM];
    const double rel = bnorm > 0.0 ? fabs(k.g[j + 1]) / bnorm : 0.0;
    k.st[KS_RES] = rel;
    if (!(rel == rel)) k.st[KS_NFAIL] = 1.0;
    if (rel <= k.st[KS_TOL] || !(rel == rel) || hn == 0.0) k.st[KS_DONE] = 1.0;
  }
  __syncthreads();
  double* H = k.H + (size_t)j * (m + 1);
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) H[i] = hacc[i];
}
void launch_arnoldi(const DGeom& g, const DKrylov& k, const double* psi_ring, int j, hipStream_t s, Prof* prof) {
  IIM_LAUNCH(prof, KID_ARNOLDI, 8.0 * k.n * (2.0 * (j + 1) + 3.0), k_arnoldi, 1, 1024, s, g, k, psi_ring, j);
}

// x += V y with H(0:kk, 0:kk) y = g(0:kk)
__global__ void __launch_bounds__(1024) k_gmres_update(DKrylov k) {
  __shared__ double y[72];
  __shared__ double Hs[64][65];   // Hs[i][q] = H(i, q), restart length <= 64
  const int kk = (int)k.st[KS_K];
  const int n = k.n, m = k.m;
  if (kk <= 0) return;
  for (int t = threadIdx.x; t < kk * kk; t += blockDim.x) {
    const int i = t % kk, q = t / kk;
    Hs[i][q] = k.H[(size_t)q * (m + 1) + i];
  }
  __syncthreads();
  // back substitution by one wave: lane l keeps g_l minus the terms of the
  // unknowns solved so far; lane i's value is final when y_i is formed
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    double s = l < kk ? k.g[l] : 0.0;
    for (int i = kk - 1; i >= 0; --i) {
      const double yi = __shfl(s, i, 64) / Hs[i][i];
      if (l < i) s -= Hs[l][i] * yi;
      if (l == i) y[i] = yi;
    }
  }
  __syncthreads();
  constexpr int G = 8;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    double xe = k.x[e];
    for (int i0 = 0; i0 < kk; i0 += G) {
      double vv[G];
#pragma unroll
      for (int u = 0; u < G; ++u) vv[u] = i0 + u < kk ? k.V[(size_t)(i0 + u) * n + e] : 0.0;
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (i0 + u < kk) xe += y[i0 + u] * vv[u];
    }
    k.x[e] = xe;
  }
  __syncthreads();
  if (threadIdx.x == 0) k.st[KS_K] = 0.0;
}
void launch_gmres_update(const DKrylov& k, hipStream_t s) { k_gmres_update<<<1, 1024, 0, s>>>(k); }

// ============================================================ recovery
// psi ghosts (fourth order with psi_b_tilde + psibar_k)
__global__ void k_ghost_psi(DGeom g, const double* __restrict__ x, double* __restrict__ psi) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ng) return;
  double acc = 0.0;
#pragma unroll 4
  for (int e = g.ext4b.ptr[q]; e < g.ext4b.ptr[q + 1]; ++e) acc += g.ext4b.w[e] * psi[g.ext4b.ridx[e]];
  for (int e = g.ext4b.bptr[q]; e < g.ext4b.bptr[q + 1]; ++e) {
    const int c = g.ext4b.bc[e];
    const int col = g.c_col[c];
    const double bcv = g.c_psibt[c] + (col >= 0 ? x[g.na + col] : 0.0);
    acc += g.ext4b.bw[e] * bcv;
  }
  psi[g.g_ridx[q]] = acc;
}

// velocity at fluid nodes and the normal components on the ring
__global__ void k_velocity(DGeom g, const double* __restrict__ psi, double* __restrict__ U, double* __restrict__ V) {
  const int nxr = g.nx + 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxr * (g.ny + 2)) return;
  const int ir = t % nxr, jr = t / nxr;   // ring coordinates
  const int i = ir - 1, j = jr - 1;
  const double c = 0.5 * g.inv_h;
  double u = 0.0, v = 0.0;
  if (i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
    const int8_t cl = g.cls[j * g.nx + i];
    if (cl == 2) return;  // ghosts: set by the velocity extension
    if (cl < 2) {
      u = g.uinf_x + c * (psi[t + nxr] - psi[t - nxr]);
      v = g.uinf_y - c * (psi[t + 1] - psi[t - 1]);
    }
  } else {
    const bool side = (i == -1 || i == g.nx) && j >= 0 && j < g.ny;
    const bool topbot = (j == -1 || j == g.ny) && i >= 0 && i < g.nx;
    if (side) u = g.uinf_x + c * (psi[t + nxr] - psi[t - nxr]);
    if (topbot) v = g.uinf_y - c * (psi[t + 1] - psi[t - 1]);
  }
  U[t] = u;
  V[t] = v;
}

// velocity extension to A- (third order with u_b)
__global__ void k_vel_ext(DGeom g, double* __restrict__ U, double* __restrict__ V) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ng) return;
  double au = 0.0, av = 0.0;
#pragma unroll 4
  for (int e = g.ext3b.ptr[q]; e < g.ext3b.ptr[q + 1]; ++e) {
    const int r = g.ext3b.ridx[e];
    au += g.ext3b.w[e] * U[r];
    av += g.ext3b.w[e] * V[r];
  }
  for (int e = g.ext3b.bptr[q]; e < g.ext3b.bptr[q + 1]; ++e) {
    const int c = g.ext3b.bc[e];
    au += g.ext3b.bw[e] * g.c_ub[2 * c];
    av += g.ext3b.bw[e] * g.c_ub[2 * c + 1];
  }
  U[g.g_ridx[q]] = au;
  V[g.g_ridx[q]] = av;
}

void launch_recover_fields(const DGeom& g, const double* x, double* psi, double* U, double* V, hipStream_t s) {
  if (g.ng) k_ghost_psi<<<(g.ng + 127) / 128, 128, 0, s>>>(g, x, psi);
  launch_velocity(g, psi, U, V, s);
  if (g.ng) k_vel_ext<<<(g.ng + 127) / 128, 128, 0, s>>>(g, U, V);
}

void launch_velocity(const DGeom& g, const double* psi, double* U, double* V, hipStream_t s) {
  const int nr = (g.nx + 2) * (g.ny + 2);
  k_velocity<<<(nr + 255) / 256, 256, 0, s>>>(g, psi, U, V);
}

// Eight lanes per composed row (DBnd): lane l sums entries l, l + 8, ...;
// the partial sums are combined by shuffles, lane 0 writes the result.  No
// row reads psi at a ghost node, so the ghost values written here never race
// with the reads.
__global__ void __launch_bounds__(256) k_boundary_forms(DGeom g, DBnd b, const double* __restrict__ omega,
                                                        const double* __restrict__ x, double* psi, double* U,
                                                        double* V, double* wb, double* w4, double* w3b,
                                                        double* w3n) {
  constexpr int L = 8;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = tid / L, l = tid % L;
  constexpr int M = (1 << 28) - 1;
  // the row's constant and destination, requested with its entries (the
  // launch has at least one row)
  const int rr = min(r, b.rows - 1);
  const double kc = b.kc[rr];
  const int d = b.dst[rr];
  double acc = 0.0;
  if (b.stride > 0) {
    // rows padded to a fixed stride: the entries are requested at once,
    // without the round trip for the row's bounds (lanes past the last row
    // read that row's entries and write nothing)
    for (int e0 = rr * b.stride + l; e0 < (rr + 1) * b.stride; e0 += 4 * L) {
      int id[4];
      double wv[4], val[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        id[u] = b.idx[e0 + u * L];
        wv[u] = b.w[e0 + u * L];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kind = id[u] >> 28, i = id[u] & M;
        const double* src = kind == 0 ? psi : (kind == 1 ? omega : x + g.na);
        val[u] = src[i];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += wv[u] * val[u];
    }
  } else if (r < b.rows) {
    // straight-line loads: entries at clamped indices (those past the row's
    // end repeat its last entry with weight zero), the source array chosen
    // by a pointer select rather than a branch per array (a branch around a
    // load waits for it inside the branch, one round trip per entry)
    const int e1 = b.ptr[r + 1];
    for (int e0 = b.ptr[r] + l; e0 < e1; e0 += 4 * L) {
      int id[4];
      double wv[4], val[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * L, e1 - 1);
        id[u] = b.idx[e];
        wv[u] = b.w[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kind = id[u] >> 28, i = id[u] & M;
        const double* src = kind == 0 ? psi : (kind == 1 ? omega : x + g.na);
        val[u] = src[i];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += (e0 + u * L < e1 ? wv[u] : 0.0) * val[u];
    }
  }
  for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (r >= b.rows || l != 0) return;
  acc += kc;
  const int kind = d >> 28, i = d & M;
  double* out = kind == 0 ? psi : kind == 1 ? U : kind == 2 ? V : kind == 3 ? wb : kind == 4 ? w4 : kind == 5 ? w3b : w3n;
  out[i] = acc;
}

void launch_boundary_forms(const DGeom& g, const DBnd& b, const double* omega, const double* x, double* psi,
                           double* U, double* V, double* wb, double* w4, double* w3b, double* w3n, hipStream_t s) {
  if (b.rows > 0)
    k_boundary_forms<<<(8 * b.rows + 255) / 256, 256, 0, s>>>(g, b, omega, x, psi, U, V, wb, w4, w3b, w3n);
}

// ============================================================ boundary vorticity
__global__ void k_omega_b(DGeom g, const double* __restrict__ U, const double* __restrict__ V, double* __restrict__ wb) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nc) return;
  double acc = g.wb_const[c];
#pragma unroll 4
  for (int e = g.wbc.ptr[c]; e < g.wbc.ptr[c + 1]; ++e) {
    const int r = g.wbc.ridx[e];
    const double val = (r & (1 << 30)) ? V[r & ((1 << 30) - 1)] : U[r];
    acc += g.wbc.w[e] * val;
  }
  wb[c] = acc;
}

__global__ void k_omega_ext(DGeom g, const double* __restrict__ omega, const double* __restrict__ wb,
                            double* __restrict__ w4, double* __restrict__ w3b, double* __restrict__ w3n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ng) return;
  double a4 = 0.0, a3 = 0.0, an = 0.0;
#pragma unroll 4
  for (int e = g.ext4b.ptr[q]; e < g.ext4b.ptr[q + 1]; ++e) a4 += g.ext4b.w[e] * omega[g.ext4b.gidx[e]];
  for (int e = g.ext4b.bptr[q]; e < g.ext4b.bptr[q + 1]; ++e) a4 += g.ext4b.bw[e] * wb[g.ext4b.bc[e]];
#pragma unroll 4
  for (int e = g.ext3b.ptr[q]; e < g.ext3b.ptr[q + 1]; ++e) a3 += g.ext3b.w[e] * omega[g.ext3b.gidx[e]];
  for (int e = g.ext3b.bptr[q]; e < g.ext3b.bptr[q + 1]; ++e) a3 += g.ext3b.bw[e] * wb[g.ext3b.bc[e]];
#pragma unroll 4
  for (int e = g.ext3n.ptr[q]; e < g.ext3n.ptr[q + 1]; ++e) an += g.ext3n.w[e] * omega[g.ext3n.gidx[e]];
  const int gi = g.g_gidx[q];
  w4[gi] = a4;
  w3b[gi] = a3;
  w3n[gi] = an;
}

void launch_omega_bc(const DGeom& g, const double* omega, const double* U, const double* V, double* wb, double* w4,
                     double* w3b, double* w3n, hipStream_t s) {
  if (g.nc) k_omega_b<<<(g.nc + 127) / 128, 128, 0, s>>>(g, U, V, wb);
  if (g.ng) k_omega_ext<<<(g.ng + 127) / 128, 128, 0, s>>>(g, omega, wb, w4, w3b, w3n);
}

// ============================================================ transport
// Face flux core: advective bracket of f values on the chosen stencil plus the
// diffusive flux.  use_left: stencil (-1, 0, 1) with (-1/6, 5/6, 1/3); else
// (0, 1, 2) with (1/3, 5/6, -1/6).
__device__ __forceinline__ double flux_core(bool use_left, double fm1, double f0, double f1, double f2,
                                            double wl, double wr, double nu_inv_h) {
  const double c6 = 1.0 / 6.0, c56 = 5.0 / 6.0, c3 = 1.0 / 3.0;
  const double F = use_left ? (-c6 * fm1 + c56 * f0 + c3 * f1) : (c3 * f0 + c56 * f1 - c6 * f2);
  return F - nu_inv_h * (wr - wl);
}

// Standard face (all four nodes fluid): upwind side by the face velocity sign.
__device__ __forceinline__ double flux_std(double um1, double u0, double u1, double u2, double wm1, double w0,
                                           double w1, double w2, double nu_inv_h) {
  const double uf = 0.5 * (u0 + u1);
  return flux_core(uf >= 0.0, um1 * wm1, u0 * w0, u1 * w1, u2 * w2, w0, w1, nu_inv_h);
}

enum { NK_FLUID = 0, NK_GHOST = 1, NK_SOLID = 2, NK_OUT = 3 };

// The grid data the transport kernel reads: a small argument, so that the
// geometry's many other table pointers do not occupy scalar registers of
// this large kernel (they spilled to scratch memory).
struct TGeom {
  int nx, ny, nsp, nbc, outflow, periodic;
  int vec;                     // bulk pairs may use 16-byte loads (nx even, arrays aligned, psi given)
  int quad;                    // bulk tiles of two rows, a 2 x 2 block of nodes per lane (needs vec)
  double h, inv_h, nu, uinf_x, uinf_y;
  const int8_t* __restrict__ cls;
  const int* __restrict__ special;
  const int* __restrict__ rects;
  int* nonfinite;              // flag raised by the RK update on a NaN / Inf result
};

// Raise the non-finite flag (every writer stores the same value).
__device__ __forceinline__ void mark_nonfinite(const TGeom& g, double v) {
  if (!isfinite(v)) *g.nonfinite = 1;
}

// Node velocities of the transport.  FROM_PSI = false: read from U / V on the
// ring (zero beyond it).  FROM_PSI = true: formed from the stream function as
// the velocity kernel forms them (central differences at fluid nodes, the
// component normal to the grid edge on the ring, zero at solid nodes and for
// the other ring component); ghost nodes still read the extension values in
// U / V.  Both give the same numbers for the same psi.
template <bool FROM_PSI>
struct Vel {
  const double* __restrict__ psi;
  const double* __restrict__ U;
  const double* __restrict__ V;
  // central differences of psi: u from the nodes above (pp) and below (pm),
  // v from the nodes right (pp) and left (pm)
  __device__ static __forceinline__ double u_of(const TGeom& g, double pp, double pm) {
    return g.uinf_x + 0.5 * g.inv_h * (pp - pm);
  }
  __device__ static __forceinline__ double v_of(const TGeom& g, double pp, double pm) {
    return g.uinf_y - 0.5 * g.inv_h * (pp - pm);
  }
  // ring index t of a fluid node (or of a ring node with that component)
  __device__ __forceinline__ double u_at(const TGeom& g, int t) const {
    if constexpr (FROM_PSI) {
      const int nxr = g.nx + 2;
      return u_of(g, psi[t + nxr], psi[t - nxr]);
    } else {
      return U[t];
    }
  }
  __device__ __forceinline__ double v_at(const TGeom& g, int t) const {
    if constexpr (FROM_PSI)
      return v_of(g, psi[t + 1], psi[t - 1]);
    else
      return V[t];
  }
  // component `axis` (0: u, 1: v) at ring index t of a node whose stencil
  // value is that component's central difference (or the stored value); the
  // axis may differ between lanes
  __device__ __forceinline__ double comp_at(const TGeom& g, int axis, int t) const {
    if constexpr (FROM_PSI) {
      const int o = axis == 0 ? g.nx + 2 : 1;
      const double d = psi[t + o] - psi[t - o];
      return axis == 0 ? g.uinf_x + 0.5 * g.inv_h * d : g.uinf_y - 0.5 * g.inv_h * d;
    } else {
      const double ue = U[t], ve = V[t];
      return axis == 0 ? ue : ve;
    }
  }
  // any node (ii, jj); axis 0: u, 1: v.  Straight-line code: every address is
  // clamped into its array and the value selected afterwards, so that the
  // loads of all the nodes of a stencil are in flight together (branches
  // around them put one memory round trip per branch on the critical path).
  // No pointer is selected by the axis either, which keeps the pointers out
  // of private (scratch) memory.
  __device__ __forceinline__ double node(const TGeom& g, int axis, int ii, int jj) const {
    const int nx = g.nx, ny = g.ny, nxr = nx + 2;
    const int t = (min(max(jj, -1), ny) + 1) * nxr + min(max(ii, -1), nx) + 1;
    const double ue = U[t], ve = V[t];
    const double e = axis == 0 ? ue : ve;
    if constexpr (FROM_PSI) {
      const bool in = ii >= 0 && jj >= 0 && ii < nx && jj < ny;
      const bool side = (ii == -1 || ii == nx) && jj >= 0 && jj < ny;
      const bool topbot = (jj == -1 || jj == ny) && ii >= 0 && ii < nx;
      const int o = axis == 0 ? nxr : 1;
      const double d = psi[min(t + o, nxr * (ny + 2) - 1)] - psi[max(t - o, 0)];
      const double val = axis == 0 ? g.uinf_x + 0.5 * g.inv_h * d : g.uinf_y - 0.5 * g.inv_h * d;
      // in the grid: the class picks the extension (ghost), zero (solid) or val
      const int8_t cl = g.cls[min(max(jj, 0), ny - 1) * nx + min(max(ii, 0), nx - 1)];
      const double v_in = cl == 2 ? e : (cl > 2 ? 0.0 : val);
      // on the ring only the component normal to the grid edge; zero beyond
      return in ? v_in : ((axis == 0 ? side : topbot) ? val : 0.0);
    } else {
      const bool ring = ii >= -1 && jj >= -1 && ii <= nx && jj <= ny;
      return ring ? e : 0.0;
    }
  }
};

// General face between node (i, j) and (i, j) + e_axis (axis 0: x, 1: y).
template <bool P>
__device__ double flux_general(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                               const double* __restrict__ w4, const double* __restrict__ w3b,
                               const double* __restrict__ w3n, int i, int j, int axis) {
  const int di = axis == 0 ? 1 : 0, dj = axis == 0 ? 0 : 1;
  const int nx = g.nx, ny = g.ny;
  int kind[4];
  double u[4], w[4], w4v[4], wb[4], wn[4];
  // straight-line: every load at a clamped address, values selected afterwards
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int ii = i + (t - 1) * di, jj = j + (t - 1) * dj;
    if (g.periodic) {   // the node a periodic edge repeats
      ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
      jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
    }
    const bool in = ii >= 0 && jj >= 0 && ii < nx && jj < ny;
    // past the outflow face, nodes nx, nx + 1 repeat the vorticity of nx - 1,
    // nx - 2, and node nx + 1 the x-velocity of nx - 2
    const bool mirrored = g.outflow && ii >= nx && ii <= nx + 1 && jj >= 0 && jj < ny;
    const int iw = mirrored ? 2 * nx - 1 - ii : ii;
    const int iu = (mirrored && axis == 0 && ii == nx + 1) ? nx - 2 : ii;
    const int qc = min(max(jj, 0), ny - 1) * nx + min(max(iw, 0), nx - 1);
    const int c = g.cls[qc];
    const double oq = omega[qc];
    const double e4 = w4 ? w4[qc] : 0.0, eb = w3b ? w3b[qc] : 0.0, en = w3n ? w3n[qc] : 0.0;
    u[t] = vel.node(g, axis, iu, jj);
    kind[t] = in ? (c < 2 ? NK_FLUID : (c == 2 ? NK_GHOST : NK_SOLID)) : NK_OUT;
    const bool fl = in && c < 2, gh = in && c == 2;
    const double base = (fl || mirrored) ? oq : 0.0;   // zero outside the grid and at solid nodes
    w[t] = base;
    w4v[t] = gh ? e4 : base;
    wb[t] = gh ? eb : base;
    wn[t] = gh ? en : base;
  }
  const bool fl0 = kind[1] == NK_FLUID || kind[1] == NK_OUT;
  const bool fl1 = kind[2] == NK_FLUID || kind[2] == NK_OUT;
  const double uf = 0.5 * (u[1] + u[2]);
  const bool up_left = uf >= 0.0;
  const bool use_left = (fl0 && fl1) ? up_left : fl0;
  double f[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    double om;
    if (kind[t] == NK_GHOST) {
      const bool on_left = t <= 1;
      om = (on_left == up_left) ? wb[t] : wn[t];
    } else {
      om = w[t];
    }
    f[t] = u[t] * om;
  }
  return flux_core(use_left, f[0], f[1], f[2], f[3], w4v[1], w4v[2], g.nu * g.inv_h);
}

// Face between node (i, j) and (i, j) + e_axis whose four stencil nodes are
// all regular fluid nodes inside the grid (the faces of a bounding region
// R_k): the values come straight from omega and psi (or U / V), no class loads.
template <bool P>
__device__ __forceinline__ double flux_interior(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                                int i, int j, int axis) {
  const int nxr = g.nx + 2;
  const int dq = axis == 0 ? 1 : g.nx, dr = axis == 0 ? 1 : nxr;
  const int q = j * g.nx + i, r = (j + 1) * nxr + i + 1;
  double u[4], w[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    w[t] = omega[q + (t - 1) * dq];
    u[t] = vel.comp_at(g, axis, r + (t - 1) * dr);
  }
  return flux_std(u[0], u[1], u[2], u[3], w[0], w[1], w[2], w[3], g.nu * g.inv_h);
}

// Bulk nodes (cls 0): every stencil node inside the grid is fluid (bodies keep
// three cells from the grid edge, so this also holds for stencils that wrap
// across a periodic edge).  Bulk part: one thread per 2 x 2 block of nodes,
// two grid rows of 512 nodes per workgroup.
//
// One node, any position.  Every lane takes the same straight-line path: the ten stencil positions are
// mapped onto the grid first (periodic edges wrap, the outflow plane mirrors
// omega and u_x), positions that carry no value (omega outside the grid, a
// velocity outside the ring) are read at a clamped address and masked to zero,
// and the node's class, the stencil values and the RK register are all in
// flight together.  A lane near the grid edge thus costs one memory round
// trip like any other, instead of a chain of dependent loads that set the
// duration of the whole launch.
template <bool P>
__device__ __forceinline__ void bulk_cell(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                          double* __restrict__ out, double* __restrict__ Q, double a, double b,
                                          double dt, int mode, int i, int j) {
  if (i >= g.nx) return;
  const int nx = g.nx, ny = g.ny, nxr = nx + 2;
  const int q = j * nx + i;
  const bool per = g.periodic != 0, mir = g.outflow != 0;
  const int8_t c = g.cls[q];
  const double qp = (mode == 1 && a != 0.0) ? Q[q] : 0.0;   // the first stage (a = 0) overwrites the register
  const double wc = omega[q];
  double wx[5], ux[5], wy[5], vy[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    // row j, column i + d - 2
    int iw = i + d - 2, iu = iw;
    if (per) {
      iw = iw < 0 ? iw + nx : (iw >= nx ? iw - nx : iw);
      iu = iw;
    } else if (mir && iw >= nx) {   // nodes nx, nx + 1 repeat nx - 1, nx - 2
      iu = iw == nx + 1 ? nx - 2 : iw;
      iw = 2 * nx - 1 - iw;
    }
    const bool wok = iw >= 0 && iw < nx, uok = iu >= -1 && iu <= nx;
    const double wv = omega[j * nx + min(max(iw, 0), nx - 1)];
    const double uv = vel.u_at(g, (j + 1) * nxr + min(max(iu, -1), nx) + 1);
    wx[d] = d == 2 ? wc : (wok ? wv : 0.0);
    ux[d] = uok ? uv : 0.0;
    // column i, row j + d - 2
    int jw = j + d - 2;
    if (per) jw = jw < 0 ? jw + ny : (jw >= ny ? jw - ny : jw);
    const bool wyok = jw >= 0 && jw < ny, vok = jw >= -1 && jw <= ny;
    const double wyv = omega[min(max(jw, 0), ny - 1) * nx + i];
    const double vv = vel.v_at(g, (min(max(jw, -1), ny) + 1) * nxr + i + 1);
    wy[d] = d == 2 ? wc : (wyok ? wyv : 0.0);
    vy[d] = vok ? vv : 0.0;
  }
  const double nih = g.nu * g.inv_h;
  const double fxr = flux_std(ux[1], ux[2], ux[3], ux[4], wx[1], wx[2], wx[3], wx[4], nih);
  const double fxl = flux_std(ux[0], ux[1], ux[2], ux[3], wx[0], wx[1], wx[2], wx[3], nih);
  const double fyt = flux_std(vy[1], vy[2], vy[3], vy[4], wy[1], wy[2], wy[3], wy[4], nih);
  const double fyb = flux_std(vy[0], vy[1], vy[2], vy[3], wy[0], wy[1], wy[2], wy[3], nih);
  double rhs = -((fxr - fxl) + (fyt - fyb)) * g.inv_h;
  // pins the arithmetic (and so every load) above the class test: the
  // compiler would otherwise sink the stencil loads below the wait for c
  asm volatile("" : "+v"(rhs));
  if (c == 1) return;   // boundary-kernel node: the lanes of the special part write it
  if (c >= 2) {         // solid: vorticity stays zero
    out[q] = 0.0;
    if (mode == 1) Q[q] = 0.0;
    return;
  }
  if (mode == 0) {
    out[q] = rhs;
  } else {
    const double qn = a * qp + dt * rhs;
    Q[q] = qn;
    const double wn = wc + b * qn;
    out[q] = wn;
    mark_nonfinite(g, wn);
  }
}

// The RK update (or the right-hand side) of one bulk-part node from its
// class: boundary-kernel nodes are left to the lanes of the special part,
// solid nodes keep zero vorticity.
__device__ __forceinline__ void bulk_store(const TGeom& g, double* __restrict__ out, double* __restrict__ Q, int8_t c,
                                           int q, double rhs, double wc, double qp, double a, double b, double dt,
                                           int mode) {
  if (c == 1) return;
  if (c >= 2) {
    out[q] = 0.0;
    if (mode == 1) Q[q] = 0.0;
    return;
  }
  if (mode == 0) {
    out[q] = rhs;
  } else {
    const double qn = a * qp + dt * rhs;
    Q[q] = qn;
    const double wn = wc + b * qn;
    out[q] = wn;
    mark_nonfinite(g, wn);
  }
}

// Nodes q, q + 1 of one row (q even): one 16-byte store per array when both
// are bulk fluid nodes, else bulk_store for each.
__device__ __forceinline__ void bulk_store2(const TGeom& g, double* __restrict__ out, double* __restrict__ Q,
                                            unsigned short cc, int q, double ra, double rb, double wa, double wb,
                                            double2 qp, double a, double b, double dt, int mode) {
  if (cc == 0) {
    if (mode == 0) {
      *reinterpret_cast<double2*>(out + q) = make_double2(ra, rb);
    } else {
      const double qa = a * qp.x + dt * ra, qb = a * qp.y + dt * rb;
      *reinterpret_cast<double2*>(Q + q) = make_double2(qa, qb);
      const double wna = wa + b * qa, wnb = wb + b * qb;
      *reinterpret_cast<double2*>(out + q) = make_double2(wna, wnb);
      mark_nonfinite(g, wna);
      mark_nonfinite(g, wnb);
    }
    return;
  }
  bulk_store(g, out, Q, (int8_t)(cc & 0xff), q, ra, wa, qp.x, a, b, dt, mode);
  bulk_store(g, out, Q, (int8_t)(cc >> 8), q + 1, rb, wb, qp.y, a, b, dt, mode);
}

__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }

// Two interior nodes i0, i0 + 1 (i0 even, every stencil position inside the
// grid, nx even, arrays 16-byte aligned) with 16-byte loads: the bulk part
// is bound by the number of load instructions (its bytes come from L2), and
// a pair needs 27 loads instead of 62.  The face between the two nodes is
// evaluated once.  Each node takes the formulas of bulk_cell (the results
// agree to rounding: the compiler may fuse other multiply-adds).
template <bool P>
__device__ __forceinline__ void bulk_pair(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                          double* __restrict__ out, double* __restrict__ Q, double a, double b,
                                          double dt, int mode, int i0, int j) {
  const int nx = g.nx, nxr = nx + 2;
  const double* __restrict__ psi = vel.psi;
  const int q = j * nx + i0;                 // even
  const int r = (j + 1) * nxr + i0 + 1;      // ring index of node i0 (odd)
  const unsigned short cc = *reinterpret_cast<const unsigned short*>(g.cls + q);
  const double2 qp = (mode == 1 && a != 0.0) ? ld2(Q + q) : make_double2(0.0, 0.0);
  // row j: omega and u at nodes i0 - 2 + m, m = 0 .. 5 (u from ring rows j + 2
  // and j, ring indices r - 3 + k, k = 0 .. 7)
  double wx[6], up[8], dn[8];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double2 w2 = ld2(omega + q - 2 + 2 * k);
    wx[2 * k] = w2.x;
    wx[2 * k + 1] = w2.y;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 u2 = ld2(psi + r + nxr - 3 + 2 * k), d2 = ld2(psi + r - nxr - 3 + 2 * k);
    up[2 * k] = u2.x;
    up[2 * k + 1] = u2.y;
    dn[2 * k] = d2.x;
    dn[2 * k + 1] = d2.y;
  }
  double ux[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) ux[m] = Vel<P>::u_of(g, up[m + 1], dn[m + 1]);
  // columns i0, i0 + 1: omega and v at rows j - 2 + d, d = 0 .. 4 (v from ring
  // columns i0 .. i0 + 3 of ring row j - 1 + d)
  double wya[5], wyb[5], vya[5], vyb[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    const double2 w2 = d == 2 ? make_double2(wx[2], wx[3]) : ld2(omega + q + (d - 2) * nx);
    wya[d] = w2.x;
    wyb[d] = w2.y;
    const int rr = (j - 1 + d) * nxr + i0;   // ring column i0 of ring row j - 1 + d
    const double2 p0 = ld2(psi + rr), p1 = ld2(psi + rr + 2);
    vya[d] = Vel<P>::v_of(g, p1.x, p0.x);
    vyb[d] = Vel<P>::v_of(g, p1.y, p0.y);
  }
  const double nih = g.nu * g.inv_h;
  const double fmid = flux_std(ux[1], ux[2], ux[3], ux[4], wx[1], wx[2], wx[3], wx[4], nih);   // face i0 + 1/2
  const double fxla = flux_std(ux[0], ux[1], ux[2], ux[3], wx[0], wx[1], wx[2], wx[3], nih);
  const double fxrb = flux_std(ux[2], ux[3], ux[4], ux[5], wx[2], wx[3], wx[4], wx[5], nih);
  const double fyta = flux_std(vya[1], vya[2], vya[3], vya[4], wya[1], wya[2], wya[3], wya[4], nih);
  const double fyba = flux_std(vya[0], vya[1], vya[2], vya[3], wya[0], wya[1], wya[2], wya[3], nih);
  const double fytb = flux_std(vyb[1], vyb[2], vyb[3], vyb[4], wyb[1], wyb[2], wyb[3], wyb[4], nih);
  const double fybb = flux_std(vyb[0], vyb[1], vyb[2], vyb[3], wyb[0], wyb[1], wyb[2], wyb[3], nih);
  double rha = -((fmid - fxla) + (fyta - fyba)) * g.inv_h;
  double rhb = -((fxrb - fmid) + (fytb - fybb)) * g.inv_h;
  // keeps every load above the class tests (see bulk_cell)
  asm volatile("" : "+v"(rha), "+v"(rhb));
  bulk_store2(g, out, Q, cc, q, rha, rhb, wx[2], wx[3], qp, a, b, dt, mode);
}

// A 2 x 2 block of interior nodes: rows j, j + 1 and columns i0, i0 + 1 (the
// conditions of bulk_pair, with the stencils of both rows inside the grid).
// The two rows share the omega and psi rows their stencils overlap on, each
// row its middle x face and each column its middle y face, so the block takes
// 34 loads instead of the 54 of two pairs.  Every node takes the formulas of
// bulk_cell (the results agree to rounding).
template <bool P>
__device__ __forceinline__ void bulk_quad(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                          double* __restrict__ out, double* __restrict__ Q, double a, double b,
                                          double dt, int mode, int i0, int j) {
  const int nx = g.nx, nxr = nx + 2;
  const double* __restrict__ psi = vel.psi;
  const int q = j * nx + i0;                 // even, as is q + nx
  const unsigned short c0 = *reinterpret_cast<const unsigned short*>(g.cls + q);
  const unsigned short c1 = *reinterpret_cast<const unsigned short*>(g.cls + q + nx);
  const bool rq = mode == 1 && a != 0.0;
  const double2 q0 = rq ? ld2(Q + q) : make_double2(0.0, 0.0);
  const double2 q1 = rq ? ld2(Q + q + nx) : make_double2(0.0, 0.0);
  // omega of rows j - 2 + d, d = 0 .. 5: columns i0 - 2 .. i0 + 3 on rows j
  // and j + 1, columns i0 and i0 + 1 on the other four
  double wr[2][6];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 w2 = ld2(omega + q + s * nx - 2 + 2 * k);
      wr[s][2 * k] = w2.x;
      wr[s][2 * k + 1] = w2.y;
    }
  double2 wo[4];   // rows j - 2, j - 1, j + 2, j + 3
#pragma unroll
  for (int d = 0; d < 4; ++d) wo[d] = ld2(omega + q + (d < 2 ? d - 2 : d) * nx);
  // psi of ring rows j + e, e = 0 .. 3 (grid rows j - 1 .. j + 2), ring
  // columns i0 - 2 .. i0 + 5: u of rows j and j + 1 and v of the middle rows;
  // ring rows j - 1 and j + 4, ring columns i0 .. i0 + 3: v of the outer rows
  const int r0 = j * nxr + i0;               // ring row j, ring column i0 (even)
  double pr[4][8];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 p2 = ld2(psi + r0 + e * nxr - 2 + 2 * k);
      pr[e][2 * k] = p2.x;
      pr[e][2 * k + 1] = p2.y;
    }
  double2 po[4];   // ring row j - 1 then j + 4, ring columns i0, i0 + 1 then i0 + 2, i0 + 3
#pragma unroll
  for (int t = 0; t < 4; ++t) po[t] = ld2(psi + r0 + (t < 2 ? -nxr : 4 * nxr) + 2 * (t & 1));
  // all 30 loads are issued before any of them is used: left alone, the
  // compiler holds the last ones back until most others have returned (to
  // save registers), which costs each wave a second memory round trip
  asm volatile("" : "+v"(wo[0].x), "+v"(wo[0].y), "+v"(wo[1].x), "+v"(wo[1].y), "+v"(wo[2].x), "+v"(wo[2].y),
               "+v"(wo[3].x), "+v"(wo[3].y), "+v"(po[0].x), "+v"(po[0].y), "+v"(po[1].x), "+v"(po[1].y),
               "+v"(po[2].x), "+v"(po[2].y), "+v"(po[3].x), "+v"(po[3].y));
  double ux[2][6];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int m = 0; m < 6; ++m) ux[s][m] = Vel<P>::u_of(g, pr[s + 2][m + 1], pr[s][m + 1]);
  // columns i0 (a) and i0 + 1 (b) on grid rows j - 2 + d (ring row j - 1 + d,
  // ring columns i0 .. i0 + 3)
  double wya[6], wyb[6], vya[6], vyb[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const double2 w2 = (d == 2 || d == 3) ? make_double2(wr[d - 2][2], wr[d - 2][3]) : wo[d < 2 ? d : d - 2];
    wya[d] = w2.x;
    wyb[d] = w2.y;
    double p[4];
    if (d == 0 || d == 5) {
      const int o = d == 0 ? 0 : 2;
      p[0] = po[o].x; p[1] = po[o].y; p[2] = po[o + 1].x; p[3] = po[o + 1].y;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) p[t] = pr[d - 1][2 + t];
    }
    vya[d] = Vel<P>::v_of(g, p[2], p[0]);
    vyb[d] = Vel<P>::v_of(g, p[3], p[1]);
  }
  const double nih = g.nu * g.inv_h;
  double fx[2][3], fya[3], fyb[3];   // x faces i0 - 1/2, i0 + 1/2, i0 + 3/2; y faces j - 1/2, j + 1/2, j + 3/2
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      fx[s][k] = flux_std(ux[s][k], ux[s][k + 1], ux[s][k + 2], ux[s][k + 3], wr[s][k], wr[s][k + 1], wr[s][k + 2],
                          wr[s][k + 3], nih);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    fya[k] = flux_std(vya[k], vya[k + 1], vya[k + 2], vya[k + 3], wya[k], wya[k + 1], wya[k + 2], wya[k + 3], nih);
    fyb[k] = flux_std(vyb[k], vyb[k + 1], vyb[k + 2], vyb[k + 3], wyb[k], wyb[k + 1], wyb[k + 2], wyb[k + 3], nih);
  }
  double r00 = -((fx[0][1] - fx[0][0]) + (fya[1] - fya[0])) * g.inv_h;
  double r01 = -((fx[0][2] - fx[0][1]) + (fyb[1] - fyb[0])) * g.inv_h;
  double r10 = -((fx[1][1] - fx[1][0]) + (fya[2] - fya[1])) * g.inv_h;
  double r11 = -((fx[1][2] - fx[1][1]) + (fyb[2] - fyb[1])) * g.inv_h;
  // keeps every load above the class tests (see bulk_cell)
  asm volatile("" : "+v"(r00), "+v"(r01), "+v"(r10), "+v"(r11));
  bulk_store2(g, out, Q, c0, q, r00, r01, wr[0][2], wr[0][3], q0, a, b, dt, mode);
  bulk_store2(g, out, Q, c1, q + nx, r10, r11, wr[1][2], wr[1][3], q1, a, b, dt, mode);
}

// Nodes i0, i0 + 1 of row j.
template <bool P>
__device__ __forceinline__ void bulk_two(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                         double* __restrict__ out, double* __restrict__ Q, double a, double b,
                                         double dt, int mode, int i0, int j) {
  if constexpr (P) {
    if (g.vec && i0 >= 2 && i0 + 4 <= g.nx && j >= 2 && j + 2 < g.ny) {
      bulk_pair(g, omega, vel, out, Q, a, b, dt, mode, i0, j);
      return;
    }
  }
  bulk_cell(g, omega, vel, out, Q, a, b, dt, mode, i0, j);
  bulk_cell(g, omega, vel, out, Q, a, b, dt, mode, i0 + 1, j);
}

// Bulk tile (bx, jt), columns 512 bx .. 512 bx + 511: row jt, a pair of
// nodes per lane, or (g.quad) rows 2 jt and 2 jt + 1, a 2 x 2 block of nodes
// per lane.
template <bool P>
__device__ __forceinline__ void transport_bulk(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                               double* __restrict__ out, double* __restrict__ Q, double a, double b,
                                               double dt, int mode, int bx, int jt) {
  const int i0 = 2 * (bx * 256 + threadIdx.x);
  if (i0 >= g.nx) return;
  if (!g.quad) {
    bulk_two(g, omega, vel, out, Q, a, b, dt, mode, i0, jt);
    return;
  }
  const int j = 2 * jt;
  if constexpr (P) {
    if (i0 >= 2 && i0 + 4 <= g.nx && j >= 2 && j + 3 < g.ny) {
      bulk_quad(g, omega, vel, out, Q, a, b, dt, mode, i0, j);
      return;
    }
  }
  bulk_two(g, omega, vel, out, Q, a, b, dt, mode, i0, j);
  if (j + 1 < g.ny) bulk_two(g, omega, vel, out, Q, a, b, dt, mode, i0, j + 1);
}

// One group of 4 lanes per boundary-kernel node: lane f computes the flux on
// face f (right, left, top, bottom); lane 0 of the group combines them.
template <bool P>
__device__ __forceinline__ void transport_special(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                                  const double* __restrict__ w4, const double* __restrict__ w3b,
                                                  const double* __restrict__ w3n, double* __restrict__ out,
                                                  double* __restrict__ Q, double a, double b, double dt, int mode,
                                                  int bx) {
  const int tid = bx * 256 + threadIdx.x;
  const int sp = tid >> 2, face = tid & 3;
  const bool act = sp < g.nsp;
  int q = 0;
  double fl = 0.0;
  double qp = 0.0, wq = 0.0;
  if (act) {
    q = g.special[sp];
    if (face == 0 && mode == 1) {
      qp = a == 0.0 ? 0.0 : Q[q];
      wq = omega[q];
    }
    const int i = q % g.nx, j = q / g.nx;
    const int fi = face == 1 ? i - 1 : i, fj = face == 3 ? j - 1 : j;
    fl = flux_general(g, omega, vel, w4, w3b, w3n, fi, fj, face >> 1);
  }
  const int base = (threadIdx.x & 63) & ~3;
  const double fxr = __shfl(fl, base, 64), fxl = __shfl(fl, base + 1, 64);
  const double fyt = __shfl(fl, base + 2, 64), fyb = __shfl(fl, base + 3, 64);
  if (!act || face != 0) return;
  const double rhs = -((fxr - fxl) + (fyt - fyb)) * g.inv_h;
  if (mode == 0) {
    out[q] = rhs;
  } else {
    const double qn = a * qp + dt * rhs;
    Q[q] = qn;
    const double wn = wq + b * qn;
    out[q] = wn;
    mark_nonfinite(g, wn);
  }
}

// Kelvin: one block per circulating body
template <bool P>
__device__ __forceinline__ void kelvin(const TGeom& g, const double* __restrict__ omega, const Vel<P>& vel,
                                       double* __restrict__ dG,
                                       double* __restrict__ Gamma, double* __restrict__ QG, double a, double b,
                                       double dt, int mode, int k, double* red) {
  const int i0 = g.rects[4 * k], i1 = g.rects[4 * k + 1], j0 = g.rects[4 * k + 2], j1 = g.rects[4 * k + 3];
  const int nv = j1 - j0 + 1, nh = i1 - i0 + 1;
  double acc = 0.0;
  const int nf = 2 * (nv + nh);
  // face t: right (+), left (-), top (+), bottom (-) faces in turn; the face
  // is selected arithmetically, so that every lane runs one flux evaluation
  auto face = [&](int t) {
    const bool vert = t < 2 * nv, first = vert ? t < nv : t < 2 * nv + nh;
    const int s = vert ? (first ? t : t - nv) : (first ? t - 2 * nv : t - 2 * nv - nh);
    const int fi = vert ? (first ? i1 : i0 - 1) : i0 + s;
    const int fj = vert ? j0 + s : (first ? j1 : j0 - 1);
    const double f = flux_interior(g, omega, vel, fi, fj, vert ? 0 : 1);
    return first ? f : -f;
  };
  for (int t = threadIdx.x; t < nf; t += 2 * blockDim.x) {
    const int t2 = t + blockDim.x;
    const double a0 = face(t), a1 = t2 < nf ? face(t2) : 0.0;
    acc += a0;
    acc += a1;
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) {
    const double rate = -g.h * tot;
    dG[k] = rate;
    if (mode == 1) {
      const double qp = a == 0.0 ? 0.0 : QG[k];
      const double qn = a * qp + dt * rate;
      QG[k] = qn;
      const double gn = Gamma[k] + b * qn;
      Gamma[k] = gn;
      mark_nonfinite(g, gn);
    }
  }
}

// Transport of every fluid node and the Kelvin update in one launch of
// 256-thread blocks: first one block per circulating body and the
// boundary-kernel nodes (4 lanes each), whose dependent loads take longest,
// so that they are dispatched first, then the bulk rows.  The three parts
// read the same inputs and write disjoint outputs.
//
// Workgroups go to the eight XCDs in turn (block b to XCD b mod 8), and each
// XCD has its own L2.  The bulk part therefore starts at a multiple of eight
// and hands XCD x one contiguous band of rows: the five-row stencils of
// neighbouring rows then hit the same L2, and only the band edges are read
// from HBM twice (with consecutive rows on alternating XCDs every row of
// omega and psi was read twice).
// Grid size (nodes) from which the bulk part takes 2 x 2 blocks per lane:
// about where the pair tiles need two rounds of waves to cover the grid.
constexpr long TRANSPORT_QUAD_MIN = 1L << 20;

template <bool P>
__global__ void __launch_bounds__(256) k_transport_all(TGeom g, const double* __restrict__ omega,
                                                       const double* __restrict__ psi,
                                                       const double* __restrict__ U, const double* __restrict__ V,
                                                       const double* __restrict__ w4, const double* __restrict__ w3b,
                                                       const double* __restrict__ w3n, double* __restrict__ out,
                                                       double* __restrict__ Q, double* __restrict__ dG,
                                                       double* __restrict__ Gamma, double* __restrict__ QG, double a,
                                                       double b, double dt, int mode) {
  __shared__ double red[16];
  const Vel<P> vel{psi, U, V};
  const int nbx = (g.nx + 511) / 512, nb_sp = (4 * g.nsp + 255) / 256;
  int blk = blockIdx.x;
  if (blk < g.nbc) {
    kelvin(g, omega, vel, dG, Gamma, QG, a, b, dt, mode, blk, red);
    return;
  }
  blk -= g.nbc;
  if (blk < nb_sp) {
    transport_special(g, omega, vel, w4, w3b, w3n, out, Q, a, b, dt, mode, blk);
    return;
  }
  const int nlead = (g.nbc + nb_sp + 7) & ~7;
  const int nb = nbx * (g.quad ? (g.ny + 1) >> 1 : g.ny), band = (nb + 7) >> 3;
  const int bb = (int)blockIdx.x - nlead;
  if (bb < 0) return;   // padding up to the first bulk block
  const int tile = (bb & 7) * band + (bb >> 3);
  if (tile >= nb) return;
  transport_bulk(g, omega, vel, out, Q, a, b, dt, mode, tile % nbx, tile / nbx);
}

void launch_transport_all(const DGeom& g, const double* omega, const double* psi, const double* U, const double* V,
                          const double* w4, const double* w3b, const double* w3n, double* out, double* Q, double* dG,
                          double* Gamma, double* QG, double a, double b, double dt, int mode, hipStream_t s,
                          Prof* prof) {
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const int vec = psi && g.nx % 2 == 0 && al16(omega) && al16(psi) && al16(out) && al16(Q) &&
                  ((uintptr_t)g.cls & 1) == 0;
  // 2 x 2 blocks per lane take fewer loads per node but give half as many
  // waves: they pay once the grid fills the chip several times over
  const int quad = vec && (long)g.nx * g.ny >= TRANSPORT_QUAD_MIN;
  // leading blocks padded to a multiple of 8; eight bands of bulk tiles
  // (one or two rows of 512 nodes each)
  const int nb = ((g.nx + 511) / 512) * (quad ? (g.ny + 1) / 2 : g.ny);
  const int blocks = ((g.nbc + (4 * g.nsp + 255) / 256 + 7) & ~7) + 8 * ((nb + 7) / 8);
  const TGeom tg{g.nx, g.ny, g.nsp, g.nbc, g.outflow, g.periodic, vec, quad, g.h, g.inv_h, g.nu, g.uinf_x, g.uinf_y, g.cls,
                 g.special, g.rects, g.nonfinite};
  if (psi) {
    // algorithmic bytes per cell: omega, psi, Q read; out, Q written
    IIM_LAUNCH(prof, KID_TRANSPORT, 40.0 * g.nx * g.ny, k_transport_all<true>, blocks, 256, s, tg, omega, psi, U, V,
               w4, w3b, w3n, out, Q, dG, Gamma, QG, a, b, dt, mode);
  } else {
    // algorithmic bytes per cell: omega, u, v, Q read; out, Q written
    IIM_LAUNCH(prof, KID_TRANSPORT, 48.0 * g.nx * g.ny, k_transport_all<false>, blocks, 256, s, tg, omega, psi, U, V,
               w4, w3b, w3n, out, Q, dG, Gamma, QG, a, b, dt, mode);
  }
}

}  // namespace iim

namespace iim {

// ============================================================ dense Schur inverse
// In-place Gauss-Jordan inversion with partial pivoting of an n x n row-major
// matrix M (device).  Step k: pick the pivot row, swap it into row k, scale
// row k, save column k; then eliminate column k from every other row.
__global__ void __launch_bounds__(1024) k_gj_pivot(double* M, int n, int k, int* perm, double* fcol, double* info) {
  __shared__ double vbest[16];
  __shared__ int ibest[16];
  double best = -1.0;
  int bi = k;
  for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
    const double v = fabs(M[(size_t)i * n + k]);
    if (v > best) { best = v; bi = i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { vbest[wid] = best; ibest[wid] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
      if (vbest[q] > vbest[0] || (vbest[q] == vbest[0] && ibest[q] < ibest[0])) { vbest[0] = vbest[q]; ibest[0] = ibest[q]; }
    perm[k] = ibest[0];
    if (!(vbest[0] > 0.0)) info[0] = 1.0;   // singular
  }
  __syncthreads();
  const int p = ibest[0];
  if (p != k)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const double a = M[(size_t)k * n + j];
      M[(size_t)k * n + j] = M[(size_t)p * n + j];
      M[(size_t)p * n + j] = a;
    }
  __syncthreads();
  const double piv = M[(size_t)k * n + k];
  const double inv = piv != 0.0 ? 1.0 / piv : 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double a = (j == k) ? 1.0 : M[(size_t)k * n + j];
    M[(size_t)k * n + j] = a * inv;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) fcol[i] = (i == k) ? 0.0 : M[(size_t)i * n + k];
}

__global__ void k_gj_elim(double* M, int n, int k, const double* __restrict__ fcol) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || i == k) return;
  const double f = fcol[i];
  const double rk = M[(size_t)k * n + j];
  const double a = (j == k) ? 0.0 : M[(size_t)i * n + j];
  M[(size_t)i * n + j] = a - f * rk;
}

// undo the row interchanges as column interchanges, last first
__global__ void k_gj_colswap(double* M, int n, const int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* row = M + (size_t)i * n;
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k) {
      const double a = row[k];
      row[k] = row[p];
      row[p] = a;
    }
  }
}

void launch_gj_invert(double* M, int n, int* perm, double* fcol, double* info, hipStream_t s) {
  for (int k = 0; k < n; ++k) {
    k_gj_pivot<<<1, 1024, 0, s>>>(M, n, k, perm, fcol, info);
    dim3 grid((n + 255) / 256, n);
    k_gj_elim<<<grid, 256, 0, s>>>(M, n, k, fcol);
  }
  k_gj_colswap<<<(n + 255) / 256, 256, 0, s>>>(M, n, perm);
}

// x[p] = sum_q Mt[q][p] b[q]   (Mt = transpose of the inverse, row-major)
// x = Mt^T b for a dense n x n row-major Mt (the transposed Schur inverse):
// a bandwidth-bound product of n^2 doubles.  The rows of Mt are split into
// segments of GEMV_ROWS: block (tile, segment) gives each of its 256 lanes one
// output p of the tile and sums its segment's rows in order, sixteen loads in
// flight at a time (coalesced along p); a second launch adds the segments'
// partial sums of each output in segment order (deterministic).  Enough
// blocks to fill the chip even for n of a few thousand.
constexpr int GEMV_ROWS = 64;
int gemv_t_parts(int n) { return (n + GEMV_ROWS - 1) / GEMV_ROWS; }

__global__ void __launch_bounds__(256) k_gemv_t_part(const double* __restrict__ Mt, int n,
                                                     const double* __restrict__ b, double* __restrict__ part) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int q0 = blockIdx.y * GEMV_ROWS, q1 = min(q0 + GEMV_ROWS, n);
  if (p >= n) return;
  double acc = 0.0;
  int q = q0;
  for (; q + 16 <= q1; q += 16) {
    double m[16], bb[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      m[u] = Mt[(size_t)(q + u) * n + p];
      bb[u] = b[q + u];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += m[u] * bb[u];
  }
  for (; q < q1; ++q) acc += Mt[(size_t)q * n + p] * b[q];
  part[(size_t)blockIdx.y * n + p] = acc;
}

__global__ void __launch_bounds__(256) k_gemv_t_sum(const double* __restrict__ part, int parts, int n,
                                                    double* __restrict__ x) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  double t = 0.0;
  int s = 0;
  for (; s + 8 <= parts; s += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(s + u) * n + p];
#pragma unroll
    for (int u = 0; u < 8; ++u) t += v[u];
  }
  for (; s < parts; ++s) t += part[(size_t)s * n + p];
  x[p] = t;
}

void launch_gemv_t(const double* Mt, int n, const double* b, double* x, double* part, hipStream_t s) {
  if (n <= 0) return;
  const int tiles = (n + 255) / 256, parts = gemv_t_parts(n);
  k_gemv_t_part<<<dim3(tiles, parts), 256, 0, s>>>(Mt, n, b, part);
  k_gemv_t_sum<<<tiles, 256, 0, s>>>(part, parts, n, x);
}

// Right-hand side and direct solve in one launch: every block builds all of b
// in LDS (the correction rows are short sparse sums of psi, the circulation
// rows one masked rectangle sum of omega per body), then 16 entries of
// x = Mt^T b, its matrix entries loaded before b is ready.  The correction
// rows are formed entry-parallel: each lane stores the products w psi of a
// few entries in LDS (all their loads in flight together), then the lane
// owning a row sums its entries in order.  The circulation rows' wave sums
// go to LDS and are added, in wave order, in the phase after the next
// barrier (no block reduction of their own).  Block 0 also stores b.
constexpr int RHS_SOLVE_MAX_LDS = 6144;   // b, the entry products and the wave sums in dynamic LDS (48 KiB)
__global__ void __launch_bounds__(1024) k_rhs_solve(DGeom g, const double* __restrict__ psi,
                                                   const double* __restrict__ omega,
                                                   const double* __restrict__ Gamma,
                                                   const double* __restrict__ Mt, int n, double* __restrict__ b,
                                                   double* __restrict__ x) {
  extern __shared__ double bs[];   // b [n], the entry products [nnz], a spare slot, the wave sums [nbc][16]
  __shared__ double part[64][17];
  const int lo = threadIdx.x & 15, sl = threadIdx.x >> 4;   // 16 outputs, 64 slices of each sum
  const int p = blockIdx.x * 16 + lo;
  double mv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = sl + 64 * u;
    mv[u] = (p < n && q < n) ? Mt[(size_t)q * n + p] : 0.0;
  }
  // this lane's first correction row: entry range and constant, loaded now
  const int a_own = threadIdx.x;
  const bool own = a_own < g.na;
  const int pb = own ? g.aop.ptr[a_own] : 0, pe = own ? g.aop.ptr[a_own + 1] : 0;
  const double bconst = own ? g.bpsi[a_own] : 0.0;
  const double gam_own = (int)threadIdx.x < g.nbc ? Gamma[threadIdx.x] : 0.0;
  double* terms = bs + n;
  const int nnz = g.aop.nnz;
  constexpr int NW = 16;   // waves of the 1024-lane block
  double* wsum = terms + nnz + 1;
  for (int e0 = threadIdx.x; e0 < nnz; e0 += 2 * blockDim.x) {
    // the second entry at a clamped index and stored unconditionally (past
    // the end into the spare slot terms[nnz]): under a per-lane branch its
    // loads would be issued, and waited for, after the first entry's
    const int e1 = e0 + blockDim.x, e1c = min(e1, nnz - 1);
    const int r0 = g.aop.ridx[e0], r1 = g.aop.ridx[e1c];
    const double w0 = g.aop.w[e0], w1 = g.aop.w[e1c];
    const double p0 = psi[r0], p1 = psi[r1];
    terms[e0] = w0 * p0;
    terms[min(e1, nnz)] = w1 * p1;
  }
  for (int k = 0; k < g.nbc; ++k) {
    const int i0 = g.rects[4 * k], i1 = g.rects[4 * k + 1], j0 = g.rects[4 * k + 2], j1 = g.rects[4 * k + 3];
    const int w = i1 - i0 + 1, cnt = w * (j1 - j0 + 1);
    double acc = 0.0;
    for (int q0 = threadIdx.x; q0 < cnt; q0 += 8 * blockDim.x) {
      double v[8];
      int8_t cl[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * blockDim.x;
        cl[u] = 3;
        v[u] = 0.0;
        if (q < cnt) {
          const int idx = (j0 + q / w) * g.nx + i0 + q % w;
          cl[u] = g.cls[idx];
          v[u] = omega[idx];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (cl[u] < 2) acc += v[u];
    }
    const double ws = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) wsum[k * NW + (threadIdx.x >> 6)] = ws;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < g.nbc; k += blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < NW; ++q) t += wsum[k * NW + q];
    bs[g.na + k] = t - (k == (int)threadIdx.x ? gam_own : Gamma[k]) * g.inv_h * g.inv_h;
  }
  for (int a = threadIdx.x; a < g.na; a += blockDim.x) {
    const bool first = a == a_own;
    const int e1 = first ? pe : g.aop.ptr[a + 1];
    double acc = 0.0;
    for (int e = first ? pb : g.aop.ptr[a]; e < e1; ++e) acc += terms[e];
    bs[a] = acc + (first ? bconst : g.bpsi[a]);
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < n; q += blockDim.x) b[q] = bs[q];
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = sl + 64 * u;
    if (q < n) acc += mv[u] * bs[q];
  }
  if (p < n)
    for (int q = sl + 512; q < n; q += 64) acc += Mt[(size_t)q * n + p] * bs[q];
  part[sl][lo] = acc;
  __syncthreads();
  if (threadIdx.x < 16 && p < n) {
    double t = 0.0;
    for (int k = 0; k < 64; ++k) t += part[k][lo];
    x[p] = t;
  }
}

bool launch_rhs_solve(const DGeom& g, const double* psi_ring, const double* omega, const double* Gamma,
                      const double* Mt, int n, double* b, double* x, hipStream_t s) {
  const size_t lds = (size_t)n + g.aop.nnz + 1 + 16 * (size_t)g.nbc;
  if (n != g.na + g.nbc || lds > RHS_SOLVE_MAX_LDS) return false;
  if (n == 0) return true;
  k_rhs_solve<<<(n + 15) / 16, 1024, lds * sizeof(double), s>>>(g, psi_ring, omega, Gamma, Mt, n, b, x);
  return true;
}

__global__ void k_unit(double* v, int n, int q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (i == q) ? 1.0 : 0.0;
}
void launch_unit(double* v, int n, int q, hipStream_t s) {
  if (n > 0) k_unit<<<(n + 255) / 256, 256, 0, s>>>(v, n, q);
}

}  // namespace iim

namespace iim {

// ============================================================ register FFT
// FFT of N >= 256 points by T threads; thread t holds E = N / T points in
// registers in the layout x[t + T m].  Every Stockham pass of radix R reads its
// butterfly inputs x[j + r N/R] (j = t + T b) straight from registers, applies
// the twiddles W_{Ns R}^{r k}, does the radix-R DFT in registers and writes the
// outputs to LDS in Stockham order; the next pass reloads the [t + T m] layout.
// The last pass leaves its output in registers, again in the [t + T m] layout.
template <int N>
struct RP;
template <> struct RP<256> { static constexpr int T = 64, E = 4; };
template <> struct RP<512> { static constexpr int T = 64, E = 8; };
#ifndef IIM_FFT1024_THREADS
#define IIM_FFT1024_THREADS 128
#endif
template <> struct RP<1024> { static constexpr int T = IIM_FFT1024_THREADS, E = 1024 / IIM_FFT1024_THREADS; };
template <> struct RP<2048> { static constexpr int T = 128, E = 16; };
template <> struct RP<4096> { static constexpr int T = 256, E = 16; };
// tori with a factor 3 or 5 (FP64), so that a padded size can follow 2N
// instead of the next power of two: E divisible by every radix of the plan
template <> struct RP<320> { static constexpr int T = 16, E = 20; };
template <> struct RP<384> { static constexpr int T = 32, E = 12; };
template <> struct RP<640> { static constexpr int T = 32, E = 20; };
template <> struct RP<768> { static constexpr int T = 64, E = 12; };
template <> struct RP<1280> { static constexpr int T = 64, E = 20; };
template <> struct RP<1536> { static constexpr int T = 128, E = 12; };
// Lanes per FFT of the row passes (ROWS) and of the column pass: the same
// except at 1024 points, where the row passes run 256 lanes of 4 points
// (faster there) and the column pass 128 lanes of 8 (faster there).
#ifndef IIM_ROW_FFT1024_THREADS
#define IIM_ROW_FFT1024_THREADS 256
#endif
template <int N, bool ROWS>
struct RPX {
  static constexpr int T = RP<N>::T, E = RP<N>::E;
};
template <>
struct RPX<1024, true> {
  static constexpr int T = IIM_ROW_FFT1024_THREADS, E = 1024 / IIM_ROW_FFT1024_THREADS;
};

#ifndef IIM_ROW_FFTS_PER_BLOCK
#define IIM_ROW_FFTS_PER_BLOCK 4
#endif
#ifndef IIM_COL_FFTS_PER_BLOCK
#define IIM_COL_FFTS_PER_BLOCK 4
#endif
// FFTs per block: the default of the row passes (ROWS) and of the column
// pass; a tuned value (DFft::row_per / col_per) selects another instantiation
// (column pass: one FFT per block once an FFT has 128 lanes or more, which
// measured faster inside the time step at 1024 points)
template <int N, bool ROWS = false>
struct RegDef {
  static constexpr int T = RPX<N, ROWS>::T;
  static constexpr int WANT = ROWS ? IIM_ROW_FFTS_PER_BLOCK : IIM_COL_FFTS_PER_BLOCK;
  static constexpr int PER = (!ROWS && T >= 128) ? 1 : (WANT * T > 256) ? (256 / T > 0 ? 256 / T : 1) : WANT;
};
template <int N, int PER_, bool ROWS = false>
struct RegCfg {
  static constexpr int T = RPX<N, ROWS>::T;
  static constexpr int PER = PER_;
  static constexpr int THREADS = PER * T;
  static constexpr int LDSN = N + N / 16 + 1;      // padded length (one pad slot per 16 points)
};
// instantiated tile shapes: at most 1024 threads and 128 KiB of LDS per block
template <int N, int PER, class CX, bool ROWS = false>
constexpr bool per_ok() {
  return PER * RPX<N, ROWS>::T <= 1024 && (size_t)PER * (N + N / 16 + 1) * sizeof(CX) <= 131072;
}

__device__ __forceinline__ int padi(int i) { return i + (i >> 4); }

// Typed view of the convolution tables: FP64, or the FP32 copies used by the
// inner matrix-vector products of the mixed-precision solve.
template <class CX>
struct FftT {
  CX* spec;                    // row transforms (row pass output, column pass input)
  CX* out;                     // column pass output, inverse row pass input
  const CX* tw_x;
  const CX* tw_xr;
  const CX* tw_y;
  const typename Real<CX>::t* ghat;
};
template <class CX>
__device__ __forceinline__ FftT<CX> fft_view(const DFft& f);
template <>
__device__ __forceinline__ FftT<double2> fft_view<double2>(const DFft& f) {
  return FftT<double2>{f.spec, f.spec_out, f.tw_x, f.tw_xr, f.tw_y, f.ghat};
}
template <>
__device__ __forceinline__ FftT<float2> fft_view<float2>(const DFft& f) {
  return FftT<float2>{f.spec32, f.spec32_out, f.tw_x32, f.tw_xr32, f.tw_y32, f.ghat32};
}

// a comma inside a macro argument (template arguments of a launched kernel)
#define IIM_COMMA ,


// The hardware deals consecutive workgroups round-robin to the 8 XCDs, each
// with its own L2.  Row passes give consecutive spectrum rows to consecutive
// logical blocks, and 128-byte lines of the spectrum span several of them:
// hand each XCD a contiguous range of logical blocks so that the blocks
// sharing a line meet in one L2 (otherwise every XCD fetches, and writes
// back, its own partial copy of the line).
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int x = b & 7, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

template <bool INV, class CX>
__device__ __forceinline__ void dft4(CX& a0, CX& a1, CX& a2, CX& a3) {
  const CX s0 = cadd(a0, a2), d0 = csub(a0, a2), s1 = cadd(a1, a3), d1 = csub(a1, a3);
  const CX e = INV ? mkc<CX>(-d1.y, d1.x) : mkc<CX>(d1.y, -d1.x);
  a0 = cadd(s0, s1);
  a2 = csub(s0, s1);
  a1 = cadd(d0, e);
  a3 = csub(d0, e);
}

// exp(-2 pi i e / 16) (forward) for e = 0..15
template <class CX>
__device__ __forceinline__ CX w16(int e, bool inv) {
  using S = typename Real<CX>::t;
  const S C1 = (S)0.92387953251128675613, S1 = (S)0.38268343236508977173, R2 = (S)0.70710678118654752440;
  S c, s;
  switch (e & 15) {
    case 0: c = 1.0; s = 0.0; break;
    case 1: c = C1; s = S1; break;
    case 2: c = R2; s = R2; break;
    case 3: c = S1; s = C1; break;
    case 4: c = 0.0; s = 1.0; break;
    case 5: c = -S1; s = C1; break;
    case 6: c = -R2; s = R2; break;
    case 7: c = -C1; s = S1; break;
    case 8: c = -1.0; s = 0.0; break;
    case 9: c = -C1; s = -S1; break;
    case 10: c = -R2; s = -R2; break;
    case 11: c = -S1; s = -C1; break;
    case 12: c = 0.0; s = -1.0; break;
    case 13: c = S1; s = -C1; break;
    case 14: c = R2; s = -R2; break;
    default: c = C1; s = -S1; break;
  }
  return mkc<CX>(c, inv ? s : -s);
}

template <int R, bool INV, class CX>
__device__ __forceinline__ void dftR(CX (&u)[R]) {
  using S = typename Real<CX>::t;
  if constexpr (R == 3) {
    // y1, y2 = x0 - (x1 + x2) / 2 -/+ i (sqrt 3 / 2)(x1 - x2) (forward W = exp(-2 pi i / 3))
    const S h = (S)0.86602540378443864676;
    const CX a = cadd(u[1], u[2]), d = csub(u[1], u[2]);
    const CX m = mkc<CX>(u[0].x - S(0.5) * a.x, u[0].y - S(0.5) * a.y);
    const CX r = INV ? mkc<CX>(-h * d.y, h * d.x) : mkc<CX>(h * d.y, -h * d.x);   // -/+ i h d
    u[0] = cadd(u[0], a);
    u[1] = cadd(m, r);
    u[2] = csub(m, r);
  } else if constexpr (R == 5) {
    // pairs (x1, x4), (x2, x3): y_k = x0 + c(k) sums - i s(k) differences
    const S c1 = (S)0.30901699437494742410, c2 = (S)-0.80901699437494742410;
    const S s1 = (S)0.95105651629515357212, s2 = (S)0.58778525229247312917;
    const CX p1 = cadd(u[1], u[4]), q1 = csub(u[1], u[4]);
    const CX p2 = cadd(u[2], u[3]), q2 = csub(u[2], u[3]);
    const CX a1 = mkc<CX>(u[0].x + c1 * p1.x + c2 * p2.x, u[0].y + c1 * p1.y + c2 * p2.y);
    const CX a2 = mkc<CX>(u[0].x + c2 * p1.x + c1 * p2.x, u[0].y + c2 * p1.y + c1 * p2.y);
    const CX b1 = mkc<CX>(s1 * q1.x + s2 * q2.x, s1 * q1.y + s2 * q2.y);
    const CX b2 = mkc<CX>(s2 * q1.x - s1 * q2.x, s2 * q1.y - s1 * q2.y);
    // -i b = (b.y, -b.x); the inverse transform takes +i b
    const CX r1 = INV ? mkc<CX>(-b1.y, b1.x) : mkc<CX>(b1.y, -b1.x);
    const CX r2 = INV ? mkc<CX>(-b2.y, b2.x) : mkc<CX>(b2.y, -b2.x);
    u[0] = cadd(u[0], cadd(p1, p2));
    u[1] = cadd(a1, r1);
    u[4] = csub(a1, r1);
    u[2] = cadd(a2, r2);
    u[3] = csub(a2, r2);
  } else if constexpr (R == 2) {
    const CX a = u[0];
    u[0] = cadd(a, u[1]);
    u[1] = csub(a, u[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(u[0], u[1], u[2], u[3]);
  } else if constexpr (R == 8) {
    // n = q + 2 m: inner DFT4 over m, twiddle W8^{q s}, outer DFT2 over q
    dft4<INV>(u[0], u[2], u[4], u[6]);
    dft4<INV>(u[1], u[3], u[5], u[7]);
    CX o[8];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const CX a = u[2 * s];
      const CX b = cmul(u[2 * s + 1], w16<CX>(2 * s, INV));
      o[s] = cadd(a, b);
      o[s + 4] = csub(a, b);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = o[q];
  } else {
    static_assert(R == 16, "radix");
    // n = q + 4 m: inner DFT4 over m (elements q, q+4, q+8, q+12), twiddle W16^{q s}, outer DFT4 over q
#pragma unroll
    for (int q = 0; q < 4; ++q) dft4<INV>(u[q], u[q + 4], u[q + 8], u[q + 12]);
    // after the inner DFT, element q + 4 s holds A[q][s]
    CX o[16];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      CX b0 = u[0 + 4 * s];
      CX b1 = cmul(u[1 + 4 * s], w16<CX>(1 * s, INV));
      CX b2 = cmul(u[2 + 4 * s], w16<CX>(2 * s, INV));
      CX b3 = cmul(u[3 + 4 * s], w16<CX>(3 * s, INV));
      dft4<INV>(b0, b1, b2, b3);
      o[s] = b0;
      o[s + 4] = b1;
      o[s + 8] = b2;
      o[s + 12] = b3;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) u[q] = o[q];
  }
}

// Twiddles of one radix pass for lane t: W^(r k step), k = (t + T b) mod NS,
// r = 1 .. R-1 (none for the first pass, NS = 1).
template <int N, int T, int E, int R, int NS, class CX>
struct PassTw {
  static constexpr int B = E / R;
  static constexpr int K = NS > 1 ? R - 1 : 0;
  CX w[B][K > 0 ? K : 1];
  __device__ __forceinline__ void load(int t, const CX* __restrict__ tw) {
    if constexpr (NS > 1) {
      constexpr int step = N / (NS * R);
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int k = (t + T * b) % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) w[b][r - 1] = tw[r * k * step];
      }
    }
  }
};
struct NoTw {
  template <class CX>
  __device__ __forceinline__ void load(int, const CX* __restrict__) {}
};

// One radix-R Stockham pass.  The next pass's twiddles are requested first,
// so that their latency hides behind this pass's butterflies and LDS
// exchange (only one pass ahead: preloading every pass's twiddles costs
// registers and measured slower).
template <int N, int T, int E, int R, int NS, bool INV, bool LAST, class CX, class NX>
__device__ __forceinline__ void reg_pass(CX (&v)[E], CX* lds, int t, const PassTw<N, T, E, R, NS, CX>& pw, NX& nx,
                                         const CX* __restrict__ tw) {
  nx.load(t, tw);
  constexpr int B = E / R;
  CX u[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) u[b][r] = v[b + r * B];
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        CX w = pw.w[b][r - 1];
        if (INV) w.y = -w.y;
        u[b][r] = cmul(u[b][r], w);
      }
    }
    dftR<R, INV>(u[b]);
  }
  if (LAST) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * B] = u[b][r];
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + T * b;
      const int k = j % NS;
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[padi(base + r * NS)] = u[b][r];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[padi(t + T * m)];
    __syncthreads();
  }
}

// Radix passes (R, NS) of each register FFT: N points, E per lane.
template <int N, int E>
struct Plan;
template <> struct Plan<256, 4> {
  static constexpr int P = 4;
  static constexpr int R[P] = {4, 4, 4, 4}, NS[P] = {1, 4, 16, 64};
};
template <> struct Plan<512, 8> {
  static constexpr int P = 3;
  static constexpr int R[P] = {8, 8, 8}, NS[P] = {1, 8, 64};
};
template <> struct Plan<1024, 16> {
  static constexpr int P = 3;
  static constexpr int R[P] = {16, 16, 4}, NS[P] = {1, 16, 256};
};
template <> struct Plan<1024, 8> {
  static constexpr int P = 4;
  static constexpr int R[P] = {8, 8, 8, 2}, NS[P] = {1, 8, 64, 512};
};
template <> struct Plan<1024, 4> {
  static constexpr int P = 5;
  static constexpr int R[P] = {4, 4, 4, 4, 4}, NS[P] = {1, 4, 16, 64, 256};
};
template <> struct Plan<2048, 16> {
  static constexpr int P = 3;
  static constexpr int R[P] = {16, 16, 8}, NS[P] = {1, 16, 256};
};
template <> struct Plan<4096, 16> {
  static constexpr int P = 3;
  static constexpr int R[P] = {16, 16, 16}, NS[P] = {1, 16, 256};
};
template <> struct Plan<320, 20> {
  static constexpr int P = 4;
  static constexpr int R[P] = {5, 4, 4, 4}, NS[P] = {1, 5, 20, 80};
};
template <> struct Plan<384, 12> {
  static constexpr int P = 5;
  static constexpr int R[P] = {3, 4, 4, 4, 2}, NS[P] = {1, 3, 12, 48, 192};
};
template <> struct Plan<640, 20> {
  static constexpr int P = 5;
  static constexpr int R[P] = {5, 4, 4, 4, 2}, NS[P] = {1, 5, 20, 80, 320};
};
template <> struct Plan<768, 12> {
  static constexpr int P = 5;
  static constexpr int R[P] = {3, 4, 4, 4, 4}, NS[P] = {1, 3, 12, 48, 192};
};
template <> struct Plan<1280, 20> {
  static constexpr int P = 5;
  static constexpr int R[P] = {5, 4, 4, 4, 4}, NS[P] = {1, 5, 20, 80, 320};
};
template <> struct Plan<1536, 12> {
  static constexpr int P = 6;
  static constexpr int R[P] = {3, 4, 4, 4, 4, 2}, NS[P] = {1, 3, 12, 48, 192, 768};
};

template <int N, int E, int I, class CX>
using PlanTw = PassTw<N, N / E, E, Plan<N, E>::R[I], Plan<N, E>::NS[I], CX>;

template <int N, bool INV, class CX, int E, int I>
__device__ __forceinline__ void fft_passes(CX (&v)[E], CX* lds, int t, const CX* __restrict__ tw,
                                           const PlanTw<N, E, I, CX>& cur) {
  using PL = Plan<N, E>;
  constexpr int T = N / E;
  if constexpr (I + 1 < PL::P) {
    PlanTw<N, E, I + 1, CX> nxt;
    reg_pass<N, T, E, PL::R[I], PL::NS[I], INV, false>(v, lds, t, cur, nxt, tw);
    fft_passes<N, INV, CX, E, I + 1>(v, lds, t, tw, nxt);
  } else {
    NoTw none;
    reg_pass<N, T, E, PL::R[I], PL::NS[I], INV, true>(v, lds, t, cur, none, tw);
  }
}

// FP64 twiddles: a radix-R pass multiplies input r of a butterfly group by
// W^(r k step); the lane loads only W^(k step) for each of its groups, once
// per kernel for all passes (the same for the forward and the conjugated
// inverse FFT), and forms the powers by products where they are applied.
// The table loads were the longest dependent-latency chain of the passes;
// the products add r - 1 roundings (about 1e-16 each) to a twiddle.
template <int N, int E, class CX>
struct Tw1 {
  using PL = Plan<N, E>;
  static constexpr int T = N / E;
  CX w[PL::P][E];
  __device__ __forceinline__ void load(int t, const CX* __restrict__ tw) {
#pragma unroll
    for (int i = 1; i < PL::P; ++i) {           // the first pass has NS = 1, no twiddles
      const int R = PL::R[i], NS = PL::NS[i], step = N / (NS * R);
#pragma unroll
      for (int b = 0; b < E; ++b)
        if (b < E / R) w[i][b] = tw[((t + T * b) % NS) * step];
    }
  }
};

template <int N, int T, int E, int R, int NS, bool INV, bool LAST, class CX>
__device__ __forceinline__ void reg_pass_w(CX (&v)[E], CX* lds, int t, const CX* w1) {
  constexpr int B = E / R;
  CX u[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) u[b][r] = v[b + r * B];
    if constexpr (NS > 1) {
      CX wb = w1[b];
      if (INV) wb.y = -wb.y;
      CX w = wb;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        if (r > 1) w = cmul(w, wb);
        u[b][r] = cmul(u[b][r], w);
      }
    }
    dftR<R, INV>(u[b]);
  }
  if (LAST) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * B] = u[b][r];
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + T * b;
      const int k = j % NS;
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[padi(base + r * NS)] = u[b][r];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[padi(t + T * m)];
    __syncthreads();
  }
}

template <int N, bool INV, class CX, int E, int I>
__device__ __forceinline__ void fft_passes_w(CX (&v)[E], CX* lds, int t, const Tw1<N, E, CX>& tw1) {
  using PL = Plan<N, E>;
  constexpr int T = N / E;
  reg_pass_w<N, T, E, PL::R[I], PL::NS[I], INV, (I + 1 == PL::P)>(v, lds, t, tw1.w[I]);
  if constexpr (I + 1 < PL::P) fft_passes_w<N, INV, CX, E, I + 1>(v, lds, t, tw1);
}

// In-register FFT of N points, E per lane (T = N / E lanes), LDS exchanges
// between passes; FP64 with the twiddles of Tw1 (preloaded by the caller).
template <int N, bool INV, class CX, int E>
__device__ __forceinline__ void fft_reg_w(CX (&v)[E], CX* lds, int t, const Tw1<N, E, CX>& tw1) {
  fft_passes_w<N, INV, CX, E, 0>(v, lds, t, tw1);
}

// In-register FFT of N points, E per lane (T = N / E lanes), LDS exchanges
// between passes.  FP64: base twiddles loaded up front (Tw1); FP32 (the
// mixed-precision products, whose error budget assumes table twiddles): every
// power from the table, one pass ahead.
// Base twiddles up front (Tw1) for FP64 powers of two.  Tori with a factor 3
// or 5 hold 12 or 20 points per lane, too many registers to keep every
// pass's base twiddles live as well: they load one pass's base twiddles one
// pass ahead (BaseTw) and form the powers by products, as Tw1 does.
template <int N, class CX>
constexpr bool use_tw1() {
  return std::is_same<CX, double2>::value && (N & (N - 1)) == 0;
}

template <int N, int E, int I, class CX>
struct BaseTw {
  using PL = Plan<N, E>;
  static constexpr int R = PL::R[I], NS = PL::NS[I], B = E / R, T = N / E;
  CX w[B];
  __device__ __forceinline__ void load(int t, const CX* __restrict__ tw) {
    if constexpr (NS > 1) {
      constexpr int step = N / (NS * R);
#pragma unroll
      for (int b = 0; b < B; ++b) w[b] = tw[((t + T * b) % NS) * step];
    }
  }
};

template <int N, bool INV, class CX, int E, int I>
__device__ __forceinline__ void fft_passes_b(CX (&v)[E], CX* lds, int t, const CX* __restrict__ tw,
                                             const BaseTw<N, E, I, CX>& cur) {
  using PL = Plan<N, E>;
  constexpr int T = N / E;
  if constexpr (I + 1 < PL::P) {
    BaseTw<N, E, I + 1, CX> nxt;
    nxt.load(t, tw);   // the next pass's base twiddles, in flight during this pass
    reg_pass_w<N, T, E, PL::R[I], PL::NS[I], INV, false>(v, lds, t, cur.w);
    fft_passes_b<N, INV, CX, E, I + 1>(v, lds, t, tw, nxt);
  } else {
    reg_pass_w<N, T, E, PL::R[I], PL::NS[I], INV, true>(v, lds, t, cur.w);
  }
}

template <int N, bool INV, class CX, int E>
__device__ __forceinline__ void fft_reg(CX (&v)[E], CX* lds, int t, const CX* __restrict__ tw) {
  if constexpr (use_tw1<N, CX>()) {
    Tw1<N, E, CX> tw1;
    tw1.load(t, tw);
    fft_reg_w<N, INV, CX, E>(v, lds, t, tw1);
  } else if constexpr (std::is_same<CX, double2>::value) {
    BaseTw<N, E, 0, CX> first;   // the first pass has no twiddles
    fft_passes_b<N, INV, CX, E, 0>(v, lds, t, tw, first);
  } else {
    PlanTw<N, E, 0, CX> first;   // the first pass has no twiddles
    fft_passes<N, INV, CX, E, 0>(v, lds, t, tw, first);
  }
}

// ---- column pass: FFT, multiply by the kernel spectrum, inverse FFT; in/out rows pruned
// PADY: the torus is the zero-padded free-space one (rows at and past MY / 2
// carry no source); false: the unpadded periodic torus of the grid itself.
template <int MY, class CX, int PER, bool PADY>
__global__ void __launch_bounds__((RegCfg<MY, PER>::THREADS))
k_cols_reg(DGeom g, DFft f, bool dense, const double* __restrict__ gam, double sgn, int rj0, int rj1, int oj0,
           int oj1, const double* __restrict__ done) {
  using C = RegCfg<MY, PER>;
  using S = typename Real<CX>::t;
  const FftT<CX> ft = fft_view<CX>(f);
  constexpr int T = RP<MY>::T, E = RP<MY>::E;
  __shared__ CX lds[C::PER][C::LDSN];
  if (done && done[KS_DONE] != 0.0) return;
  const int w = threadIdx.x / T, t = threadIdx.x % T;
  const int kx = blockIdx.x * C::PER + w;
  const bool valid = kx <= f.hx;
  const CX* col = ft.spec + (size_t)(valid ? kx : 0) * f.ld;
  CX* out = ft.out + (size_t)(valid ? kx : 0) * f.ld;
  CX v[E];
  // rows at and past MY / 2 are the zero padding of every source on the
  // padded free-space torus (folded at compile time); the periodic torus is
  // the grid itself
  constexpr bool pad_y = PADY;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + T * m;
    const bool row_ok = pad_y ? (m < E / 2) : true;
    v[m] = (row_ok && valid && dense && n >= rj0 && n <= rj1) ? col[n + 1] : mkc<CX>(0, 0);
  }
  if (gam && f.corr) {
    // Correction sources from the pre-pass: this column's value of each
    // affected row (slot loads and value loads unconditional, at clamped
    // indices, and the value weighted by 0 or 1: under a per-lane branch
    // each would be waited for inside it)
    const CX* corr = reinterpret_cast<const CX*>(f.corr) + (size_t)(valid ? kx : 0) * g.n_corr_rows;
    const int jb = max(rj0, 0), je = min(rj1, g.ny - 1);
    int sl[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int n = t + T * m;
      const int q = g.row_slot[min(n, g.ny - 1)];
      sl[m] = ((!pad_y || m < E / 2) && n >= jb && n <= je) ? q : -1;   // padded: sources lie below MY / 2
    }
    CX cv[E];
#pragma unroll
    for (int m = 0; m < E; ++m) cv[m] = corr[max(sl[m], 0)];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const S w = sl[m] >= 0 ? (S)1 : (S)0;
      v[m] = mkc<CX>(v[m].x + w * cv[m].x, v[m].y + w * cv[m].y);
    }
  } else if (gam) {
    // Correction sources: the column's T lanes compute the terms
    // sgn gam[a_e] W^(kx i_e) of all entries e of rows [rj0, rj1] (a few per
    // lane, loads batched), stage them in this FFT's LDS buffer (free until
    // the FFT), and the lane owning a row sums the terms of its entries.
    // Entries are grouped by row, so a row's terms are contiguous; more
    // entries than the buffer holds are taken in chunks.  Every lane of the
    // block runs the same chunks (the bounds depend on rj0, rj1 only).
    // rows covering every affected row (all callers so far) take the whole
    // entry range without reading the row offsets
    const int jb = max(rj0, 0), je = min(rj1, g.ny - 1);
    const int eb = jb <= je ? (jb <= g.a_j0 ? 0 : g.row_ptr[jb]) : 0;
    const int ee = jb <= je ? (je >= g.a_j1 ? g.na : g.row_ptr[je + 1]) : 0;
    int rb[E], re[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int n = t + T * m;
      const bool in = (pad_y ? m < E / 2 : true) && n >= jb && n <= je;   // padded: sources lie below MY / 2
      rb[m] = in ? g.row_ptr[n] : 0;
      re[m] = in ? g.row_ptr[n + 1] : 0;
    }
    const int mx = f.mx;
    for (int c0 = eb; c0 < ee; c0 += C::LDSN) {
      const int c1 = min(ee, c0 + C::LDSN);
      for (int e0 = c0 + t; e0 < c1; e0 += 4 * T) {
        // every load unconditional, at a clamped index (lanes past c1 repeat
        // entry c1 - 1 and write nothing): a load under a per-lane branch,
        // or feeding a per-lane select, is waited for inside a branch, one
        // round trip per entry
        int2 ia[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ia[u] = g.row_ia[min(e0 + u * T, c1 - 1)];
        // twiddles and circulation values of the entries, all in flight
        // together; the mirror source's twiddle (outflow) is loaded on every
        // torus and weighted by 0 or 1, for the same reason
        CX w1[4], w2[4];
        double gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ii = ia[u].x;
          w1[u] = twiddle_r(ft.tw_xr, torus_mod(kx * ii, mx), mx);
          w2[u] = twiddle_r(ft.tw_xr, torus_mod(kx * (2 * g.nx - 1 - ii), mx), mx);
          gv[u] = gam[ia[u].y];
        }
        const S mir = f.outflow ? (S)1 : (S)0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (e0 + u * T >= c1) break;
          const S vv = (S)(sgn * gv[u]);
          lds[w][e0 + u * T - c0] = mkc<CX>(vv * (w1[u].x + mir * w2[u].x), vv * (w1[u].y + mir * w2[u].y));
        }
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) {
        if (!pad_y || m < E / 2) {   // padded: rows past MY / 2 carry no source
          const int q1 = min(re[m], c1);
          for (int q = max(rb[m], c0); q < q1; ++q) v[m] = cadd(v[m], lds[w][q - c0]);
        }
      }
      __syncthreads();
    }
  }
  // kernel spectrum of this thread's bins, loaded before the forward FFT
  const S* gh = ft.ghat + (size_t)(valid ? kx : 0) * (MY / 2 + 1);
  S gk[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + T * m;
    gk[m] = gh[n <= MY / 2 ? n : MY - n];
  }
  if constexpr (use_tw1<MY, CX>()) {
    Tw1<MY, E, CX> tw1;   // both FFTs' base twiddles
    tw1.load(t, ft.tw_y);
    fft_reg_w<MY, false>(v, lds[w], t, tw1);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      v[m].x *= gk[m];
      v[m].y *= gk[m];
    }
    fft_reg_w<MY, true>(v, lds[w], t, tw1);
  } else {
    fft_reg<MY, false>(v, lds[w], t, ft.tw_y);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      v[m].x *= gk[m];
      v[m].y *= gk[m];
    }
    fft_reg<MY, true>(v, lds[w], t, ft.tw_y);
  }
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int n = t + T * m;
      if (pad_y) {
        // ring row -1 is torus row MY - 1, ring row ny torus row ny
        const int jo = (n == MY - 1) ? -1 : n;
        if (jo >= oj0 && jo <= oj1) out[jo + 1] = v[m];
      } else {
        // the grid's own rows; the ring rows -1 and ny repeat rows ny - 1 and 0
        if (n >= oj0 && n <= oj1) out[n + 1] = v[m];
        if (n == MY - 1 && oj0 <= -1) out[0] = v[m];
        if (n == 0 && oj1 >= g.ny) out[g.ny + 1] = v[m];
      }
    }
  }
}

// ---- forward rows: real FFT of length 2 HX (half-length complex FFT + split)
// CORR = false: rows j0 .. j0 + count - 1 of the masked vorticity -> spec
// (row jj at slot jj + 1).  CORR = true: the correction sources sgn gam[a]
// placed at the affected points of the grid rows corr_rows[slot], slot <
// count (rows outside [j0, jb_end] carry none) -> f.corr[k][slot]: the
// row transforms that the column pass adds for those rows.  Both follow
// the same even mirror past the outflow plane.
template <int HX, class CX, int PER, bool CORR>
__device__ __forceinline__ void rows_fwd_body(const DGeom& g, const DFft& f, const double* __restrict__ omega,
                                              const double* __restrict__ gam, double sgn, int j0, int j1, int count) {
  using C = RegCfg<HX, PER, true>;
  using S = typename Real<CX>::t;
  const FftT<CX> ft = fft_view<CX>(f);
  constexpr int T = RPX<HX, true>::T, E = RPX<HX, true>::E;
  __shared__ CX lds[C::PER][C::LDSN];
  const int w = threadIdx.x / T, t = threadIdx.x % T;
  const int lb = xcd_block();
  const int r0 = lb * C::PER + w;   // this FFT's row (CORR: its slot)
  int jrow;
  bool valid;
  if constexpr (CORR) {
    jrow = r0 < count ? g.corr_rows[r0] : 0;
    valid = r0 < count && jrow >= j0 && jrow <= j1;
  } else {
    jrow = j0 + r0;
    valid = (r0 < count) && jrow >= 0 && jrow < g.ny;
  }
  CX v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + T * m;
    CX z = mkc<CX>(0, 0);
    if (valid) {
      const int i0 = 2 * n, i1 = 2 * n + 1;
      int m0 = i0, m1 = i1;
      if (f.outflow) {
        m0 = i0 < g.nx ? i0 : 2 * g.nx - 1 - i0;
        m1 = i1 < g.nx ? i1 : 2 * g.nx - 1 - i1;
      }
      const size_t rb = (size_t)jrow * g.nx;
      const bool in0 = m0 >= 0 && m0 < g.nx, in1 = m1 >= 0 && m1 < g.nx;
      if constexpr (CORR) {
        // the affected index of the node, then its circulation value (both
        // loads unconditional at valid addresses, the value weighted by 0 or 1)
        const int a0 = g.a_id[rb + (in0 ? m0 : 0)], a1 = g.a_id[rb + (in1 ? m1 : 0)];
        const double v0 = gam[max(a0, 0)], v1 = gam[max(a1, 0)];
        z.x = (S)(sgn * v0 * ((in0 && a0 >= 0) ? 1.0 : 0.0));
        z.y = (S)(sgn * v1 * ((in1 && a1 >= 0) ? 1.0 : 0.0));
      } else {
        // class and vorticity loaded together (both addresses are valid), then selected
        const int8_t c0 = in0 ? g.cls[rb + m0] : (int8_t)3, c1 = in1 ? g.cls[rb + m1] : (int8_t)3;
        const double o0 = in0 ? omega[rb + m0] : 0.0, o1 = in1 ? omega[rb + m1] : 0.0;
        z.x = c0 < 2 ? (S)o0 : (S)0;
        z.y = c1 < 2 ? (S)o1 : (S)0;
      }
    }
    v[m] = z;
  }
  fft_reg<HX, false>(v, lds[w], t, ft.tw_x);
#pragma unroll
  for (int m = 0; m < E; ++m) lds[w][padi(t + T * m)] = v[m];
  // split twiddles of this thread's bins, loaded before the barrier
  constexpr int IT = ((HX + 1) * C::PER + C::THREADS - 1) / C::THREADS;
  CX wk[IT];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int idx = threadIdx.x + q * C::THREADS;
    wk[q] = idx < (HX + 1) * C::PER ? ft.tw_xr[idx / C::PER] : mkc<CX>(1, 0);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int idx = threadIdx.x + q * C::THREADS;
    if (idx >= (HX + 1) * C::PER) break;
    const int rr = idx % C::PER, k = idx / C::PER;
    const int slot = lb * C::PER + rr;
    if constexpr (CORR) {
      if (slot >= count) continue;
    } else {
      const int jj = j0 + slot;
      if (slot >= count || jj < 0 || jj >= g.ny) continue;
    }
    const CX zk = lds[rr][padi(k == HX ? 0 : k)];
    const CX zc = conj2(lds[rr][padi(k == 0 ? 0 : HX - k)]);
    const CX E2 = mkc<CX>(S(0.5) * (zk.x + zc.x), S(0.5) * (zk.y + zc.y));
    const CX Od = csub(zk, zc);
    const CX O = mkc<CX>(S(0.5) * Od.y, S(-0.5) * Od.x);
    const CX val = cadd(E2, cmul(wk[q], O));
    if constexpr (CORR)
      reinterpret_cast<CX*>(f.corr)[(size_t)k * count + slot] = val;
    else
      ft.spec[(size_t)k * f.ld + j0 + slot + 1] = val;
  }
}

template <int HX, class CX, int PER>
__global__ void __launch_bounds__((RegCfg<HX, PER, true>::THREADS))
k_rows_fwd_reg(DGeom g, DFft f, const double* __restrict__ omega, int j0, int count,
               const double* __restrict__ done) {
  if (done && done[KS_DONE] != 0.0) return;
  rows_fwd_body<HX, CX, PER, false>(g, f, omega, nullptr, 0.0, j0, 0, count);
}

// the correction sources' row transforms of rows [jb, je] (slots 0 .. R - 1)
template <int HX, class CX, int PER>
__global__ void __launch_bounds__((RegCfg<HX, PER, true>::THREADS))
k_rows_fwd_corr(DGeom g, DFft f, const double* __restrict__ gam, double sgn, int jb, int je,
                const double* __restrict__ done) {
  if (done && done[KS_DONE] != 0.0) return;
  rows_fwd_body<HX, CX, PER, true>(g, f, nullptr, gam, sgn, jb, je, g.n_corr_rows);
}

// ---- inverse rows: complex-to-real of length 2 HX; rows jo in [j0, j0 + count) of the ring
template <int HX, class CX, int PER>
__global__ void __launch_bounds__((RegCfg<HX, PER, true>::THREADS))
k_rows_inv_reg(DGeom g, DFft f, int j0, int count, double* __restrict__ psi, const double* __restrict__ done) {
  using C = RegCfg<HX, PER, true>;
  const FftT<CX> ft = fft_view<CX>(f);
  constexpr int T = RPX<HX, true>::T, E = RPX<HX, true>::E;
  __shared__ CX lds[C::PER][C::LDSN];
  if (done && done[KS_DONE] != 0.0) return;
  const int lb = xcd_block();
  const int w = threadIdx.x / T, t = threadIdx.x % T;
  CX twk[E];                 // split twiddles of this thread's bins
  Tw1<HX, E, CX> tw1;        // the FFT's base twiddles (FP64 powers of two)
  {
    // all loads of this thread in flight before the LDS stores: the
    // spectrum, then the twiddles (which would otherwise be requested after
    // the barrier, one more round trip)
    constexpr int IT = ((HX + 1) * C::PER + C::THREADS - 1) / C::THREADS;
    CX tmp[IT];
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int idx = threadIdx.x + q * C::THREADS;
      const int rr = idx % C::PER, k = idx / C::PER;
      const int jo = j0 + lb * C::PER + rr;
      tmp[q] = (idx < (HX + 1) * C::PER && jo < j0 + count) ? ft.out[(size_t)k * f.ld + jo + 1]
                                                             : mkc<CX>(0, 0);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) twk[m] = conj2(ft.tw_xr[t + T * m]);
    if constexpr (use_tw1<HX, CX>()) tw1.load(t, ft.tw_x);
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int idx = threadIdx.x + q * C::THREADS;
      if (idx < (HX + 1) * C::PER) lds[idx % C::PER][padi(idx / C::PER)] = tmp[q];
    }
  }
  __syncthreads();
  CX v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const CX xk = lds[w][padi(k)];
    const CX xc = conj2(lds[w][padi(HX - k)]);
    const CX Ev = cadd(xk, xc);
    const CX Ov = cmul(csub(xk, xc), twk[m]);
    v[m] = mkc<CX>(Ev.x - Ov.y, Ev.y + Ov.x);
  }
  __syncthreads();
  if constexpr (use_tw1<HX, CX>())
    fft_reg_w<HX, true>(v, lds[w], t, tw1);
  else
    fft_reg<HX, true>(v, lds[w], t, ft.tw_x);
  const int jo = j0 + lb * C::PER + w;
  if (jo >= j0 + count) return;
  const int nxr = g.nx + 2;
  double* row = psi + (size_t)(jo + 1) * nxr;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + T * m;
    const int i0 = 2 * n, i1 = 2 * n + 1;
    if (i0 <= g.nx) row[i0 + 1] = v[m].x;
    if (i1 <= g.nx) row[i1 + 1] = v[m].y;
    if (i1 == 2 * HX - 1) row[0] = v[m].y;
    if (f.periodic && i0 == 0) row[g.nx + 1] = v[m].x;   // ring column nx repeats column 0
  }
}

template <int HX, class CX, int PER>
void rows_fwd_go(const DGeom& g, const DFft& f, const double* omega, int j0, int count, const double* done,
                 hipStream_t s, Prof* prof, double bytes) {
  using C = RegCfg<HX, PER, true>;
  const int blocks = (count + C::PER - 1) / C::PER;
  if (blocks > 0)
    IIM_LAUNCH(prof, KID_ROWS_FWD, bytes, k_rows_fwd_reg<HX IIM_COMMA CX IIM_COMMA PER>, blocks, C::THREADS, s, g, f,
               omega, j0, count, done);
}
template <int MY, class CX, int PER>
void cols_go(const DGeom& g, const DFft& f, bool dense, const double* gam, double sgn, int rj0, int rj1, int oj0,
             int oj1, const double* done, hipStream_t s, Prof* prof, double bytes) {
  using C = RegCfg<MY, PER>;
  const int blocks = (f.hx + 1 + C::PER - 1) / C::PER;
  if (f.periodic)
    IIM_LAUNCH(prof, KID_COLS, bytes, k_cols_reg<MY IIM_COMMA CX IIM_COMMA PER IIM_COMMA false>, blocks, C::THREADS, s,
               g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done);
  else
    IIM_LAUNCH(prof, KID_COLS, bytes, k_cols_reg<MY IIM_COMMA CX IIM_COMMA PER IIM_COMMA true>, blocks, C::THREADS, s,
               g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done);
}
template <int HX, class CX, int PER>
void rows_inv_go(const DGeom& g, const DFft& f, int j0, int count, double* psi, const double* done, hipStream_t s,
                 Prof* prof, double bytes) {
  using C = RegCfg<HX, PER, true>;
  const int blocks = (count + C::PER - 1) / C::PER;
  if (blocks > 0)
    IIM_LAUNCH(prof, KID_ROWS_INV, bytes, k_rows_inv_reg<HX IIM_COMMA CX IIM_COMMA PER>, blocks, C::THREADS, s, g, f,
               j0, count, psi, done);
}

// Dispatch on the tuned FFTs-per-block (FP64 only; the FP32 inner products
// keep the default shape).  0 or an unavailable value: the default.
#define IIM_PER_DISPATCH(N, CX, PER_RUNTIME, ROWS, GO, ...)                            \
  do {                                                                                 \
    constexpr int D_ = RegDef<N, ROWS>::PER;                                           \
    if constexpr (std::is_same<CX, double2>::value) {                                  \
      if ((PER_RUNTIME) == 1 && per_ok<N, 1, CX, ROWS>()) { GO<N, CX, 1>(__VA_ARGS__); break; } \
      if constexpr (per_ok<N, 2, CX, ROWS>())                                          \
        if ((PER_RUNTIME) == 2) { GO<N, CX, 2>(__VA_ARGS__); break; }                  \
      if constexpr (per_ok<N, 4, CX, ROWS>())                                          \
        if ((PER_RUNTIME) == 4) { GO<N, CX, 4>(__VA_ARGS__); break; }                  \
    }                                                                                  \
    GO<N, CX, D_>(__VA_ARGS__);                                                        \
  } while (0)

// The correction sources' row transforms (DFft::corr), for the column pass
// of a product with many affected points: a forward row pass over the rows
// holding affected points, with the sources placed at those points.
template <int HX, class CX>
void corr_rows_launch(const DGeom& g, const DFft& f, const double* gam, double sgn, int rj0, int rj1,
                      const double* done, hipStream_t s) {
  constexpr int PER = RegDef<HX, true>::PER;
  using C = RegCfg<HX, PER, true>;
  const int blocks = (g.n_corr_rows + C::PER - 1) / C::PER;
  if (blocks > 0)
    k_rows_fwd_corr<HX, CX, PER><<<blocks, C::THREADS, 0, s>>>(g, f, gam, sgn, max(rj0, 0), min(rj1, g.ny - 1),
                                                                done);
}

// Fewer rows than the chip has compute units (the band a product's
// right-hand side reads): one row per workgroup whatever the tuned shape,
// so that the rows spread over as many CUs as possible.
constexpr int ROWS_FEW = 256;
template <int HX, class CX>
void rows_fwd_reg_launch(const DGeom& g, const DFft& f, const double* omega, int j0, int count, const double* done,
                         hipStream_t s, Prof* prof, double bytes) {
  IIM_PER_DISPATCH(HX, CX, count < ROWS_FEW ? 1 : f.row_per, true, rows_fwd_go, g, f, omega, j0, count, done, s,
                   prof, bytes);
}
template <int MY, class CX>
void cols_reg_launch(const DGeom& g, const DFft& f, bool dense, const double* gam, double sgn, int rj0, int rj1,
                     int oj0, int oj1, const double* done, hipStream_t s, Prof* prof, double bytes) {
  IIM_PER_DISPATCH(MY, CX, f.col_per, false, cols_go, g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done, s, prof,
                   bytes);
}
template <int HX, class CX>
void rows_inv_reg_launch(const DGeom& g, const DFft& f, int j0, int count, double* psi, const double* done,
                         hipStream_t s, Prof* prof, double bytes) {
  IIM_PER_DISPATCH(HX, CX, count < ROWS_FEW ? 1 : f.row_per, true, rows_inv_go, g, f, j0, count, psi, done, s, prof,
                   bytes);
}

// Register FFT sizes: powers of two 256 .. 4096 (FP64 and FP32) and, FP64
// only, 320, 384, 640, 768, 1280, 1536 (factors 3 and 5)
#define IIM_REG_SWITCH(VAL, FN, CXT, ...)                                              \
  switch (VAL) {                                                                       \
    case 256: FN<256, CXT>(__VA_ARGS__); break;                                        \
    case 512: FN<512, CXT>(__VA_ARGS__); break;                                        \
    case 1024: FN<1024, CXT>(__VA_ARGS__); break;                                      \
    case 2048: FN<2048, CXT>(__VA_ARGS__); break;                                      \
    case 4096: FN<4096, CXT>(__VA_ARGS__); break;                                      \
    default:                                                                           \
      if constexpr (std::is_same<CXT, double2>::value) {                               \
        switch (VAL) {                                                                 \
          case 320: FN<320, CXT>(__VA_ARGS__); break;                                  \
          case 384: FN<384, CXT>(__VA_ARGS__); break;                                  \
          case 640: FN<640, CXT>(__VA_ARGS__); break;                                  \
          case 768: FN<768, CXT>(__VA_ARGS__); break;                                  \
          case 1280: FN<1280, CXT>(__VA_ARGS__); break;                                \
          case 1536: FN<1536, CXT>(__VA_ARGS__); break;                                \
          default: break;                                                              \
        }                                                                              \
      }                                                                                \
      break;                                                                           \
  }

bool reg_fft_size(int n, bool fp32) {
  switch (n) {
    case 256: case 512: case 1024: case 2048: case 4096: return true;
    case 320: case 384: case 640: case 768: case 1280: case 1536: return !fp32;
    default: return false;
  }
}
bool conv_reg_supported(int hx, int my) { return hx >= 256 && my >= 256; }

// ---- launch-resource check of the register FFT instantiations that a tile
// shape selects: the block must fit the kernel's register-limited thread
// count, its LDS the device's per-block limit, and it must use no scratch
// memory.  A launch that fails these is refused by the runtime, so the
// autotuner and the set-up check them before any shape is used.
struct FitCheck {
  int max_lds = 0;
  bool ok = true;
  std::string why;
  void add(const void* fn, int threads, const char* what) {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) {
      ok = false;
      why += std::string(what) + ": attributes unavailable; ";
      return;
    }
    if (a.maxThreadsPerBlock < threads || (int)a.sharedSizeBytes > max_lds || a.localSizeBytes > 0) {
      ok = false;
      why += std::string(what) + ": " + std::to_string(threads) + " threads (max " +
             std::to_string(a.maxThreadsPerBlock) + "), " + std::to_string(a.sharedSizeBytes) + " B LDS (max " +
             std::to_string(max_lds) + "), " + std::to_string(a.localSizeBytes) + " B scratch; ";
    }
  }
};
template <int HX, class CX, int PER>
void rows_fwd_fit(FitCheck& fc) {
  fc.add((const void*)k_rows_fwd_reg<HX, CX, PER>, RegCfg<HX, PER, true>::THREADS, "row pass");
}
template <int MY, class CX, int PER>
void cols_fit(FitCheck& fc) {
  fc.add((const void*)k_cols_reg<MY, CX, PER, true>, RegCfg<MY, PER>::THREADS, "column pass");
  fc.add((const void*)k_cols_reg<MY, CX, PER, false>, RegCfg<MY, PER>::THREADS, "column pass (periodic)");
}
template <int HX, class CX, int PER>
void rows_inv_fit(FitCheck& fc) {
  fc.add((const void*)k_rows_inv_reg<HX, CX, PER>, RegCfg<HX, PER, true>::THREADS, "inverse row pass");
}
template <int HX, class CX>
void rows_fit_sw(const DFft& f, FitCheck& fc) {
  IIM_PER_DISPATCH(HX, CX, f.row_per, true, rows_fwd_fit, fc);
  IIM_PER_DISPATCH(HX, CX, f.row_per, true, rows_inv_fit, fc);
}
template <int MY, class CX>
void cols_fit_sw(const DFft& f, FitCheck& fc) {
  IIM_PER_DISPATCH(MY, CX, f.col_per, false, cols_fit, fc);
}

bool reg_shapes_fit(const DFft& f, bool fp32, std::string* why) {
  if (!conv_reg_supported(f.hx, f.my)) return true;
  FitCheck fc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&fc.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    if (why) *why = "device attributes unavailable";
    return false;
  }
  if (fp32) {
    IIM_REG_SWITCH(f.hx, rows_fit_sw, float2, f, fc);
    IIM_REG_SWITCH(f.my, cols_fit_sw, float2, f, fc);
  } else {
    IIM_REG_SWITCH(f.hx, rows_fit_sw, double2, f, fc);
    IIM_REG_SWITCH(f.my, cols_fit_sw, double2, f, fc);
  }
  if (why) *why = fc.why;
  return fc.ok;
}

void launch_conv_reg(const DGeom& g, const DFft& f, const double* omega, const double* gam, double sgn, int rj0,
                     int rj1, int oj0, int oj1, double* psi_ring, const double* done, hipStream_t s, Prof* prof,
                     bool fp32, bool rows_ready) {
  const int nin = rj1 - rj0 + 1, nout = oj1 - oj0 + 1;
  const bool dense = omega != nullptr, rows = dense && !rows_ready;
  // algorithmic bytes: source rows read (omega) + half spectrum written;
  // spectrum rows in (dense source) + kernel spectrum + rows out; half
  // spectrum in + ring rows out
  const double cb = fp32 ? 8.0 : 16.0, rb = fp32 ? 4.0 : 8.0;
  const double b_fwd = (double)nin * (8.0 * g.nx + cb * (f.hx + 1));
  // (with the correction pre-pass the column pass also reads its rows)
  const double b_col = (double)(f.hx + 1) * ((dense ? cb * nin : 0.0) + rb * (f.my / 2 + 1) + cb * nout +
                                             ((gam && f.corr) ? cb * g.n_corr_rows : 0.0));
  const double b_inv = (double)nout * (cb * (f.hx + 1) + 8.0 * (g.nx + 2));
  if (fp32) {
    if (rows) IIM_REG_SWITCH(f.hx, rows_fwd_reg_launch, float2, g, f, omega, rj0, nin, done, s, prof, b_fwd);
    if (gam && f.corr) IIM_REG_SWITCH(f.hx, corr_rows_launch, float2, g, f, gam, sgn, rj0, rj1, done, s);
    IIM_REG_SWITCH(f.my, cols_reg_launch, float2, g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done, s, prof, b_col);
    IIM_REG_SWITCH(f.hx, rows_inv_reg_launch, float2, g, f, oj0, nout, psi_ring, done, s, prof, b_inv);
  } else {
    if (rows) IIM_REG_SWITCH(f.hx, rows_fwd_reg_launch, double2, g, f, omega, rj0, nin, done, s, prof, b_fwd);
    if (gam && f.corr) IIM_REG_SWITCH(f.hx, corr_rows_launch, double2, g, f, gam, sgn, rj0, rj1, done, s);
    IIM_REG_SWITCH(f.my, cols_reg_launch, double2, g, f, dense, gam, sgn, rj0, rj1, oj0, oj1, done, s, prof, b_col);
    IIM_REG_SWITCH(f.hx, rows_inv_reg_launch, double2, g, f, oj0, nout, psi_ring, done, s, prof, b_inv);
  }
}

}  // namespace iim
