// Lattice Green's function of the 5-point Laplacian (free-space exact
// inverse used by the FFT solution operator of Sec. 4.2).
//
// g(m, n) = -A(m, n) with the potential kernel
//   A(m, n) = (2 pi)^-2 iint (1 - cos(m a + n b)) / (4 - 2 cos a - 2 cos b) da db
// so that -(discrete Laplacian of g) = delta and g(0, 0) = 0.  Integrating in
// b analytically leaves a one-dimensional integral over a in [0, pi]:
//   A(m, n) = 1/(2 pi) int_0^pi (1 - exp(-K t) cos(k a)) / sinh t da,
//   cosh t = 2 - cos a,  K = max(|m|,|n|), k = min(|m|,|n|).
// With u = sin(a/2): t = 2 asinh(u), sinh t = 2 u sqrt(1 + u^2).  The
// integrand is smooth but varies on the scale 1/K near a = 0, so the interval
// is split into panels growing geometrically from 1/(2K); each panel uses
// 32-point Gauss-Legendre quadrature.
#include <cmath>
#include <thread>
#include <vector>

#include "iim_host.hpp"

namespace iim {
namespace {

struct GL {
  std::vector<double> x, w;
  explicit GL(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        double dp = n * (z * p0 - p1) / (z * z - 1.0);
        double dz = p0 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) {
          // recompute derivative at the converged node
          p0 = 1.0; p1 = 0.0;
          for (int k = 1; k <= n; ++k) {
            double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
          }
          dp = n * (z * p0 - p1) / (z * z - 1.0);
          w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
          break;
        }
      }
      x[i] = z;
    }
  }
};

// A(K, k) for a fixed K and all k in [0, kmax]
void potential_row(int K, int kmax, const GL& gl, double* out) {
  for (int k = 0; k <= kmax; ++k) out[k] = 0.0;
  if (K == 0) return;
  std::vector<double> edges;
  edges.push_back(0.0);
  for (double e = 0.5 / K; e < M_PI; e *= 2.0) edges.push_back(e);
  edges.push_back(M_PI);
  const int n = (int)gl.x.size();
  double base_sum = 0.0;
  for (size_t p = 0; p + 1 < edges.size(); ++p) {
    const double a = edges[p], b = edges[p + 1];
    const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    for (int q = 0; q < n; ++q) {
      const double th = mid + half * gl.x[q];
      const double u = std::sin(0.5 * th);
      const double t = 2.0 * std::asinh(u);
      const double sinh_t = 2.0 * u * std::sqrt(1.0 + u * u);
      const double e = std::exp(-K * t);
      const double base = -std::expm1(-K * t);
      const double wq = half * gl.w[q] / sinh_t;
      // 1 - exp(-K t) cos(k th) = base + 2 e sin^2(k th / 2)
      base_sum += wq * base;
      if (e * wq < 1e-30) continue;
      for (int k = 0; k <= kmax; ++k) {
        const double sk = std::sin(0.5 * k * th);
        out[k] += 2.0 * wq * e * sk * sk;
      }
    }
  }
  for (int k = 0; k <= kmax; ++k) out[k] = (out[k] + base_sum) * (1.0 / (2.0 * M_PI));
}

}  // namespace

void lgf_table(int mx, int my, double* out, int threads) {
  const GL gl(32);
  const int Kmax = mx > my ? mx : my;
  if (threads <= 0) {
    threads = (int)std::thread::hardware_concurrency();
    if (threads <= 0) threads = 1;
    if (threads > 16) threads = 16;
  }
  auto work = [&](int tid) {
    std::vector<double> row(Kmax + 1);
    for (int K = tid; K <= Kmax; K += threads) {
      int kmax = -1;
      if (K <= mx) kmax = std::max(kmax, std::min(K, my));
      if (K <= my) kmax = std::max(kmax, std::min(K, mx));
      if (kmax < 0) continue;
      potential_row(K, kmax, gl, row.data());
      // entries whose larger index is K: (m, n) = (K, k) and (k, K)
      if (K <= mx)
        for (int k = 0; k <= std::min(K, my); ++k) out[(size_t)k * (mx + 1) + K] = -row[k];
      if (K <= my)
        for (int k = 0; k <= std::min(K, mx); ++k) out[(size_t)K * (mx + 1) + k] = -row[k];
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) pool.emplace_back(work, t);
  for (auto& th : pool) th.join();
}

void lgf_spectrum(int mx, int my, double h, const double* table, int tab_mx, double* out) {
  // K(i, j) = h^2 g(min(i, mx-i), min(j, my-j)) is real and even in both
  // directions; its DFT is real:  sum_i sum_j K cos(2 pi kx i / mx) cos(2 pi ky j / my).
  // The kernel grows like log r, so the high-frequency coefficients are small
  // differences of large sums: both cosine sums accumulate in 80-bit long
  // double, which keeps the result accurate to double rounding.
  typedef long double LD;
  const int hx = mx / 2, hy = my / 2;
  const LD two_pi = 6.283185307179586476925286766559005768L;
  std::vector<LD> cx(mx), cy(my);
  for (int i = 0; i < mx; ++i) cx[i] = std::cos(two_pi * (LD)i / (LD)mx);
  for (int j = 0; j < my; ++j) cy[j] = std::cos(two_pi * (LD)j / (LD)my);
  // first along x: C1[j][kx] for j in [0, hy]
  std::vector<LD> C1((size_t)(hy + 1) * (hx + 1));
  int threads = (int)std::thread::hardware_concurrency();
  if (threads <= 0) threads = 1;
  if (threads > 16) threads = 16;
  const LD h2 = (LD)h * (LD)h;
  auto kern = [&](int i, int j) { return h2 * (LD)table[(size_t)j * (tab_mx + 1) + i]; };
  auto passx = [&](int tid) {
    for (int j = tid; j <= hy; j += threads)
      for (int kx = 0; kx <= hx; ++kx) {
        LD acc = 0.0L;
        for (int i = 1; i < hx; ++i) acc += kern(i, j) * cx[((size_t)kx * i) % mx];
        C1[(size_t)j * (hx + 1) + kx] = kern(0, j) + ((kx & 1) ? -1.0L : 1.0L) * kern(hx, j) + 2.0L * acc;
      }
  };
  {
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) pool.emplace_back(passx, t);
    for (auto& th : pool) th.join();
  }
  const LD scale = 1.0L / ((LD)mx * (LD)my);
  auto passy = [&](int tid) {
    for (int kx = tid; kx <= hx; kx += threads)
      for (int ky = 0; ky <= hy; ++ky) {
        LD acc = 0.0L;
        for (int j = 1; j < hy; ++j) acc += C1[(size_t)j * (hx + 1) + kx] * cy[((size_t)ky * j) % my];
        const LD v = C1[kx] + ((ky & 1) ? -1.0L : 1.0L) * C1[(size_t)hy * (hx + 1) + kx] + 2.0L * acc;
        out[(size_t)kx * (hy + 1) + ky] = (double)(v * scale);
      }
  };
  {
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) pool.emplace_back(passy, t);
    for (auto& th : pool) th.join();
  }
}

}  // namespace iim
