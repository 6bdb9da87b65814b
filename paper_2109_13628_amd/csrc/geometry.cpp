// Host geometry of the immersed interface method (Sec. 2.1-2.2, App. A).
//
// Bodies arrive as closed point sets; each becomes the periodic cubic spline
// through its points (uniform parameter).  Its crossings with the grid lines
// give the control points; node classes follow from crossing parity along
// both axes.  The affected points A+ (fluid) / A- (solid, "ghosts") are the
// nodes adjacent to a control point.  A ghost value is the mean over valid
// directions of a one-dimensional Lagrange extrapolation along the grid line
// through the control point, evaluated one node past the boundary; stencils
// that use the boundary value leave out the fluid node next to it (Sec. 2.1).
//
// Tables built here (all read by the device kernels):
//   ext4b  cubic through {c, x_i-1, x_i-2, x_i-3}      (psi ghosts, omega for diffusion)
//   ext3b  quadratic through {c, x_i-1, x_i-2}         (velocity, omega upwind end)
//   ext3n  quadratic through {x_i, x_i-1, x_i-2}       (omega downwind end, no boundary value)
//   aop    gamma = A psi + B psi_b (Sec. 4.2): A+ rows -h^-2 sum of solid-neighbour ghosts,
//          A- rows +h^-2 sum of fluid neighbours
//   wbc    boundary vorticity stencil (Sec. 5.3)
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <numeric>
#include <tuple>

#include "iim_host.hpp"

namespace iim {
namespace {

struct Spline {
  // X(k + s) = a + b s + c s^2 + d s^3, per segment k and coordinate
  std::vector<double> a[2], b[2], c[2], d[2];
  int P = 0;
};

// periodic cubic spline: second derivatives from the cyclic system
// M_{k-1} + 4 M_k + M_{k+1} = 6 (Q_{k+1} - 2 Q_k + Q_{k-1}), solved with the
// Sherman-Morrison correction of a tridiagonal Thomas sweep.
void solve_cyclic_141(const std::vector<double>& rhs, std::vector<double>& x) {
  const int n = (int)rhs.size();
  // A = T + u v^T with T tridiag(1, 4, 1) modified in the corners
  const double gamma = -4.0;
  std::vector<double> diag(n, 4.0), cp(n), z(n), y(n), u(n, 0.0);
  diag[0] = 4.0 - gamma;
  diag[n - 1] = 4.0 - 1.0 * 1.0 / gamma;
  u[0] = gamma;
  u[n - 1] = 1.0;
  auto thomas = [&](const std::vector<double>& r, std::vector<double>& out) {
    std::vector<double> dd(n), rr(n);
    dd[0] = diag[0];
    rr[0] = r[0];
    for (int i = 1; i < n; ++i) {
      double m = 1.0 / dd[i - 1];
      dd[i] = diag[i] - m;
      rr[i] = r[i] - m * rr[i - 1];
    }
    out[n - 1] = rr[n - 1] / dd[n - 1];
    for (int i = n - 2; i >= 0; --i) out[i] = (rr[i] - out[i + 1]) / dd[i];
  };
  thomas(rhs, y);
  thomas(u, z);
  // v = (1, 0, ..., 0, 1/gamma)
  double vy = y[0] + y[n - 1] / gamma;
  double vz = z[0] + z[n - 1] / gamma;
  double f = vy / (1.0 + vz);
  x.resize(n);
  for (int i = 0; i < n; ++i) x[i] = y[i] - f * z[i];
}

Spline make_spline(const std::vector<double>& xy) {
  Spline s;
  const int P = (int)xy.size() / 2;
  s.P = P;
  for (int ax = 0; ax < 2; ++ax) {
    std::vector<double> Q(P), rhs(P), M;
    for (int k = 0; k < P; ++k) Q[k] = xy[2 * k + ax];
    for (int k = 0; k < P; ++k) rhs[k] = 6.0 * (Q[(k + 1) % P] - 2.0 * Q[k] + Q[(k + P - 1) % P]);
    solve_cyclic_141(rhs, M);
    s.a[ax].resize(P);
    s.b[ax].resize(P);
    s.c[ax].resize(P);
    s.d[ax].resize(P);
    for (int k = 0; k < P; ++k) {
      const int k1 = (k + 1) % P;
      s.a[ax][k] = Q[k];
      s.b[ax][k] = (Q[k1] - Q[k]) - (2.0 * M[k] + M[k1]) / 6.0;
      s.c[ax][k] = 0.5 * M[k];
      s.d[ax][k] = (M[k1] - M[k]) / 6.0;
    }
  }
  return s;
}

inline double ev(const Spline& s, int ax, int k, double t) {
  return s.a[ax][k] + t * (s.b[ax][k] + t * (s.c[ax][k] + t * s.d[ax][k]));
}
inline double evd(const Spline& s, int ax, int k, double t) {
  return s.b[ax][k] + t * (2.0 * s.c[ax][k] + 3.0 * t * s.d[ax][k]);
}

struct Cross {
  int body;
  int seg;        // spline segment and parameter t in (0, 1) of the crossing
  double t;
  int line;       // line index
  double along;   // coordinate along the line
  double px, py;  // point
  double nx, ny;  // unit normal (fluid side = right of travel)
};

// Roots of X_ax(k + t) = level on (0, 1), for every level in `levels` (sorted).
void spline_crossings(const Spline& s, int body, int ax, const std::vector<double>& levels,
                      std::vector<std::vector<Cross>>& per_line) {
  const int P = s.P;
  for (int k = 0; k < P; ++k) {
    const double A = s.a[ax][k], B = s.b[ax][k], C = s.c[ax][k], D = s.d[ax][k];
    // critical points: 3 D t^2 + 2 C t + B = 0 on (0, 1)
    double crit[2];
    int ncrit = 0;
    const double qa = 3.0 * D, qb = 2.0 * C, qc = B;
    if (qa != 0.0) {
      double disc = qb * qb - 4.0 * qa * qc;
      if (disc >= 0.0) {
        double sq = std::sqrt(disc);
        // numerically stable quadratic roots
        double q = -0.5 * (qb + (qb >= 0 ? sq : -sq));
        double r1 = q / qa, r2 = (q != 0.0) ? qc / q : r1;
        if (r1 > r2) std::swap(r1, r2);
        if (r1 > 0.0 && r1 < 1.0) crit[ncrit++] = r1;
        if (r2 > 0.0 && r2 < 1.0 && !(ncrit && r2 == crit[0])) crit[ncrit++] = r2;
      }
    } else if (qb != 0.0) {
      double r = -qc / qb;
      if (r > 0.0 && r < 1.0) crit[ncrit++] = r;
    }
    double knots[4];
    int nk = 0;
    knots[nk++] = 0.0;
    for (int q = 0; q < ncrit; ++q) knots[nk++] = crit[q];
    knots[nk++] = 1.0;
    for (int p = 0; p + 1 < nk; ++p) {
      const double ta = knots[p], tb = knots[p + 1];
      const double ya = ev(s, ax, k, ta), yb = ev(s, ax, k, tb);
      const double lo = std::min(ya, yb), hi = std::max(ya, yb);
      auto it0 = std::lower_bound(levels.begin(), levels.end(), lo);
      auto it1 = std::upper_bound(levels.begin(), levels.end(), hi);
      for (auto it = it0; it != it1; ++it) {
        const double Y = *it;
        const int L = (int)(it - levels.begin());
        const double fa = ya - Y, fb = yb - Y;
        if (fa == 0.0 || fb == 0.0)
          throw GeomError("body " + std::to_string(body) + ": boundary curve touches grid line " +
                          std::to_string(L) + " exactly");
        if ((fa < 0) == (fb < 0)) continue;
        // safeguarded Newton on [ta, tb] (monotone there)
        double l = ta, r = tb, t = 0.5 * (ta + tb);
        const bool inc = fb > fa;
        for (int it2 = 0; it2 < 200; ++it2) {
          const double f = ev(s, ax, k, t) - Y;
          if (f == 0.0) { l = r = t; break; }
          if ((f > 0) == inc) r = t; else l = t;
          const double df = evd(s, ax, k, t);
          double tn = (df != 0.0) ? t - f / df : 0.5 * (l + r);
          if (!(tn > l && tn < r)) tn = 0.5 * (l + r);
          if (r - l <= 4e-16 || tn == t) { t = tn; break; }
          t = tn;
        }
        if (t < 1e-12 || t > 1.0 - 1e-12)
          throw GeomError("body " + std::to_string(body) + ": a boundary point lies on a grid line");
        for (int q = 0; q < ncrit; ++q)
          if (std::fabs(t - crit[q]) < 1e-9)
            throw GeomError("body " + std::to_string(body) + ": boundary tangent to a grid line");
        Cross c;
        c.body = body;
        c.seg = k;
        c.t = t;
        c.line = L;
        c.px = ev(s, 0, k, t);
        c.py = ev(s, 1, k, t);
        c.along = ax == 1 ? c.px : c.py;
        const double tx = evd(s, 0, k, t), ty = evd(s, 1, k, t);
        const double nn = std::hypot(tx, ty);
        c.nx = ty / nn;
        c.ny = -tx / nn;
        per_line[L].push_back(c);
      }
    }
  }
}

void lagrange_at(const double* nodes, int n, double x, double* w) {
  for (int k = 0; k < n; ++k) {
    double p = 1.0;
    for (int l = 0; l < n; ++l)
      if (l != k) p *= (x - nodes[l]) / (nodes[k] - nodes[l]);
    w[k] = p;
  }
}

void lagrange_deriv_at(const double* nodes, int n, double x, double* w) {
  for (int k = 0; k < n; ++k) {
    double den = 1.0;
    for (int l = 0; l < n; ++l)
      if (l != k) den *= nodes[k] - nodes[l];
    double tot = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == k) continue;
      double p = 1.0;
      for (int l = 0; l < n; ++l)
        if (l != k && l != m) p *= x - nodes[l];
      tot += p;
    }
    w[k] = tot / den;
  }
}

std::string node_str(int i, int j) { return "(" + std::to_string(i) + ", " + std::to_string(j) + ")"; }

}  // namespace

void build_geometry(Geometry& g, const GridSpec& grid, const std::vector<BodySpec>& bodies) {
  g = Geometry();
  g.grid = grid;
  g.bodies = bodies;
  const int nx = grid.nx, ny = grid.ny;
  const double h = grid.h;
  if (nx < 16 || ny < 16 || !(h > 0)) throw ArgError("grid must be at least 16 x 16 with h > 0");
  std::vector<double> xs(nx), ys(ny);
  for (int i = 0; i < nx; ++i) xs[i] = grid.x0 + h * i;
  for (int j = 0; j < ny; ++j) ys[j] = grid.y0 + h * j;
  const int nb = (int)bodies.size();
  int n_encl = 0;
  for (auto& b : bodies) n_encl += b.enclosure ? 1 : 0;
  if (n_encl > 1) throw ArgError("at most one enclosing wall");

  // per-body crossings and inside masks
  std::vector<uint8_t> solid((size_t)nx * ny, 0);
  std::vector<int> owner((size_t)nx * ny, -1);
  std::vector<std::vector<Cross>> hline(ny), vline(nx);  // all bodies
  for (int k = 0; k < nb; ++k) {
    const auto& b = bodies[k];
    const int P = (int)b.xy.size() / 2;
    if (P < 4) throw ArgError("body " + std::to_string(k) + ": needs at least 4 boundary points");
    double area = 0, xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int p = 0; p < P; ++p) {
      const int q = (p + 1) % P;
      area += 0.5 * (b.xy[2 * p] * b.xy[2 * q + 1] - b.xy[2 * q] * b.xy[2 * p + 1]);
      xmin = std::min(xmin, b.xy[2 * p]);
      xmax = std::max(xmax, b.xy[2 * p]);
      ymin = std::min(ymin, b.xy[2 * p + 1]);
      ymax = std::max(ymax, b.xy[2 * p + 1]);
    }
    if (b.enclosure && area >= 0)
      throw GeomError("body " + std::to_string(k) + ": an enclosing wall must be ordered clockwise");
    if (!b.enclosure && area <= 0)
      throw GeomError("body " + std::to_string(k) + ": an obstacle must be ordered counter-clockwise");
    const double margin = 3 * h;
    if (xmin < xs[0] + margin || xmax > xs[nx - 1] - margin || ymin < ys[0] + margin ||
        ymax > ys[ny - 1] - margin)
      throw GeomError("body " + std::to_string(k) + " is too close to the grid edge");
    Spline sp = make_spline(b.xy);
    std::vector<std::vector<Cross>> hk(ny), vk(nx);
    spline_crossings(sp, k, 1, ys, hk);  // horizontal lines y = y_j
    spline_crossings(sp, k, 0, xs, vk);  // vertical lines x = x_i
    std::vector<uint8_t> in_h((size_t)nx * ny, 0), in_v((size_t)nx * ny, 0);
    for (int j = 0; j < ny; ++j) {
      std::vector<double> pos;
      for (auto& c : hk[j]) pos.push_back(c.along);
      std::sort(pos.begin(), pos.end());
      for (int i = 0; i < nx; ++i) {
        auto it = std::lower_bound(pos.begin(), pos.end(), xs[i]);
        if (it != pos.end() && *it == xs[i])
          throw GeomError("body " + std::to_string(k) + ": node " + node_str(i, j) + " lies on the boundary");
        in_h[(size_t)j * nx + i] = ((it - pos.begin()) % 2) == 1;
      }
    }
    for (int i = 0; i < nx; ++i) {
      std::vector<double> pos;
      for (auto& c : vk[i]) pos.push_back(c.along);
      std::sort(pos.begin(), pos.end());
      for (int j = 0; j < ny; ++j) {
        auto it = std::lower_bound(pos.begin(), pos.end(), ys[j]);
        if (it != pos.end() && *it == ys[j])
          throw GeomError("body " + std::to_string(k) + ": node " + node_str(i, j) + " lies on the boundary");
        in_v[(size_t)j * nx + i] = ((it - pos.begin()) % 2) == 1;
      }
    }
    for (size_t q = 0; q < in_h.size(); ++q)
      if (in_h[q] != in_v[q])
        throw GeomError("body " + std::to_string(k) + ": horizontal and vertical classification disagree at " +
                        node_str((int)(q % nx), (int)(q / nx)));
    for (size_t q = 0; q < in_h.size(); ++q) {
      const bool reg = b.enclosure ? !in_h[q] : (bool)in_h[q];
      if (!reg) continue;
      if (solid[q]) throw GeomError("body " + std::to_string(k) + " overlaps another body");
      solid[q] = 1;
      owner[q] = k;
    }
    for (int j = 0; j < ny; ++j) hline[j].insert(hline[j].end(), hk[j].begin(), hk[j].end());
    for (int i = 0; i < nx; ++i) vline[i].insert(vline[i].end(), vk[i].begin(), vk[i].end());
  }
  auto is_solid = [&](int i, int j) { return solid[(size_t)j * nx + i] != 0; };

  // ---- control points
  struct CRec {
    long key0;
    int axis, sigma, i_f, j_f, body, seg;
    double theta, x, y, nx, ny, t;
  };
  std::vector<CRec> recs;
  auto scan_line = [&](int axis, int L, std::vector<Cross>& cl) {
    // axis 0: horizontal line j = L, nodes along x; axis 1: vertical line i = L
    std::sort(cl.begin(), cl.end(), [](const Cross& a, const Cross& b) { return a.along < b.along; });
    const int n_along = axis == 0 ? nx : ny;
    const std::vector<double>& nodes = axis == 0 ? xs : ys;
    for (int a = 0; a + 1 < n_along; ++a) {
      const bool s0 = axis == 0 ? is_solid(a, L) : is_solid(L, a);
      const bool s1 = axis == 0 ? is_solid(a + 1, L) : is_solid(L, a + 1);
      if (s0 == s1) continue;
      const double lo = nodes[a], hi = nodes[a + 1];
      std::vector<const Cross*> cand;
      for (auto& c : cl)
        if (c.along > lo && c.along < hi) cand.push_back(&c);
      if (cand.size() % 2 == 0)
        throw GeomError("inconsistent crossings on a fluid-solid edge near " +
                        (axis == 0 ? node_str(a, L) : node_str(L, a)));
      for (auto* c : cand)
        if (c->body != cand[0]->body) throw GeomError("two bodies cross the same grid edge");
      const Cross* best;
      int f_idx, sigma;
      double theta;
      if (!s0) {  // fluid at a, ghost at a+1: nearest crossing to lo
        best = cand.front();
        f_idx = a;
        sigma = 1;
        theta = (best->along - lo) / h;
      } else {    // fluid at a+1, ghost at a
        best = cand.back();
        f_idx = a + 1;
        sigma = -1;
        theta = (hi - best->along) / h;
      }
      CRec r;
      r.axis = axis;
      r.sigma = sigma;
      r.i_f = axis == 0 ? f_idx : L;
      r.j_f = axis == 0 ? L : f_idx;
      r.body = best->body;
      r.seg = best->seg;
      r.t = best->t;
      r.theta = theta;
      r.x = best->px;
      r.y = best->py;
      r.nx = best->nx;
      r.ny = best->ny;
      const int gi = axis == 0 ? r.i_f + sigma : r.i_f;
      const int gj = axis == 0 ? r.j_f : r.j_f + sigma;
      r.key0 = (long)gj * nx + gi;
      recs.push_back(r);
    }
  };
  for (int j = 0; j < ny; ++j) scan_line(0, j, hline[j]);
  for (int i = 0; i < nx; ++i) scan_line(1, i, vline[i]);
  std::sort(recs.begin(), recs.end(), [](const CRec& a, const CRec& b) {
    return std::tie(a.key0, a.axis, a.sigma) < std::tie(b.key0, b.axis, b.sigma);
  });
  const int nc = (int)recs.size();
  g.nc = nc;
  g.c_x.resize(nc); g.c_y.resize(nc); g.c_theta.resize(nc); g.c_nx.resize(nc); g.c_ny.resize(nc);
  g.c_axis.resize(nc); g.c_sigma.resize(nc); g.c_if.resize(nc); g.c_jf.resize(nc);
  g.c_ig.resize(nc); g.c_jg.resize(nc); g.c_body.resize(nc); g.c_seg.resize(nc); g.c_t.resize(nc);
  g.c_ub.resize(2 * (size_t)nc); g.c_psib.resize(nc);
  // prescribed boundary data: periodic cubic splines of the samples in the
  // same parameter as the boundary curve, evaluated at each control point
  std::vector<Spline> s_vel(bodies.size()), s_psi(bodies.size());
  for (size_t k = 0; k < bodies.size(); ++k) {
    const auto& smp = bodies[k].samples;
    if (smp.empty()) continue;
    const size_t P = bodies[k].xy.size() / 2;
    std::vector<double> uv(2 * P), pz(2 * P, 0.0);
    for (size_t p = 0; p < P; ++p) {
      uv[2 * p] = smp[3 * p];
      uv[2 * p + 1] = smp[3 * p + 1];
      pz[2 * p] = smp[3 * p + 2];
    }
    s_vel[k] = make_spline(uv);
    s_psi[k] = make_spline(pz);
  }
  for (int c = 0; c < nc; ++c) {
    const auto& r = recs[c];
    if (!(r.theta > 0.0 && r.theta <= 1.0)) throw GeomError("control point outside its grid edge");
    g.c_x[c] = r.x; g.c_y[c] = r.y; g.c_theta[c] = r.theta; g.c_nx[c] = r.nx; g.c_ny[c] = r.ny;
    g.c_axis[c] = r.axis; g.c_sigma[c] = r.sigma; g.c_if[c] = r.i_f; g.c_jf[c] = r.j_f;
    g.c_ig[c] = r.axis == 0 ? r.i_f + r.sigma : r.i_f;
    g.c_jg[c] = r.axis == 0 ? r.j_f : r.j_f + r.sigma;
    g.c_body[c] = r.body;
    g.c_seg[c] = r.seg;
    g.c_t[c] = r.t;
    const auto& b = bodies[r.body];
    if (!b.samples.empty()) {
      g.c_ub[2 * c] = ev(s_vel[r.body], 0, r.seg, r.t);
      g.c_ub[2 * c + 1] = ev(s_vel[r.body], 1, r.seg, r.t);
      g.c_psib[c] = ev(s_psi[r.body], 0, r.seg, r.t);
      continue;
    }
    // rigid motion: u = u_rigid + omega x (x - center), psi its stream function
    const double dx = r.x - b.center[0], dy = r.y - b.center[1];
    g.c_ub[2 * c] = b.u_rigid[0] - b.omega * dy;
    g.c_ub[2 * c + 1] = b.u_rigid[1] + b.omega * dx;
    g.c_psib[c] = b.u_rigid[0] * r.y - b.u_rigid[1] * r.x - 0.5 * b.omega * (dx * dx + dy * dy);
  }

  // ---- sets
  g.cls.assign((size_t)nx * ny, CLS_FLUID);
  g.ghost_id.assign((size_t)nx * ny, -1);
  g.a_id.assign((size_t)nx * ny, -1);
  const int di4[4] = {1, -1, 0, 0}, dj4[4] = {0, 0, 1, -1};
  std::vector<uint8_t> aplus((size_t)nx * ny, 0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t q = (size_t)j * nx + i;
      bool fl_nb = false, so_nb = false;
      for (int d = 0; d < 4; ++d) {
        const int ii = i + di4[d], jj = j + dj4[d];
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
        if (is_solid(ii, jj)) so_nb = true; else fl_nb = true;
      }
      if (solid[q]) g.cls[q] = fl_nb ? CLS_GHOST : CLS_SOLID;
      else aplus[q] = so_nb;
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t q = (size_t)j * nx + i;
      if (g.cls[q] == CLS_GHOST) {
        g.ghost_id[q] = g.ng++;
        g.g_i.push_back(i);
        g.g_j.push_back(j);
      }
      if (g.cls[q] == CLS_GHOST || aplus[q]) {
        g.a_id[q] = g.na++;
        g.a_i.push_back(i);
        g.a_j.push_back(j);
        g.a_ghost.push_back(g.cls[q] == CLS_GHOST);
      }
    }
  g.g_ctrl.assign(g.ng, {});
  g.a_body.assign(g.na, -1);
  for (int c = 0; c < nc; ++c) {
    const int gid = g.ghost_id[(size_t)g.c_jg[c] * nx + g.c_ig[c]];
    if (gid < 0) throw GeomError("control point without a ghost node");
    g.g_ctrl[gid].push_back(c);
    for (int side = 0; side < 2; ++side) {
      const int i = side ? g.c_ig[c] : g.c_if[c], j = side ? g.c_jg[c] : g.c_jf[c];
      const int a = g.a_id[(size_t)j * nx + i];
      if (g.a_body[a] >= 0 && g.a_body[a] != g.c_body[c])
        throw GeomError("affected point " + node_str(i, j) + " is adjacent to two bodies");
      g.a_body[a] = g.c_body[c];
    }
  }
  for (int a = 0; a < g.na; ++a)
    if (g.a_body[a] < 0) throw GeomError("affected point without a control point");

  // ---- ghost extrapolation tables
  auto fluid_at = [&](int i, int j) { return i >= 0 && j >= 0 && i < nx && j < ny && !is_solid(i, j); };
  auto behind = [&](int c, int m, int& i, int& j) {
    if (g.c_axis[c] == 0) { i = g.c_if[c] - m * g.c_sigma[c]; j = g.c_jf[c]; }
    else { i = g.c_if[c]; j = g.c_jf[c] - m * g.c_sigma[c]; }
  };
  auto build_ext = [&](Stencil& st, int count, bool with_bc, const char* name) {
    st = Stencil();
    for (int gid = 0; gid < g.ng; ++gid) {
      std::vector<int> valid;
      for (int c : g.g_ctrl[gid]) {
        bool ok = true;
        for (int m = 0; m < count; ++m) {
          int i, j;
          behind(c, m, i, j);
          if (!fluid_at(i, j)) { ok = false; break; }
        }
        if (ok) valid.push_back(c);
      }
      if (valid.empty())
        throw GeomError(std::string("ghost node ") + node_str(g.g_i[gid], g.g_j[gid]) + " (body " +
                        std::to_string(g.c_body[g.g_ctrl[gid][0]]) + ") has no valid " + name + " stencil");
      const double inv = 1.0 / valid.size();
      for (int c : valid) {
        double nodes[4], w[4];
        if (with_bc) {
          nodes[0] = g.c_theta[c];
          for (int m = 1; m < count; ++m) nodes[m] = -m;
          lagrange_at(nodes, count, 1.0, w);
          st.bc.push_back(c);
          st.bcomp.push_back(0);
          st.bw.push_back(inv * w[0]);
          for (int m = 1; m < count; ++m) {
            int i, j;
            behind(c, m, i, j);
            st.ii.push_back(i); st.jj.push_back(j); st.comp.push_back(0); st.w.push_back(inv * w[m]);
          }
        } else {
          for (int m = 0; m < count; ++m) nodes[m] = -m;
          lagrange_at(nodes, count, 1.0, w);
          for (int m = 0; m < count; ++m) {
            int i, j;
            behind(c, m, i, j);
            st.ii.push_back(i); st.jj.push_back(j); st.comp.push_back(0); st.w.push_back(inv * w[m]);
          }
        }
      }
      st.ptr.push_back((int)st.w.size());
      st.bptr.push_back((int)st.bw.size());
    }
  };
  build_ext(g.ext4b, 4, true, "fourth-order");
  build_ext(g.ext3b, 3, true, "third-order");
  build_ext(g.ext3n, 3, false, "third-order (no boundary value)");

  // ---- Poisson corrections gamma = A psi + B psi_b
  {
    const double ih2 = 1.0 / (h * h);
    Stencil& st = g.aop;
    st = Stencil();
    for (int a = 0; a < g.na; ++a) {
      const int i = g.a_i[a], j = g.a_j[a];
      std::map<std::pair<int, int>, double> acc;  // (j, i) -> w   (sorted, deterministic)
      std::map<int, double> bacc;
      for (int d = 0; d < 4; ++d) {
        const int ii = i + di4[d], jj = j + dj4[d];
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
        if (g.a_ghost[a]) {
          if (!is_solid(ii, jj)) acc[{jj, ii}] += ih2;
        } else if (is_solid(ii, jj)) {
          const int gid = g.ghost_id[(size_t)jj * nx + ii];
          for (int e = g.ext4b.ptr[gid]; e < g.ext4b.ptr[gid + 1]; ++e)
            acc[{g.ext4b.jj[e], g.ext4b.ii[e]}] -= ih2 * g.ext4b.w[e];
          for (int e = g.ext4b.bptr[gid]; e < g.ext4b.bptr[gid + 1]; ++e)
            bacc[g.ext4b.bc[e]] -= ih2 * g.ext4b.bw[e];
        }
      }
      for (auto& kv : acc) {
        st.ii.push_back(kv.first.second); st.jj.push_back(kv.first.first);
        st.comp.push_back(0); st.w.push_back(kv.second);
      }
      for (auto& kv : bacc) { st.bc.push_back(kv.first); st.bcomp.push_back(0); st.bw.push_back(kv.second); }
      st.ptr.push_back((int)st.w.size());
      st.bptr.push_back((int)st.bw.size());
    }
  }

  // ---- bounding regions R_k (default: bounding box of the body's affected points + 3)
  for (int k = 0; k < nb; ++k) {
    if (bodies[k].enclosure) continue;
    int i0, i1, j0, j1;
    if (bodies[k].rect[0] >= 0) {
      i0 = bodies[k].rect[0]; i1 = bodies[k].rect[1]; j0 = bodies[k].rect[2]; j1 = bodies[k].rect[3];
    } else {
      i0 = j0 = 1 << 30; i1 = j1 = -1;
      for (int a = 0; a < g.na; ++a)
        if (g.a_body[a] == k) {
          i0 = std::min(i0, g.a_i[a]); i1 = std::max(i1, g.a_i[a]);
          j0 = std::min(j0, g.a_j[a]); j1 = std::max(j1, g.a_j[a]);
        }
      i0 -= 3; i1 += 3; j0 -= 3; j1 += 3;
    }
    const std::string nm = "R_" + std::to_string(k);
    if (i0 < 2 || j0 < 2 || i1 > nx - 3 || j1 > ny - 3) throw GeomError(nm + " leaves the grid");
    for (int a = 0; a < g.na; ++a) {
      const bool inr = g.a_i[a] >= i0 && g.a_i[a] <= i1 && g.a_j[a] >= j0 && g.a_j[a] <= j1;
      if (g.a_body[a] == k && !inr) throw GeomError(nm + " does not contain its body");
      if (g.a_body[a] != k && inr) throw GeomError(nm + " contains another body");
    }
    for (int j = j0 - 2; j <= j1 + 2; ++j)
      for (int i = i0 - 2; i <= i1 + 2; ++i) {
        const bool inner = i >= i0 + 2 && i <= i1 - 2 && j >= j0 + 2 && j <= j1 - 2;
        if (inner) continue;
        const size_t q = (size_t)j * nx + i;
        if (solid[q] || aplus[q]) throw GeomError("the faces of " + nm + " are too close to a boundary");
      }
    g.rects.push_back({i0, i1, j0, j1});
    g.circ_body.push_back(k);
  }

  // ---- boundary vorticity stencils (Sec. 5.3)
  {
    auto has_value = [&](int i, int j) {
      return i >= 0 && j >= 0 && i < nx && j < ny && g.cls[(size_t)j * nx + i] != CLS_SOLID;
    };
    Stencil& st = g.wbc;
    st = Stencil();
    for (int c = 0; c < nc; ++c) {
      const int i = g.c_if[c], j = g.c_jf[c], s = g.c_sigma[c];
      const double xi_c = s * g.c_theta[c];
      const double along[3] = {(double)-s, 0.0, (double)s};
      double dw[3];
      lagrange_deriv_at(along, 3, xi_c, dw);
      int tau, lin_comp;
      double line_sign;
      if (g.c_axis[c] == 0) {
        tau = g.c_ny[c] >= 0 ? 1 : -1;
        for (int m = 0; m < 3; ++m) {  // + d_x u_y
          st.ii.push_back(i + (int)along[m]); st.jj.push_back(j); st.comp.push_back(1); st.w.push_back(dw[m] / h);
        }
        lin_comp = 0;
        line_sign = -1.0;  // - d_y u_x
      } else {
        tau = g.c_nx[c] >= 0 ? 1 : -1;
        for (int m = 0; m < 3; ++m) {  // - d_y u_x
          st.ii.push_back(i); st.jj.push_back(j + (int)along[m]); st.comp.push_back(0); st.w.push_back(-dw[m] / h);
        }
        lin_comp = 1;
        line_sign = 1.0;  // + d_x u_y
      }
      const double coef[3] = {-3.0, 4.0, -1.0};
      const double scale = line_sign * tau / (2.0 * h);
      st.bc.push_back(c); st.bcomp.push_back(lin_comp); st.bw.push_back(scale * coef[0]);
      for (int r = 1; r <= 2; ++r) {
        const int offs_set[2][3] = {{-s, 0, s}, {-2 * s, -s, 0}};
        int chosen = -1;
        for (int o = 0; o < 2 && chosen < 0; ++o) {
          bool ok = true;
          for (int m = 0; m < 3; ++m) {
            const int a = g.c_axis[c] == 0 ? i + offs_set[o][m] : i + r * tau;
            const int b = g.c_axis[c] == 0 ? j + r * tau : j + offs_set[o][m];
            if (!has_value(a, b)) { ok = false; break; }
          }
          if (ok) chosen = o;
        }
        if (chosen < 0)
          throw GeomError("control point near " + node_str(i, j) + " (body " + std::to_string(g.c_body[c]) +
                          "): no boundary-vorticity stencil");
        double nodes[3] = {(double)offs_set[chosen][0], (double)offs_set[chosen][1], (double)offs_set[chosen][2]};
        double wi[3];
        lagrange_at(nodes, 3, xi_c, wi);
        for (int m = 0; m < 3; ++m) {
          const int a = g.c_axis[c] == 0 ? i + offs_set[chosen][m] : i + r * tau;
          const int b = g.c_axis[c] == 0 ? j + r * tau : j + offs_set[chosen][m];
          st.ii.push_back(a); st.jj.push_back(b); st.comp.push_back(lin_comp);
          st.w.push_back(scale * coef[r] * wi[m]);
        }
      }
      st.ptr.push_back((int)st.w.size());
      st.bptr.push_back((int)st.bw.size());
    }
  }

  // ---- transport: fluid nodes whose stencils meet a solid or ghost node
  // (nodes near the grid edge whose stencils are otherwise fluid stay in the
  // bulk kernel, which treats nodes outside the grid as vorticity-free fluid)
  auto solid_in_grid = [&](int i, int j) { return i >= 0 && j >= 0 && i < nx && j < ny && is_solid(i, j); };
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      if (is_solid(i, j)) continue;
      bool sp = false;
      for (int d = -2; d <= 2 && !sp; ++d) {
        if (d == 0) continue;
        if (solid_in_grid(i + d, j) || solid_in_grid(i, j + d)) sp = true;
      }
      if (sp) g.special.push_back(j * nx + i);
    }

  // ---- pruned Krylov windows
  g.src_j0 = ny; g.src_j1 = -1; g.out_j0 = ny; g.out_j1 = -1;
  for (int a = 0; a < g.na; ++a) {
    g.src_j0 = std::min(g.src_j0, g.a_j[a]);
    g.src_j1 = std::max(g.src_j1, g.a_j[a]);
  }
  for (size_t e = 0; e < g.aop.jj.size(); ++e) {
    g.out_j0 = std::min(g.out_j0, g.aop.jj[e]);
    g.out_j1 = std::max(g.out_j1, g.aop.jj[e]);
  }
}

}  // namespace iim
