// Host FP64 numerics of libmra: Gauss-Legendre rules, Legendre scaling functions, the
// two-scale filter (Sec. 2.1-2.2), the Gaussian-sum fits of 1/r and exp(-mu r)/r (Sec. 2.3)
// and the 1D operator blocks of one Gaussian term with their norms (Sec. 2.2 Toeplitz
// blocks; non-standard children blocks).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "mra_internal.hpp"

namespace mra {

// ------------------------------------------------------------------ Gauss-Legendre
// Nodes by Newton iteration on P_n from the Chebyshev-like initial guess
// cos(pi (i + 3/4) / (n + 1/2)); weights 2 / ((1 - x^2) P_n'(x)^2), mapped to [0, 1].
static GLRule make_rule(int n) {
  GLRule r;
  r.x.resize(n);
  r.w.resize(n);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? x : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (x * pn - pm) / (x * x - 1.0);
      double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        // one more evaluation of the derivative at the converged node
        p0 = 1.0;
        p1 = x;
        for (int j = 2; j <= n; ++j) {
          double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
          p0 = p1;
          p1 = p2;
        }
        pn = (n == 1) ? x : p1;
        pm = (n == 1) ? 1.0 : p0;
        dp = n * (x * pn - pm) / (x * x - 1.0);
        break;
      }
    }
    r.x[n - 1 - i] = 0.5 * (x + 1.0);
    r.w[n - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);   // 2/(..) times the 1/2 of [0,1]
  }
  return r;
}

const GLRule& gauss_legendre01(int n) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<GLRule>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(n);
  if (it == cache.end()) it = cache.emplace(n, std::make_unique<GLRule>(make_rule(n))).first;
  return *it->second;
}

void scaling_functions(int k, double x, double* out) {
  if (x < 0.0 || x > 1.0) {
    for (int i = 0; i < k; ++i) out[i] = 0.0;
    return;
  }
  double t = 2.0 * x - 1.0;
  double pm = 1.0, p = t;
  out[0] = 1.0;
  if (k > 1) out[1] = std::sqrt(3.0) * t;
  for (int i = 1; i + 1 < k; ++i) {
    double pn = ((2.0 * i + 1.0) * t * p - i * pm) / (i + 1.0);
    pm = p;
    p = pn;
    out[i + 1] = std::sqrt(2.0 * (i + 1) + 1.0) * pn;
  }
}

void two_scale_filters(int k, std::vector<double>& h0, std::vector<double>& h1) {
  // h0[i][j] = 2^{-1/2} int_0^1 phi_i(u/2) phi_j(u) du, h1 with phi_i((u+1)/2).
  h0.assign(k * k, 0.0);
  h1.assign(k * k, 0.0);
  const GLRule& g = gauss_legendre01(k);
  std::vector<double> pa(k), pb(k), pc(k);
  for (int q = 0; q < k; ++q) {
    double u = g.x[q];
    scaling_functions(k, 0.5 * u, pa.data());
    scaling_functions(k, 0.5 * (u + 1.0), pb.data());
    scaling_functions(k, u, pc.data());
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        h0[i * k + j] += g.w[q] * pa[i] * pc[j] * M_SQRT1_2;
        h1[i * k + j] += g.w[q] * pb[i] * pc[j] * M_SQRT1_2;
      }
  }
}

// ------------------------------------------------------------------ fits (Sec. 2.3)
double erfc_inverse(double p) {
  // Newton on erfc(y) = p from y0 = sqrt(-log p) (p in (0, 1)).
  if (!(p > 0.0 && p < 2.0)) fail(MRA_E_INVALID, "erfc_inverse: argument out of range");
  double y = (p < 1.0) ? std::sqrt(-std::log(p)) : -std::sqrt(-std::log(2.0 - p));
  for (int it = 0; it < 200; ++it) {
    double f = std::erfc(y) - p;
    double df = -2.0 / std::sqrt(M_PI) * std::exp(-y * y);
    double dy = f / df;
    y -= dy;
    if (std::fabs(dy) <= 1e-16 * std::max(1.0, std::fabs(y))) break;
  }
  return y;
}

// Trapezoid grid of (2/sqrt(pi)) int exp(-r^2 e^{2s} + s) ds: step pi^2/(2(ln(1/eps)+3)),
// upper end ln(erfcinv(eps/4)/r_lo), lower end ln(eps sqrt(pi)/(8 r_hi)).
static void fit_grid(double r_lo, double eps, double r_hi, double& h, double& s_lo, int& m) {
  if (!(r_lo > 0.0 && eps > 0.0 && eps < 1.0 && r_hi > r_lo))
    fail(MRA_E_INVALID, "fit: need 0 < lo < r_hi and 0 < eps < 1");
  h = M_PI * M_PI / (2.0 * (std::log(1.0 / eps) + 3.0));
  double s_hi = std::log(erfc_inverse(eps / 4.0) / r_lo);
  s_lo = std::log(eps * std::sqrt(M_PI) / (8.0 * r_hi));
  m = (int)std::ceil((s_hi - s_lo) / h) + 1;
}

void fit_coulomb(double r_lo, double eps, double r_hi, std::vector<double>& c,
                 std::vector<double>& t) {
  double h, s_lo;
  int m;
  fit_grid(r_lo, eps, r_hi, h, s_lo, m);
  c.resize(m);
  t.resize(m);
  for (int j = 0; j < m; ++j) {
    double s = s_lo + h * j;
    c[j] = 2.0 / std::sqrt(M_PI) * h * std::exp(s);
    t[j] = std::exp(2.0 * s);
  }
}

// Bound of the omitted lower tail (2/sqrt pi) int_{-inf}^{s} exp(s' - mu^2 e^{-2s'}/4) ds':
// min((2/sqrt pi) e^s, mu/(2 sqrt pi) x^{-3/2} e^{-x}), x = mu^2 e^{-2s}/4.
static double bsh_tail(double s, double mu) {
  double coul = 2.0 / std::sqrt(M_PI) * std::exp(s);
  double x = mu * mu * std::exp(-2.0 * s) / 4.0;
  if (x <= 0.0) return coul;
  return std::min(coul, mu / (2.0 * std::sqrt(M_PI)) * std::pow(x, -1.5) * std::exp(-x));
}

void fit_bsh(double mu, double r_lo, double eps, double r_hi, std::vector<double>& c,
             std::vector<double>& t) {
  if (!(mu >= 0.0)) fail(MRA_E_INVALID, "fit_bsh: mu must be >= 0");
  double h, s_lo;
  int m;
  fit_grid(r_lo, eps, r_hi, h, s_lo, m);
  double target = eps / (4.0 * r_hi);
  int j0 = 0;
  while (j0 + 1 < m && bsh_tail(s_lo + (j0 + 1) * h, mu) <= target) ++j0;
  c.resize(m - j0);
  t.resize(m - j0);
  for (int j = j0; j < m; ++j) {
    double s = s_lo + h * j;
    c[j - j0] = 2.0 / std::sqrt(M_PI) * h * std::exp(s - mu * mu * std::exp(-2.0 * s) / 4.0);
    t[j - j0] = std::exp(2.0 * s);
  }
}

// ------------------------------------------------------------------ 1D blocks
static double support_halfwidth(double beta) {
  if (beta <= 0.0) return INFINITY;
  return std::sqrt((50.0 + 0.5 * std::log1p(beta)) / beta);
}

// C_ij(w) = int_{max(0,w)}^{min(1,1+w)} phi_i(u) phi_j(u - w) du, exact with k-point GL.
static void correlation(int k, double w, double* C) {
  const GLRule& g = gauss_legendre01(k);
  double lo = std::max(0.0, w), hi = std::min(1.0, 1.0 + w);
  for (int i = 0; i < k * k; ++i) C[i] = 0.0;
  double len = hi - lo;
  if (len <= 0.0) return;
  double pi[kMaxK], pj[kMaxK];
  for (int q = 0; q < k; ++q) {
    double u = lo + len * g.x[q];
    double wt = len * g.w[q];
    scaling_functions(k, u, pi);
    scaling_functions(k, u - w, pj);
    for (int i = 0; i < k; ++i) {
      double a = wt * pi[i];
      for (int j = 0; j < k; ++j) C[i * k + j] += a * pj[j];
    }
  }
}

void block_t(int k, double h, int delta, double texp, double* out) {
  // t[i][j] = h int_{-1}^{1} exp(-beta (delta + w)^2) C_ij(w) dw; pieces [-1,0], [0,1]
  // split at the peak w = -delta, restricted to the Gaussian's numerical support, panels
  // of width <= min(1, beta^{-1/2}) with 2k+20 Gauss-Legendre nodes.
  double beta = texp * h * h;
  double half = support_halfwidth(beta);
  double wc = -(double)delta;
  double width = beta > 0.0 ? std::min(1.0, 1.0 / std::sqrt(beta)) : 1.0;
  const GLRule& g = gauss_legendre01(2 * k + 20);
  for (int i = 0; i < k * k; ++i) out[i] = 0.0;
  std::vector<double> C(k * k);
  const double pieces[2][2] = {{-1.0, 0.0}, {0.0, 1.0}};
  for (auto& pc : pieces) {
    double a2 = std::max(pc[0], wc - half), b2 = std::min(pc[1], wc + half);
    if (b2 <= a2) continue;
    double cuts[3] = {a2, b2, 0};
    int ncut = 2;
    if (a2 < wc && wc < b2) {
      cuts[0] = a2;
      cuts[1] = wc;
      cuts[2] = b2;
      ncut = 3;
    }
    for (int p = 0; p + 1 < ncut; ++p) {
      double pa = cuts[p], pb = cuts[p + 1];
      int npan = std::max(1, (int)std::ceil((pb - pa) / width));
      double step = (pb - pa) / npan;
      for (int q = 0; q < npan; ++q) {
        double ea = pa + q * step, eb = (q + 1 == npan) ? pb : pa + (q + 1) * step;
        for (int r = 0; r < (int)g.x.size(); ++r) {
          double w = ea + (eb - ea) * g.x[r];
          double d = (double)delta + w;
          double wt = (eb - ea) * g.w[r] * std::exp(-beta * d * d);
          if (wt == 0.0) continue;
          correlation(k, w, C.data());
          for (int i = 0; i < k * k; ++i) out[i] += wt * C[i];
        }
      }
    }
  }
  for (int i = 0; i < k * k; ++i) out[i] *= h;
}

double spectral_norm(int m, const double* a) {
  // sigma_max(A) = sqrt(lambda_max(A^T A)) by cyclic Jacobi rotations.
  std::vector<double> g(m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int r = 0; r < m; ++r) s += a[r * m + i] * a[r * m + j];
      g[i * m + j] = s;
    }
  double tr = 0.0;
  for (int i = 0; i < m; ++i) tr += g[i * m + i];
  if (tr == 0.0) return 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += g[p * m + q] * g[p * m + q];
    if (off <= 1e-34 * tr * tr) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        double apq = g[p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = g[p * m + p], aqq = g[q * m + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < m; ++r) {
          double grp = g[r * m + p], grq = g[r * m + q];
          g[r * m + p] = c * grp - s * grq;
          g[r * m + q] = s * grp + c * grq;
        }
        for (int r = 0; r < m; ++r) {
          double gpr = g[p * m + r], gqr = g[q * m + r];
          g[p * m + r] = c * gpr - s * gqr;
          g[q * m + r] = s * gpr + c * gqr;
        }
      }
  }
  double lmax = 0.0;
  for (int i = 0; i < m; ++i) lmax = std::max(lmax, g[i * m + i]);
  return std::sqrt(lmax);
}

double e_bound(int k, double h, double beta) {
  // 2 * 1.0865 * h * beta^{k/2} / sqrt(2^k k!) (Taylor remainder of order k of the Gaussian
  // kernel in each variable, Cramer's bound on Hermite functions); never above h.
  double lf = std::lgamma(k + 1.0) + k * std::log(2.0);
  double v = 2.0 * 1.0865 * h * std::pow(beta, 0.5 * k) / std::exp(0.5 * lf);
  return std::min(h, v);
}

double decay_bound(double h, double beta, int delta) {
  int d = std::abs(delta);
  if (d == 0) return 2.0 * h;
  return 2.0 * h * std::exp(-beta * (double)(d - 1) * (double)(d - 1));
}

}  // namespace mra
