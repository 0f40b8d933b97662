// Flat octree construction and adaptive projection of Gaussian sums (Sec. 2.1).
//
// Projection: f = sum_g c_g exp(-a_g |x - X_g|^2) is separable, so a box's coefficients are
// sum_g c_g X_i Y_j Z_m with exact 1D integrals (composite Gauss-Legendre, k+20 nodes per
// panel of width <= min(1, beta^{-1/2}), beta = a h^2, over the Gaussian's numerical
// support).  A box at level n < max_level is refined iff the Frobenius norm of its wavelet
// coefficients d = B - unfilter(filter(B)) (B = children block) exceeds thresh; a box that
// is not refined becomes a leaf holding its own projection.
#include <algorithm>
#include <cmath>
#include <memory>
#include <thread>
#include <unordered_map>

#include "mra_internal.hpp"

namespace mra {

int Func::level_of(int64_t node) const {
  int n = (int)(std::upper_bound(level_off.begin(), level_off.end(), node) - level_off.begin()) - 1;
  return n;
}

void build_tree(Func& f, const std::vector<std::vector<uint64_t>>& levels) {
  f.nlev = (int)levels.size();
  while (f.nlev > 0 && levels[f.nlev - 1].empty()) --f.nlev;
  f.level_off.assign(f.nlev + 1, 0);
  for (int n = 0; n < f.nlev; ++n) f.level_off[n + 1] = f.level_off[n] + (int64_t)levels[n].size();
  int64_t total = f.level_off[f.nlev];
  if (total > INT32_MAX / 2) fail(MRA_E_UNSUPPORTED, "tree too large");
  f.code.resize(total);
  f.first_child.assign(total, -1);
  for (int n = 0; n < f.nlev; ++n)
    std::copy(levels[n].begin(), levels[n].end(), f.code.begin() + f.level_off[n]);
  for (int n = 0; n + 1 < f.nlev; ++n) {
    // both code lists are ascending: one merge walk links every parent to its first child
    const auto& kids = levels[n + 1];
    const int64_t nk = (int64_t)kids.size();
    int64_t j = 0;
    for (int64_t i = f.level_off[n]; i < f.level_off[n + 1]; ++i) {
      const uint64_t c0 = f.code[i] << 3;
      while (j < nk && kids[j] < c0) ++j;
      if (j < nk && kids[j] == c0) {
        if (j + 7 >= nk || kids[j + 7] != c0 + 7) fail(MRA_E_INVALID, "tree is not a full octree");
        f.first_child[i] = (int32_t)(f.level_off[n + 1] + j);
      }
    }
  }
  f.finalize_structure();
}

void Func::finalize_structure() {
  leaves.clear();
  interior.clear();
  inter_level_off.assign(nlev + 1, 0);
  for (int n = 0; n < nlev; ++n) {
    for (int64_t i = level_off[n]; i < level_off[n + 1]; ++i) {
      if (first_child[i] < 0)
        leaves.push_back((int32_t)i);
      else
        interior.push_back((int32_t)i);
    }
    inter_level_off[n + 1] = (int64_t)interior.size();
  }
}

const int32_t* Func::device_leaves() {
  if (d_leaves.n != leaves.size() || !d_leaves.p) d_leaves.upload(ctx, leaves);
  return d_leaves.p;
}

// ------------------------------------------------------------------ projection
namespace {

double support_halfwidth(double beta) {
  if (beta <= 0.0) return INFINITY;
  return std::sqrt((50.0 + 0.5 * std::log1p(beta)) / beta);
}

// int exp(-a (x - X)^2) phi^n_{l,i}(x) dx, i < k, for the box l of width h from cell start lo.
void gaussian_1d(int k, double a, double X, double lo, double h, int64_t l, double* out) {
  for (int i = 0; i < k; ++i) out[i] = 0.0;
  double beta = a * h * h;
  double u0 = (X - lo) / h - (double)l;
  double half = support_halfwidth(beta);
  double ua = std::max(0.0, u0 - half), ub = std::min(1.0, u0 + half);
  if (ub <= ua) return;
  double width = beta > 0.0 ? std::min(1.0, 1.0 / std::sqrt(beta)) : 1.0;
  int npan = std::max(1, (int)std::ceil((ub - ua) / width));
  double step = (ub - ua) / npan;
  const GLRule& g = gauss_legendre01(k + 20);
  double ph[kMaxK];
  for (int p = 0; p < npan; ++p) {
    double ea = ua + p * step, eb = (p + 1 == npan) ? ub : ua + (p + 1) * step;
    for (size_t q = 0; q < g.x.size(); ++q) {
      double u = ea + (eb - ea) * g.x[q];
      double wt = (eb - ea) * g.w[q] * std::exp(-beta * (u - u0) * (u - u0));
      scaling_functions(k, u, ph);
      for (int i = 0; i < k; ++i) out[i] += wt * ph[i];
    }
  }
  double sh = std::sqrt(h);
  for (int i = 0; i < k; ++i) out[i] *= sh;
}

struct Projector {
  const mra_gaussian* g;
  int ng, k;
  double lo, W;
  std::vector<double> h0, h1;
  // 1D integrals per (gaussian, axis, level, l): a shared read-only table filled before each
  // parallel level, and a private memo for anything not in it
  const std::unordered_map<uint64_t, std::vector<double>>* shared = nullptr;
  std::unordered_map<uint64_t, std::vector<double>> memo;

  static uint64_t key_of(int gi, int axis, int n, int64_t l) {
    return ((uint64_t)gi << 50) | ((uint64_t)axis << 48) | ((uint64_t)n << 40) | (uint64_t)l;
  }
  const std::vector<double>& one_d(int gi, int axis, int n, int64_t l) {
    uint64_t key = key_of(gi, axis, n, l);
    if (shared) {
      auto it = shared->find(key);
      if (it != shared->end()) return it->second;
    }
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    std::vector<double> v(k);
    double h = W / std::ldexp(1.0, n);
    gaussian_1d(k, g[gi].expnt, g[gi].center[axis], lo, h, l, v.data());
    return memo.emplace(key, std::move(v)).first->second;
  }

  // coefficients of box (n, lx, ly, lz) into out[k^3]
  void box(int n, int64_t lx, int64_t ly, int64_t lz, double* out) {
    int k3 = k * k * k;
    for (int i = 0; i < k3; ++i) out[i] = 0.0;
    for (int gi = 0; gi < ng; ++gi) {
      const auto& x = one_d(gi, 0, n, lx);
      bool zx = true;
      for (double v : x) zx = zx && v == 0.0;
      if (zx) continue;
      const auto& y = one_d(gi, 1, n, ly);
      bool zy = true;
      for (double v : y) zy = zy && v == 0.0;
      if (zy) continue;
      const auto& z = one_d(gi, 2, n, lz);
      double c = g[gi].coeff;
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          double cij = c * x[i] * y[j];
          double* o = out + (i * k + j) * k;
          for (int m = 0; m < k; ++m) o[m] += cij * z[m];
        }
    }
  }

  // Frobenius norm of the wavelet part of the 8 children of (n, lx, ly, lz).
  double wavelet_norm(int n, int64_t lx, int64_t ly, int64_t lz, std::vector<double>& kids) {
    int k3 = k * k * k;
    kids.resize(8 * k3);
    for (int c = 0; c < 8; ++c)
      box(n + 1, 2 * lx + ((c >> 2) & 1), 2 * ly + ((c >> 1) & 1), 2 * lz + (c & 1),
          kids.data() + c * k3);
    // s = sum_c (h^{bx} x h^{by} x h^{bz}) child_c ; ||d||^2 = ||B||^2 - ||s||^2 is prone to
    // cancellation, so form d = B - unfilter(s) explicitly.
    std::vector<double> s(k3, 0.0), t1(k3), t2(k3);
    for (int c = 0; c < 8; ++c) {
      const double* hx = ((c >> 2) & 1) ? h1.data() : h0.data();
      const double* hy = ((c >> 1) & 1) ? h1.data() : h0.data();
      const double* hz = (c & 1) ? h1.data() : h0.data();
      const double* src = kids.data() + c * k3;
      // t1[i][j'][m'] = sum_i' hx[i][i'] src[i'][j'][m']
      for (int i = 0; i < k; ++i)
        for (int r = 0; r < k * k; ++r) {
          double acc = 0.0;
          for (int ip = 0; ip < k; ++ip) acc += hx[i * k + ip] * src[ip * k * k + r];
          t1[i * k * k + r] = acc;
        }
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
          for (int m = 0; m < k; ++m) {
            double acc = 0.0;
            for (int jp = 0; jp < k; ++jp) acc += hy[j * k + jp] * t1[(i * k + jp) * k + m];
            t2[(i * k + j) * k + m] = acc;
          }
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
          for (int m = 0; m < k; ++m) {
            double acc = 0.0;
            for (int mp = 0; mp < k; ++mp) acc += hz[m * k + mp] * t2[(i * k + j) * k + mp];
            s[(i * k + j) * k + m] += acc;
          }
    }
    double d2 = 0.0;
    for (int c = 0; c < 8; ++c) {
      const double* hx = ((c >> 2) & 1) ? h1.data() : h0.data();
      const double* hy = ((c >> 1) & 1) ? h1.data() : h0.data();
      const double* hz = (c & 1) ? h1.data() : h0.data();
      // u = (hx^T x hy^T x hz^T) s
      for (int ip = 0; ip < k; ++ip)
        for (int r = 0; r < k * k; ++r) {
          double acc = 0.0;
          for (int i = 0; i < k; ++i) acc += hx[i * k + ip] * s[i * k * k + r];
          t1[ip * k * k + r] = acc;
        }
      for (int ip = 0; ip < k; ++ip)
        for (int jp = 0; jp < k; ++jp)
          for (int m = 0; m < k; ++m) {
            double acc = 0.0;
            for (int j = 0; j < k; ++j) acc += hy[j * k + jp] * t1[(ip * k + j) * k + m];
            t2[(ip * k + jp) * k + m] = acc;
          }
      const double* src = kids.data() + c * k3;
      for (int ip = 0; ip < k; ++ip)
        for (int jp = 0; jp < k; ++jp)
          for (int mp = 0; mp < k; ++mp) {
            double acc = 0.0;
            for (int m = 0; m < k; ++m) acc += hz[m * k + mp] * t2[(ip * k + jp) * k + m];
            double d = src[(ip * k + jp) * k + mp] - acc;
            d2 += d * d;
          }
    }
    return std::sqrt(d2);
  }
};

uint64_t interleave(int n, int64_t lx, int64_t ly, int64_t lz) {
  uint64_t code = 0;
  for (int b = 0; b < n; ++b) {
    code |= (uint64_t)((lx >> b) & 1) << (3 * b + 2);
    code |= (uint64_t)((ly >> b) & 1) << (3 * b + 1);
    code |= (uint64_t)((lz >> b) & 1) << (3 * b);
  }
  return code;
}

}  // namespace

void project_gaussians(Ctx* ctx, const mra_gaussian* g, int ng, int k, double thresh,
                       int initial_level, int max_level, Func& out,
                       std::vector<double>& leaf_coeffs) {
  // Level by level: the refinement tests of one level run in parallel host threads, each
  // with its own memo of 1D integrals.
  std::vector<double> h0, h1;
  two_scale_filters(k, h0, h1);
  const int k3 = k * k * k;
  unsigned nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<Projector> pr(nthr);
  for (auto& p : pr) {
    p.g = g;
    p.ng = ng;
    p.k = k;
    p.lo = ctx->lo;
    p.W = ctx->width();
    p.h0 = h0;
    p.h1 = h1;
  }
  struct Box {
    int64_t lx, ly, lz;
  };
  std::vector<Box> frontier;
  int64_t nb = (int64_t)1 << initial_level;
  for (int64_t x = 0; x < nb; ++x)
    for (int64_t y = 0; y < nb; ++y)
      for (int64_t z = 0; z < nb; ++z) frontier.push_back({x, y, z});
  std::vector<std::pair<uint64_t, std::vector<double>>> leafvals;  // (prefixed code, coeffs)
  std::unordered_map<uint64_t, std::vector<double>> table;
  for (int n = initial_level; n <= max_level && !frontier.empty(); ++n) {
    // the 1D integrals this level needs (boxes at n, children at n+1), computed once
    {
      std::vector<uint64_t> need;
      for (const Box& b : frontier) {
        const int64_t l3[3] = {b.lx, b.ly, b.lz};
        for (int gi = 0; gi < ng; ++gi)
          for (int ax = 0; ax < 3; ++ax) {
            need.push_back(Projector::key_of(gi, ax, n, l3[ax]));
            if (n < max_level) {
              need.push_back(Projector::key_of(gi, ax, n + 1, 2 * l3[ax]));
              need.push_back(Projector::key_of(gi, ax, n + 1, 2 * l3[ax] + 1));
            }
          }
      }
      std::sort(need.begin(), need.end());
      need.erase(std::unique(need.begin(), need.end()), need.end());
      std::vector<std::vector<double>> vals1(need.size(), std::vector<double>(k));
      const unsigned nt1 = (unsigned)std::max<size_t>(1, std::min<size_t>(nthr, need.size()));
      auto fill = [&](unsigned t) {
        for (size_t i = t; i < need.size(); i += nt1) {
          uint64_t key = need[i];
          int gi = (int)(key >> 50), ax = (int)((key >> 48) & 3), lev = (int)((key >> 40) & 255);
          int64_t l = (int64_t)(key & ((1ULL << 40) - 1));
          gaussian_1d(k, g[gi].expnt, g[gi].center[ax], ctx->lo, ctx->width() / std::ldexp(1.0, lev),
                      l, vals1[i].data());
        }
      };
      std::vector<std::thread> th1;
      for (unsigned t = 1; t < nt1; ++t) th1.emplace_back(fill, t);
      fill(0);
      for (auto& t : th1) t.join();
      table.clear();
      table.reserve(need.size() * 2);
      for (size_t i = 0; i < need.size(); ++i) table.emplace(need[i], std::move(vals1[i]));
      for (auto& p : pr) {
        p.shared = &table;
        p.memo.clear();
      }
    }
    std::vector<char> refine(frontier.size(), 0);
    std::vector<std::vector<double>> vals(frontier.size());
    const unsigned nt = (unsigned)std::min<size_t>(nthr, frontier.size());
    auto work = [&](unsigned t) {
      std::vector<double> kids;
      for (size_t i = t; i < frontier.size(); i += nt) {
        const Box& b = frontier[i];
        if (n < max_level && pr[t].wavelet_norm(n, b.lx, b.ly, b.lz, kids) > thresh) {
          refine[i] = 1;
        } else {
          vals[i].resize(k3);
          pr[t].box(n, b.lx, b.ly, b.lz, vals[i].data());
        }
      }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& t : th) t.join();
    std::vector<Box> next;
    for (size_t i = 0; i < frontier.size(); ++i) {
      const Box& b = frontier[i];
      if (refine[i]) {
        for (int c = 0; c < 8; ++c)
          next.push_back({2 * b.lx + ((c >> 2) & 1), 2 * b.ly + ((c >> 1) & 1), 2 * b.lz + (c & 1)});
      } else {
        leafvals.push_back({((uint64_t)n << 58) | interleave(n, b.lx, b.ly, b.lz), std::move(vals[i])});
      }
    }
    frontier.swap(next);
  }
  // node sets: leaves plus all ancestors
  std::vector<std::vector<uint64_t>> sets(max_level + 1);
  for (auto& lv : leafvals) {
    int n = (int)(lv.first >> 58);
    uint64_t code = lv.first & ((1ULL << 58) - 1);
    sets[n].push_back(code);
    for (int m = n - 1; m >= 0; --m) {
      code >>= 3;
      sets[m].push_back(code);
    }
  }
  for (auto& s : sets) {
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
  }
  out.ctx = ctx;
  out.k = k;
  build_tree(out, sets);
  // leaf coefficients in node order
  leaf_coeffs.assign((size_t)out.nodes() * k3, 0.0);
  for (auto& lv : leafvals) {
    int n = (int)(lv.first >> 58);
    uint64_t code = lv.first & ((1ULL << 58) - 1);
    auto beg = out.code.begin() + out.level_off[n], end = out.code.begin() + out.level_off[n + 1];
    auto it = std::lower_bound(beg, end, code);
    int64_t node = it - out.code.begin();
    std::copy(lv.second.begin(), lv.second.end(), leaf_coeffs.begin() + node * k3);
  }
}

void project_gaussians_device(Ctx* ctx, const mra_gaussian* g, int ng, int k, double thresh,
                              int initial_level, int max_level, Func& out) {
  // Level by level: the host keeps the frontier (its box indices) and the refinement
  // decisions; the device computes every integral, coefficient and wavelet norm.
  if (ng > 4096) fail(MRA_E_UNSUPPORTED, "the device projection takes at most 4096 Gaussians");
  const int k3 = k * k * k;
  std::vector<double> gp(5 * (size_t)ng);
  for (int i = 0; i < ng; ++i) {
    gp[5 * i] = g[i].expnt;
    for (int a = 0; a < 3; ++a) gp[5 * i + 1 + a] = g[i].center[a];
    gp[5 * i + 4] = g[i].coeff;
  }
  std::vector<double> h0v, h1v;
  two_scale_filters(k, h0v, h1v);
  const GLRule& rule = gauss_legendre01(k + 20);
  DevArray<double> d_gp, d_h0, d_h1, d_glx, d_glw;
  d_gp.upload(ctx, gp);
  d_h0.upload(ctx, h0v);
  d_h1.upload(ctx, h1v);
  d_glx.upload(ctx, rule.x);
  d_glw.upload(ctx, rule.w);
  struct Box {
    int64_t lx, ly, lz;
  };
  std::vector<Box> frontier;
  const int64_t nb = (int64_t)1 << initial_level;
  for (int64_t x = 0; x < nb; ++x)
    for (int64_t y = 0; y < nb; ++y)
      for (int64_t z = 0; z < nb; ++z) frontier.push_back({x, y, z});
  struct Leaf {
    uint64_t key;       // level-prefixed code, as in the host projection
    int32_t lev, slot;  // staging buffer (per level) and slab in it
  };
  std::vector<Leaf> leaves;
  std::vector<std::unique_ptr<DevArray<double>>> staging;
  for (int n = initial_level; n <= max_level && !frontier.empty(); ++n) {
    const int64_t nbox = (int64_t)frontier.size();
    if (nbox > INT32_MAX) fail(MRA_E_UNSUPPORTED, "projection level too large");
    // distinct 1D box indices per axis, concatenated x, y, z
    std::vector<int64_t> lv[3];
    for (const Box& b : frontier) {
      lv[0].push_back(b.lx);
      lv[1].push_back(b.ly);
      lv[2].push_back(b.lz);
    }
    std::vector<int64_t> lvals;
    int64_t off[4] = {0, 0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      std::sort(lv[a].begin(), lv[a].end());
      lv[a].erase(std::unique(lv[a].begin(), lv[a].end()), lv[a].end());
      lvals.insert(lvals.end(), lv[a].begin(), lv[a].end());
      off[a + 1] = (int64_t)lvals.size();
    }
    std::vector<int32_t> boxu(3 * (size_t)nbox);
    for (int64_t b = 0; b < nbox; ++b) {
      const int64_t l3[3] = {frontier[b].lx, frontier[b].ly, frontier[b].lz};
      for (int a = 0; a < 3; ++a)
        boxu[3 * b + a] = (int32_t)(off[a] + (std::lower_bound(lv[a].begin(), lv[a].end(), l3[a]) -
                                               lv[a].begin()));
    }
    const int nl = (int)lvals.size();
    if ((double)nl * ng * 5 * k * sizeof(double) > 8.0 * (1 << 30))
      fail(MRA_E_UNSUPPORTED, "projection level too large (1D integral table above 8 GiB)");
    DevArray<int64_t> d_lvals;
    DevArray<int32_t> d_boxu;
    DevArray<double> d_T, d_d2;
    DevArray<uint8_t> d_nz;
    d_lvals.upload(ctx, lvals);
    d_boxu.upload(ctx, boxu);
    d_T.alloc(ctx, (size_t)nl * ng * 5 * k);
    d_nz.alloc(ctx, (size_t)nl * ng);
    const bool test = n < max_level;
    d_d2.alloc(ctx, test ? nbox : 1);
    staging.emplace_back(new DevArray<double>());
    staging.back()->alloc(ctx, (size_t)nbox * k3);
    launch_gauss1d(k, d_gp.p, ng, d_lvals.p, nl, (int)off[1], (int)off[2], n, ctx->lo,
                   ctx->width(), d_glx.p, d_glw.p, (int)rule.x.size(), d_h0.p, d_h1.p, d_T.p,
                   d_nz.p, ctx->stream);
    launch_project_level(k, d_T.p, d_nz.p, d_boxu.p, (int)nbox, ng, d_gp.p, test ? 1 : 0,
                         d_d2.p, staging.back()->p, ctx->stream);
    std::vector<double> d2(test ? nbox : 0);
    if (test)
      hip_check(hipMemcpyAsync(d2.data(), d_d2.p, nbox * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream),
                "hipMemcpyAsync D2H");
    ctx->sync();
    std::vector<Box> next;
    for (int64_t b = 0; b < nbox; ++b) {
      const Box& x = frontier[b];
      if (test && std::sqrt(d2[b]) > thresh) {
        for (int c = 0; c < 8; ++c)
          next.push_back({2 * x.lx + ((c >> 2) & 1), 2 * x.ly + ((c >> 1) & 1), 2 * x.lz + (c & 1)});
      } else {
        leaves.push_back({((uint64_t)n << 58) | interleave(n, x.lx, x.ly, x.lz),
                          (int32_t)(staging.size() - 1), (int32_t)b});
      }
    }
    frontier.swap(next);
  }
  // node sets: leaves plus all ancestors
  std::vector<std::vector<uint64_t>> sets(max_level + 1);
  for (const Leaf& lf : leaves) {
    int n = (int)(lf.key >> 58);
    uint64_t code = lf.key & ((1ULL << 58) - 1);
    sets[n].push_back(code);
    for (int m = n - 1; m >= 0; --m) {
      code >>= 3;
      sets[m].push_back(code);
    }
  }
  for (auto& st : sets) {
    std::sort(st.begin(), st.end());
    st.erase(std::unique(st.begin(), st.end()), st.end());
  }
  out.ctx = ctx;
  out.k = k;
  build_tree(out, sets);
  out.coeff.alloc(ctx, (size_t)out.nodes() * k3);
  launch_zero(out.coeff.p, out.coeff.n, ctx->stream);
  // leaf slabs from the staging buffers into node order, one copy launch per level
  std::vector<std::vector<int32_t>> to(staging.size()), from(staging.size());
  for (const Leaf& lf : leaves) {
    const int n = (int)(lf.key >> 58);
    const uint64_t code = lf.key & ((1ULL << 58) - 1);
    auto beg = out.code.begin() + out.level_off[n], end = out.code.begin() + out.level_off[n + 1];
    to[lf.lev].push_back((int32_t)(std::lower_bound(beg, end, code) - out.code.begin()));
    from[lf.lev].push_back(lf.slot);
  }
  for (size_t v = 0; v < staging.size(); ++v) {
    if (to[v].empty()) continue;
    DevArray<int32_t> d_to, d_from;
    d_to.upload(ctx, to[v]);
    d_from.upload(ctx, from[v]);
    launch_copy_slabs(k, out.coeff.p, d_to.p, staging[v]->p, d_from.p, (int)to[v].size(),
                      ctx->stream);
    ctx->sync();
  }
}

}  // namespace mra
