// Non-standard apply (Sec. 2.2-2.3) for one function or a batch of functions.
//
// Steps, all on the context's stream:
//   1. filter-up (device): s_P and ||B_P||_F^2 of every refined box of every function, one
//      launch per level for the whole batch; one copy of the norms to the host;
//   2. screening (host, threads over (function, level, term) jobs): triples (P, delta, mu)
//      with eta = |c_mu| N(delta) ||B_P||_F >= tau_drop and target inside the cell; at
//      levels n > 0 a triple with eta < tau_tier goes to the low-precision tier;
//   3. per function (threads over functions): targets grouped by a counting sort, the
//      output tree (targets, their children, ancestors, closed under siblings) and the
//      target-sorted work list; long lists are split over several workgroups;
//   4. transform-and-accumulate (device): one launch for all children blocks, one for the
//      sum of split partials, one for the level-n subtractions (all functions together),
//      one for the low-precision tier (which adds after the FP64 results);
//   5. sum-down (device), one launch per level for the whole batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "mra_internal.hpp"

namespace mra {

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Bit b of v (v < 2^21) moved to bit 3b, and back: the usual shift-and-mask spreading.
inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ULL;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
  v = (v ^ (v >> 32)) & 0x1fffffULL;
  return v;
}
void decode(uint64_t code, int n, int64_t& x, int64_t& y, int64_t& z) {
  const uint64_t c = n >= 21 ? code : code & ((1ULL << (3 * n)) - 1);
  x = (int64_t)compact3(c >> 2);
  y = (int64_t)compact3(c >> 1);
  z = (int64_t)compact3(c);
}

uint64_t encode(int n, int64_t x, int64_t y, int64_t z) {
  const uint64_t m = n >= 21 ? 0x1fffffULL : (1ULL << n) - 1;
  return spread3((uint64_t)x & m) << 2 | spread3((uint64_t)y & m) << 1 | spread3((uint64_t)z & m);
}

int64_t find_node(const Func& f, int n, uint64_t code) {
  if (n >= f.nlev) return -1;
  auto beg = f.code.begin() + f.level_off[n], end = f.code.begin() + f.level_off[n + 1];
  auto it = std::lower_bound(beg, end, code);
  if (it == end || *it != code) return -1;
  return it - f.code.begin();
}

template <class F>
void parallel_for(size_t count, F&& fn) {
  Pool::get().run(count, std::function<void(size_t, unsigned)>(fn));
}

// |c| N(delta) of the screening bound (N = prod(a + e) - prod(a) at n > 0, prod(r) at n = 0).
// One definition with contraction off, so that the target pre-pass and the enumeration
// compare bit-identical values (and the same values as an evaluation without fused
// multiply-adds).
inline double screen_cn(double c, int n, const double* ae, const double* aa, const double* rr,
                        int ax, int ay, int az) {
#pragma clang fp contract(off)
  const double N = n > 0 ? ae[ax] * ae[ay] * ae[az] - aa[ax] * aa[ay] * aa[az]
                         : rr[ax] * rr[ay] * rr[az];
  return c * N;
}

// Exact pruning of a job's displacement cube.  Every factor of screen_cn's products is
// non-negative and rounding is monotone, so raising one factor can only raise the computed
// c N (and c N maxb), while dropping the subtracted term of the n > 0 form can only raise
// it too.  With S[d] = max over |delta| >= d of the 1D factor (a + e, or r at n = 0), the
// product with S[d] in place of an axis' factor bounds every displacement at distance >= d
// along that axis; a line of the cube ends where that bound falls below tau.  The visited
// candidates keep their order, and every candidate that passes the test is visited.
struct ScreenBound {
  double c = 0.0, maxb = 0.0, tau = 0.0;
  const double* f = nullptr;   // 1D factors, 0..D
  std::vector<double> S;       // suffix maxima, 0..D
  int D = 0;
  ScreenBound(double c_, double maxb_, double tau_, const double* f_, int D_)
      : c(c_), maxb(maxb_), tau(tau_), f(f_), S(D_ + 2, 0.0), D(D_) {
    for (int d = D; d >= 0; --d) S[d] = std::max(f[d], S[d + 1]);
  }
  // the products in screen_cn's order ((x y) z); passes iff the bound reaches tau
  bool pass(double fx, double fy, double fz) const {
#pragma clang fp contract(off)
    return c * (fx * fy * fz) * maxb >= tau;
  }
  // largest |dz| whose plane can hold a kept candidate (-1: none)
  int rz() const {
    int r = D;
    while (r >= 0 && !pass(S[0], S[0], S[r])) --r;
    return r;
  }
  // largest |dy| in plane |dz| = az
  int ry(int az) const {
    int r = D;
    while (r >= 0 && !pass(S[0], S[r], f[az])) --r;
    return r;
  }
  // largest |dx| on line (|dy|, |dz|) = (ay, az)
  int rx(int ay, int az) const {
    int r = D;
    while (r >= 0 && !pass(S[r], f[ay], f[az])) --r;
    return r;
  }
};

// Sorts codes below 2^bits ascending and removes duplicates (LSD radix, 11-bit digits).
void radix_sort_unique(std::vector<uint64_t>& v, int bits) {
  if (v.size() > 1 && bits > 0) {
    constexpr int RB = 11;
    std::vector<uint64_t> tmp(v.size());
    std::vector<uint32_t> cnt(1u << RB);
    for (int sh = 0; sh < bits; sh += RB) {
      std::fill(cnt.begin(), cnt.end(), 0u);
      for (uint64_t x : v) ++cnt[(x >> sh) & ((1u << RB) - 1)];
      uint32_t run = 0;
      for (auto& c : cnt) {
        const uint32_t t = c;
        c = run;
        run += t;
      }
      for (uint64_t x : v) tmp[cnt[(x >> sh) & ((1u << RB) - 1)]++] = x;
      v.swap(tmp);
    }
  }
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

struct Triple {
  uint64_t tcode;  // (level << 58) | code of the target
  int32_t src;     // index into f.interior
  int16_t mu;
  int16_t dx, dy, dz;
  int8_t low;      // 1: low-precision tier
};

struct LevelData {
  int fn = 0, n = 0;
  int64_t ib = 0, np = 0;
  double maxb = 0.0;
  std::vector<double> bn;
  std::vector<int64_t> px, py, pz, order;
};

struct Job {
  int lev, mu, D;
  const BlockEntry* be;
};

// Host-side plan of one function.
struct Plan {
  Op* op = nullptr;
  Func* f = nullptr;
  Func* out = nullptr;
  std::vector<const BlockEntry*> entry_tab;  // (level, mu) -> cache entry
};

// Output tree of one function from its target codes (ascending by level, then code):
// targets, their children, ancestors, closed under siblings (full octree).  Every level's
// code list is built from at most three ascending runs (children of the level above, the
// level's own targets, parents of the level below), which are merged rather than sorted.
void build_output_tree(Ctx* ctx, Plan& p, const std::vector<uint64_t>& tcodes) {
  Func& out = *p.out;
  int maxlev = 0;
  for (uint64_t t : tcodes) maxlev = std::max(maxlev, (int)(t >> 58) + 1);
  const int L = std::max(maxlev + 1, 1);
  std::vector<std::vector<uint64_t>> sets(L);
  std::vector<std::vector<size_t>> runs(L);   // start offsets of ascending runs
  auto start_run = [&](int n) {
    if (runs[n].empty() || runs[n].back() != sets[n].size()) runs[n].push_back(sets[n].size());
  };
  int cur = -1;
  for (uint64_t t : tcodes) {
    const int n = (int)(t >> 58);
    const uint64_t code = t & ((1ULL << 58) - 1);
    if (n != cur) {
      start_run(n);
      start_run(n + 1);
      cur = n;
    }
    sets[n].push_back(code);
    for (int c = 0; c < 8; ++c) sets[n + 1].push_back((code << 3) | c);
  }
  // level n + 1 received the children of level n before level n + 1's own targets, so the
  // runs are recorded in push order; merge them pairwise
  auto merge_runs = [&](int n) {
    auto& v = sets[n];
    auto& r = runs[n];
    r.push_back(v.size());
    while (r.size() > 2) {
      std::vector<size_t> nr{r[0]};
      for (size_t i = 0; i + 2 < r.size(); i += 2) {
        std::inplace_merge(v.begin() + r[i], v.begin() + r[i + 1], v.begin() + r[i + 2]);
        nr.push_back(r[i + 2]);
      }
      if ((r.size() - 1) % 2 == 1) nr.push_back(r.back());
      r.swap(nr);
    }
    v.erase(std::unique(v.begin(), v.end()), v.end());
  };
  sets[0].push_back(0);
  if (runs[0].empty() || runs[0].front() != 0) runs[0].insert(runs[0].begin(), 0);
  for (int n = L - 1; n >= 1; --n) {
    merge_runs(n);
    auto& s = sets[n];
    std::vector<uint64_t> full;
    full.reserve(s.size() * 2);
    uint64_t lastp = ~0ULL;
    start_run(n - 1);
    for (uint64_t code : s) {
      const uint64_t par = code >> 3;
      if (par == lastp) continue;
      lastp = par;
      for (int c = 0; c < 8; ++c) full.push_back((par << 3) | c);
      sets[n - 1].push_back(par);
    }
    s.swap(full);
  }
  merge_runs(0);
  out.ctx = ctx;
  out.k = p.f->k;
  build_tree(out, sets);
}

// The kept triples of one (function, level) unit, grouped by target and, within a target,
// ordered by source then term (so that a source block is staged once per run of terms).
// Triples of a level are split by the top bits of the target's Morton code into kBuckets
// buckets (ascending code ranges) so that grouping runs in parallel on small pieces; the
// units of a level, in bucket order, list the targets in ascending code order.
constexpr int kBuckets = 16;
inline int target_bucket(int n, uint64_t code) {
  const int bits = 3 * n;
  return bits > 4 ? (int)(code >> (bits - 4)) : (int)code;
}

struct Unit {
  int fn = 0, n = 0;
  size_t jb = 0, je = 0;               // jobs of this unit
  int bucket = 0;                      // target-code bucket of this unit
  std::vector<Triple> sorted;
  std::vector<uint64_t> tcodes;        // ascending
  std::vector<int64_t> toff;           // tcodes.size() + 1
  std::vector<int64_t> tmid;           // per target: first low-tier triple
  std::vector<int64_t> fpre, lpre;     // per target: prefix counts of FP64 / low items
  std::vector<int32_t> node;           // per target: output node
  size_t item_base = 0, low_base = 0;  // offsets of this unit's items in the batch arrays
};

void group_unit(Unit& u, const std::vector<std::vector<Triple>>& jobout, const LevelData& L,
                bool factored) {
  auto piece = [&](size_t j) -> const std::vector<Triple>& { return jobout[j * kBuckets + u.bucket]; };
  size_t m = 0;
  for (size_t j = u.jb; j < u.je; ++j) m += piece(j).size();
  // composite key (target code, tier, source rank); an LSD radix sort on it is stable, and
  // the jobs of a unit are in ascending term order, so terms stay ascending per source.
  // For a factored kernel the FP64 triples leave the source rank out of the key: they keep
  // the enumeration order, which per target is (term, dz, dy, dx).
  int sbits = 1;
  while (((int64_t)1 << sbits) <= L.np) ++sbits;
  const int bits = 3 * u.n + 1 + sbits;
  if (bits > 64) {   // very deep level with many boxes: stable comparison sort
    u.sorted.clear();
    u.sorted.reserve(m);
    for (size_t j = u.jb; j < u.je; ++j)
      u.sorted.insert(u.sorted.end(), piece(j).begin(), piece(j).end());
    std::stable_sort(u.sorted.begin(), u.sorted.end(), [factored](const Triple& a, const Triple& b) {
      if (a.tcode != b.tcode) return a.tcode < b.tcode;
      if (a.low != b.low) return a.low < b.low;
      if (factored && !a.low) return false;
      return a.src < b.src;
    });
    u.tcodes.clear();
    u.toff.clear();
    u.tmid.clear();
    for (size_t q = 0; q < m; ++q) {
      const Triple& t = u.sorted[q];
      if (q == 0 || t.tcode != u.sorted[q - 1].tcode) {
        u.tcodes.push_back(t.tcode);
        u.toff.push_back((int64_t)q);
        u.tmid.push_back(-1);
      }
      if (t.low && u.tmid.back() < 0) u.tmid.back() = (int64_t)q;
    }
    u.toff.push_back((int64_t)m);
    for (size_t r = 0; r < u.tmid.size(); ++r)
      if (u.tmid[r] < 0) u.tmid[r] = u.toff[r + 1];
    return;
  }
  const uint64_t cmask = (1ULL << (3 * u.n)) - 1;
  std::vector<uint64_t> key(m), key2(m);
  std::vector<uint32_t> idx(m), idx2(m);
  std::vector<const Triple*> ptr(m);
  bool any_low = false;
  {
    size_t q = 0;
    for (size_t j = u.jb; j < u.je; ++j)
      for (const Triple& t : piece(j)) {
        key[q] = ((t.tcode & cmask) << (1 + sbits)) | ((uint64_t)t.low << sbits) |
                 ((t.low || !factored) ? (uint64_t)(t.src - L.ib) : 0);
        any_low |= t.low != 0;
        idx[q] = (uint32_t)q;
        ptr[q] = &t;
        ++q;
      }
  }
  // only key bits that vary are sorted on: without low-tier triples a factored unit's keys
  // have zero tier and source fields, and the bucket fixes the top 4 bits of the code
  const int lo_bit = (factored && !any_low) ? 1 + sbits : 0;
  const int hi_bit = 3 * u.n > 4 ? bits - 4 : 1 + sbits;
  constexpr int RB = 11;
  std::vector<uint32_t> cnt(1u << RB);
  for (int sh = lo_bit; sh < hi_bit; sh += RB) {
    std::fill(cnt.begin(), cnt.end(), 0u);
    for (size_t q = 0; q < m; ++q) ++cnt[(key[q] >> sh) & ((1u << RB) - 1)];
    uint32_t run = 0;
    for (auto& c : cnt) {
      uint32_t v = c;
      c = run;
      run += v;
    }
    for (size_t q = 0; q < m; ++q) {
      uint32_t d = cnt[(key[q] >> sh) & ((1u << RB) - 1)]++;
      key2[d] = key[q];
      idx2[d] = idx[q];
    }
    key.swap(key2);
    idx.swap(idx2);
  }
  u.sorted.resize(m);
  u.tcodes.clear();
  u.toff.clear();
  u.tmid.clear();
  const uint64_t lev = (uint64_t)u.n << 58;
  uint64_t last = ~0ULL;
  for (size_t q = 0; q < m; ++q) {
    const Triple& t = *ptr[idx[q]];
    u.sorted[q] = t;
    const uint64_t code = key[q] >> (1 + sbits);
    if (code != last) {
      u.tcodes.push_back(lev | code);
      u.toff.push_back((int64_t)q);
      u.tmid.push_back(-1);
      last = code;
    }
    if (t.low && u.tmid.back() < 0) u.tmid.back() = (int64_t)q;
  }
  u.toff.push_back((int64_t)m);
  for (size_t r = 0; r < u.tmid.size(); ++r)
    if (u.tmid[r] < 0) u.tmid[r] = u.toff[r + 1];
}

// Work items of the targets [r0, r1) of one unit, written at their final positions: per
// target the FP64 triples (NSItem), then the low-tier triples (LowItem, source block by its
// filter-up slot).  Every index is checked against the arrays it will address; returns the
// sum of eta over the low-tier triples, or throws on an inconsistent plan.
double fill_items(Unit& u, const Plan& p, const LevelData& L, const std::vector<int64_t>& slot,
                  int64_t r0, int64_t r1, NSItem* items, LowItem* low, int64_t nR, int64_t nT,
                  int64_t nL, int64_t nslots) {
  const Func& f = *p.f;
  const Func& out = *p.out;
  const int n = u.n;
  const int M = (int)p.op->c.size();
  const int64_t nin = f.nodes(), nout = out.nodes();
  auto bad = [](const char* what) {
    fail(MRA_E_INVALID, std::string("internal plan error: ") + what);
  };
  double eta = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const uint64_t code = u.tcodes[r] & ((1ULL << 58) - 1);
    const int64_t node = find_node(out, n, code);
    if (node < 0 || node >= nout || out.first_child[node] < 0 ||
        out.first_child[node] + 8 > nout)
      bad("target node");
    u.node[r] = (int32_t)node;
    NSItem* fi = items + u.item_base + u.fpre[r];
    LowItem* li = low + u.low_base + u.lpre[r];
    for (int64_t q = u.toff[r]; q < u.toff[r + 1]; ++q) {
      const Triple& t = u.sorted[q];
      if (t.mu < 0 || t.mu >= M) bad("term index");
      const BlockEntry& be = *p.entry_tab[(size_t)n * M + t.mu];
      const int64_t rx = be.r_base + t.dx + be.D, ry = be.r_base + t.dy + be.D,
                    rz = be.r_base + t.dz + be.D;
      if (!t.low) {
        NSItem it;
        it.src = f.interior[t.src];
        it.src_fc = f.first_child[it.src];
        it.mu = t.mu;
        it.rx = (int32_t)rx;
        it.ry = (int32_t)ry;
        it.rz = (int32_t)rz;
        it.tx = (int32_t)(be.t_base + t.dx + be.D);
        it.ty = (int32_t)(be.t_base + t.dy + be.D);
        it.tz = (int32_t)(be.t_base + t.dz + be.D);
        it.slot = (int32_t)slot[t.src];
        if (it.src < 0 || it.src >= nin || it.src_fc < 0 || it.src_fc + 8 > nin)
          bad("source node");
        if (it.slot < 0 || it.slot >= nslots) bad("source slot");
        if (std::min({rx, ry, rz}) < 0 || std::max({rx, ry, rz}) >= nR) bad("R block");
        if (std::min({it.tx, it.ty, it.tz}) < 0 || std::max({it.tx, it.ty, it.tz}) >= nT)
          bad("t block");
        *fi++ = it;
      } else {
        const int64_t sl = slot[t.src];
        if (sl < 0 || sl >= nslots) bad("low-tier source block");
        if (std::min({rx, ry, rz}) < 0 || std::max({rx, ry, rz}) >= nL) bad("low-tier block");
        *li++ = {(int32_t)sl, (int32_t)t.mu, (int32_t)rx, (int32_t)ry, (int32_t)rz};
        const int ax = std::abs(t.dx), ay = std::abs(t.dy), az = std::abs(t.dz);
        const double N = (be.a[ax] + be.e[ax]) * (be.a[ay] + be.e[ay]) * (be.a[az] + be.e[az]) -
                         be.a[ax] * be.a[ay] * be.a[az];
        eta += std::fabs(p.op->c[t.mu]) * N * L.bn[t.src - L.ib];
      }
    }
  }
  return eta;
}

}  // namespace

void apply_nonstandard_batch(Ctx* ctx, const std::vector<Op*>& ops,
                             const std::vector<Func*>& funcs, double tau, double tau_tier,
                             const std::vector<Func*>& outs) {
  const int nf = (int)funcs.size();
  if (nf == 0) return;
  const double t_entry = now_ms();
  for (Func* f : funcs)
    if (f->interior.empty())
      fail(MRA_E_INVALID, "non-standard apply needs a refined root (project with initial_level >= 1)");
  const int k = funcs[0]->k;
  const int K3 = k * k * k;
  const bool tiers = tau_tier > 0.0;
  const size_t XB = (size_t)4 * k * k * low_up(k);   // BF16 per mirrored children block
  std::vector<double> h0v, h1v;
  two_scale_filters(k, h0v, h1v);

  // ---- 1. filter-up for the whole batch
  hip_check(hipEventRecord(ctx->ev[0], ctx->stream), "event");
  std::vector<double*> coeff_in(nf);
  for (int i = 0; i < nf; ++i) coeff_in[i] = funcs[i]->coeff.p;
  int maxlev = 0;
  for (Func* f : funcs) maxlev = std::max(maxlev, f->nlev);
  std::vector<NodeRef> fu_refs;
  std::vector<int64_t> fu_off(maxlev + 1, 0);        // refs of level maxlev-1-j
  std::vector<std::vector<int64_t>> fu_index(nf);    // per function: entry of each interior
  for (int i = 0; i < nf; ++i) fu_index[i].resize(funcs[i]->interior.size());
  for (int n = maxlev - 1, j = 0; n >= 0; --n, ++j) {
    for (int i = 0; i < nf; ++i) {
      const Func& f = *funcs[i];
      if (n >= f.nlev) continue;
      for (int64_t q = f.inter_level_off[n]; q < f.inter_level_off[n + 1]; ++q) {
        fu_index[i][q] = (int64_t)fu_refs.size();
        fu_refs.push_back({i, f.interior[q], f.first_child[f.interior[q]], -1});
      }
    }
    fu_off[j + 1] = (int64_t)fu_refs.size();
  }
  Arena& A0 = ctx->arena[0];
  A0.begin(ctx);
  const size_t o_h0 = A0.put(h0v), o_h1 = A0.put(h1v), o_in = A0.put(coeff_in);
  const size_t o_fu = A0.put(fu_refs);
  const size_t o_bn2 = A0.scratch(std::max<size_t>(1, fu_refs.size()) * sizeof(double));
  const size_t o_mir = A0.scratch(tiers ? fu_refs.size() * XB * sizeof(uint16_t) : 0);
  // the children blocks in slab order for a kernel that streams them (by filter-up slot)
  const bool slab_mirror = ns_uses_slab_mirror(k);
  const size_t o_slabs = A0.scratch(slab_mirror ? fu_refs.size() * 8 * (size_t)K3 * sizeof(double) : 0);
  // pinned host landing place of the box norms, so that their copy is asynchronous (a copy
  // into pageable memory would hold the host until the filter-up is done)
  const size_t o_bn2h = A0.reserve(std::max<size_t>(1, fu_refs.size()) * sizeof(double));
  A0.commit();
  const double* h0p = A0.at<double>(o_h0);
  const double* h1p = A0.at<double>(o_h1);
  double* const* in_tab_d = A0.at<double*>(o_in);
  const NodeRef* fu_d = A0.at<NodeRef>(o_fu);
  double* bn2_d = A0.scr_at<double>(o_bn2);
  uint16_t* mirror_d = tiers ? A0.scr_at<uint16_t>(o_mir) : nullptr;
  double* slabs_d = slab_mirror ? A0.scr_at<double>(o_slabs) : nullptr;
  for (int j = 0; j < maxlev; ++j) {
    int64_t b = fu_off[j], e = fu_off[j + 1];
    if (e > b)
      launch_filter_up(k, in_tab_d, fu_d + b, (int)(e - b), h0p, h1p, bn2_d + b,
                       tiers ? mirror_d + (size_t)b * XB : nullptr, ctx->stream);
  }
  if (slab_mirror)   // every slab is final once the whole filter-up has run
    launch_slab_mirror(k, in_tab_d, fu_d, (int)fu_refs.size(), slabs_d, ctx->stream);
  const double* const bn2_all = A0.host_at<double>(o_bn2h);   // valid after the sync below
  if (!fu_refs.empty())
    hip_check(hipMemcpyAsync(A0.host_at<double>(o_bn2h), bn2_d, fu_refs.size() * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream),
              "hipMemcpyAsync D2H");
  hip_check(hipEventRecord(ctx->ev[1], ctx->stream), "event");
  // wake the planner's thread pool while the device runs the filter-up: workers that went
  // to sleep since the last apply would otherwise be woken by the first planning loop
  const double t_filter_issued = now_ms();
  Pool::get().run(Pool::get().workers(), [](size_t, unsigned) {});
  ctx->sync();
  for (Func* f : funcs) f->interior_valid = true;
  double t_plan0 = now_ms();
  const bool timing = std::getenv("MRA_TIMING") != nullptr;
  if (timing)
    std::fprintf(stderr, "[mra] %-28s %8.3f ms\n[mra] %-28s %8.3f ms\n", "filter issued",
                 t_filter_issued - t_entry, "filter wait", t_plan0 - t_filter_issued);
  double t_mark = t_plan0;
  auto mark = [&](const char* what) {
    if (!timing) return;
    double t = now_ms();
    std::fprintf(stderr, "[mra] %-28s %8.3f ms\n", what, t - t_mark);
    t_mark = t;
  };

  // ---- 2a. levels and (level, term) jobs; the block cache is filled here (sequential)
  const double W = ctx->width();
  std::vector<Plan> plans(nf);
  std::vector<LevelData> lv;
  std::vector<Job> jobs;
  for (int i = 0; i < nf; ++i) {
    Func& f = *funcs[i];
    Op& op = *ops[i];
    plans[i].op = &op;
    plans[i].f = &f;
    plans[i].out = outs[i];
    const int M = (int)op.c.size();
    plans[i].entry_tab.assign((size_t)std::max(1, f.nlev) * M, nullptr);
    for (int n = 0; n < f.nlev; ++n) {
      int64_t ib = f.inter_level_off[n], ie = f.inter_level_off[n + 1];
      if (ie <= ib) continue;
      LevelData L;
      L.fn = i;
      L.n = n;
      L.ib = ib;
      L.np = ie - ib;
      lv.push_back(std::move(L));
    }
  }
  // per level: source norms, positions, and the sources by descending norm (in parallel)
  parallel_for(lv.size(), [&](size_t li, unsigned) {
    LevelData& L = lv[li];
    const Func& f = *funcs[L.fn];
    L.bn.resize(L.np);
    L.px.resize(L.np);
    L.py.resize(L.np);
    L.pz.resize(L.np);
    for (int64_t q = 0; q < L.np; ++q) {
      L.bn[q] = std::sqrt(bn2_all[fu_index[L.fn][L.ib + q]]);
      L.maxb = std::max(L.maxb, L.bn[q]);
      decode(f.code[f.interior[L.ib + q]], L.n, L.px[q], L.py[q], L.pz[q]);
    }
    L.order.resize(L.np);
    std::iota(L.order.begin(), L.order.end(), 0);
    std::stable_sort(L.order.begin(), L.order.end(),
                     [&](int64_t a, int64_t b) { return L.bn[a] > L.bn[b]; });
  });
  mark("levels");
  // displacement ranges of the (level, term) jobs, in parallel; -1 marks a dropped term
  {
    std::vector<size_t> lv_off(lv.size() + 1, 0);
    for (size_t li = 0; li < lv.size(); ++li)
      lv_off[li + 1] = lv_off[li] + ops[lv[li].fn]->c.size();
    std::vector<int> jobD(lv_off.back(), -1);
    parallel_for(lv.size(), [&](size_t li, unsigned) {
      const LevelData& LL = lv[li];
      const Op& op = *ops[LL.fn];
      const int n = LL.n;
      const int64_t nb = (int64_t)1 << n;
      const double h = W / std::ldexp(1.0, n);
      for (size_t mu = 0; mu < op.c.size(); ++mu) {
        double c = std::fabs(op.c[mu]);
        double beta = op.t[mu] * h * h;
        double ab = 2.0 * h;
        double fac = 1.0;
        if (n > 0) {
          if (c * LL.maxb * 3.0 * e_bound(k, h, beta) * ab * ab < tau) continue;
          fac = 3.0;
        }
        int D = 0;
        while (D + 1 <= nb - 1 && c * LL.maxb * fac * ab * ab * decay_bound(h, beta, D + 1) >= tau)
          ++D;
        jobD[lv_off[li] + mu] = D;
      }
    });
    for (size_t li = 0; li < lv.size(); ++li)
      for (size_t mu = 0; mu < lv_off[li + 1] - lv_off[li]; ++mu) {
        const int D = jobD[lv_off[li] + mu];
        if (D < 0) continue;
        if (D > 32000) fail(MRA_E_UNSUPPORTED, "displacement range too large");
        jobs.push_back({(int)li, (int)mu, D, nullptr});
      }
  }
  mark("displacement ranges");
  // Fill the block caches: distinct operators in parallel, each operator's entries in order.
  {
    std::vector<Op*> uops;
    for (Op* op : ops)
      if (std::find(uops.begin(), uops.end(), op) == uops.end()) uops.push_back(op);
    std::vector<std::vector<size_t>> by_op(uops.size());
    for (size_t j = 0; j < jobs.size(); ++j) {
      Op* op = ops[lv[jobs[j].lev].fn];
      by_op[std::find(uops.begin(), uops.end(), op) - uops.begin()].push_back(j);
    }
    std::vector<std::string> errs(uops.size());
    parallel_for(uops.size(), [&](size_t u, unsigned) {
      try {
        for (size_t j : by_op[u]) {
          Job& jb = jobs[j];
          jb.be = &uops[u]->ensure(lv[jb.lev].n, jb.mu, jb.D);
        }
      } catch (const Error& e) {
        errs[u] = e.msg;
      }
    });
    for (auto& e : errs)
      if (!e.empty()) fail(MRA_E_INVALID, e);
    if (tiers)
      for (Op* op : uops) op->ensure_low();   // data-parallel over blocks inside
    for (const Job& jb : jobs) {
      const LevelData& L = lv[jb.lev];
      plans[L.fn].entry_tab[(size_t)L.n * ops[L.fn]->c.size() + jb.mu] = jb.be;
    }
  }

  mark("levels and jobs");
  // every job's blocks are in the caches now: one upload before the first launch
  std::vector<Op*> uniq_ops;
  for (Op* op : ops)
    if (std::find(uniq_ops.begin(), uniq_ops.end(), op) == uniq_ops.end()) uniq_ops.push_back(op);
  for (Op* op : uniq_ops) op->sync_device();
  const double t_prep = now_ms() - t_plan0;

  // ---- sub-batches: contiguous ranges of functions, balanced by (refined boxes x terms).
  // Sub-batch s is planned on the host while the device runs sub-batch s - 1; its upload
  // arena alternates between two, and is reused only after the device has finished the
  // sub-batch that used it before.
  std::vector<size_t> job_begin(nf + 1, jobs.size());
  for (size_t j = jobs.size(); j-- > 0;) job_begin[lv[jobs[j].lev].fn] = j;
  for (int i = nf - 1; i >= 0; --i) job_begin[i] = std::min(job_begin[i], job_begin[i + 1]);
  std::vector<double> weight(nf, 0.0);
  for (const Job& jb : jobs) weight[lv[jb.lev].fn] += (double)lv[jb.lev].np;
  const int S = std::min(nf, ctx->sched_sub_batches > 0 ? ctx->sched_sub_batches
                                                         : (nf >= 8 ? 4 : (nf >= 2 ? 2 : 1)));
  std::vector<int> fb{0};
  {
    double total = 0.0, acc = 0.0;
    for (double w : weight) total += w;
    for (int i = 0; i < nf && (int)fb.size() < S; ++i) {
      acc += weight[i];
      if (acc >= total * (double)fb.size() / S && i + 1 < nf) fb.push_back(i + 1);
    }
    fb.push_back(nf);
  }
  const int nsb = (int)fb.size() - 1;
  struct Events {
    hipEvent_t e[4]{};
    Events() {
      for (auto& x : e) hip_check(hipEventCreate(&x), "hipEventCreate");
    }
    ~Events() {
      for (auto& x : e)
        if (x) (void)hipEventDestroy(x);
    }
  };
  // per chunk: transform start, main kernel end, low-tier start, chunk end;
  // per sub-batch: sum-down start, sum-down end
  std::vector<std::unique_ptr<Events>> cev, sev;

  const double f_ns = 6.0 * std::pow(2.0 * k, 4), f_sub = 6.0 * std::pow((double)k, 4);
  const bool fused = ns_kernel_fuses_subtraction(k);
  const bool factored = ns_kernel_factored(k);
  int64_t ntriples = 0, ntargets = 0, nlow = 0, in_leaves = 0, out_nodes = 0, out_leaves = 0;
  double flops = 0.0, flops_low = 0.0, eta_low = 0.0, flops_kernel = 0.0, plan_ms = t_prep;
  bool any_low = false;
  int64_t n_low_launch = 0;
  // per (job, bucket) outputs; the vectors keep their capacity across applies on this host
  // thread, so enumeration neither allocates nor frees in steady state
  static thread_local std::vector<std::vector<Triple>> t_jobout;
  std::vector<std::vector<Triple>>& jobout = t_jobout;

  for (int sb = 0; sb < nsb; ++sb) {
    const int f0 = fb[sb], f1 = fb[sb + 1];
    const size_t j0 = job_begin[f0], j1 = job_begin[f1];
    if (sb >= 2) hip_check(hipEventSynchronize(sev[sb - 2]->e[1]), "hipEventSynchronize");
    double t_sb0 = now_ms();
    t_mark = t_sb0;
    // ---- 2b. target sets of the (function, level) level-units, exact and term-independent:
    // T = P + d is a target iff max_mu c_mu N_mu(d) ||B_P|| >= tau over the terms whose
    // displacement range contains d, the same products the enumeration compares
    std::vector<size_t> lu_j;   // level-unit u = jobs [lu_j[u], lu_j[u + 1])
    for (size_t j = j0; j < j1; ++j)
      if (j == j0 || jobs[j].lev != jobs[j - 1].lev) lu_j.push_back(j);
    lu_j.push_back(j1);
    const size_t nlu = lu_j.size() - 1;
    std::vector<std::vector<uint64_t>> lu_codes(nlu);
    std::vector<double> lu_weight(nlu, 0.0);
    // Pipelining pays only when planning is long against its fixed costs (a pre-pass, more and
    // smaller launches): large sub-batches are planned and launched in chunks of level-units,
    // small ones in one piece (targets then come from the grouping itself).
    double est = 0.0;
    for (size_t j = j0; j < j1; ++j) est += (double)lv[jobs[j].lev].np;
    const char* pm = std::getenv("MRA_PIPELINE_MIN");   // in sources x terms; tests lower it
    const double pipe_min = pm ? std::atof(pm) : 1.0e5;
    const bool pipelined = est >= pipe_min;
    // enumerate and group the jobs of level-units [ua, ub) (the chunk's units, in order)
    std::vector<Unit> units;
    std::vector<int> unit_lev;
    auto enumerate_group = [&](size_t ua, size_t ub) {
      const size_t ja = lu_j[ua], jz = lu_j[ub];
      const size_t njb = (jz - ja) * kBuckets;
      if (jobout.size() < njb) jobout.resize(njb);
      for (size_t q = 0; q < njb; ++q) jobout[q].clear();
      parallel_for(jz - ja, [&](size_t jj, unsigned) {
        const Job& jb = jobs[ja + jj];
        const LevelData& L = lv[jb.lev];
        const Op& op = *ops[L.fn];
        const int n = L.n, D = jb.D, mu = jb.mu;
        const int64_t nb = (int64_t)1 << n;
        const double c = std::fabs(op.c[mu]);
        std::vector<double> ae(D + 1), aa(D + 1), rr(D + 1);
        for (int d = 0; d <= D; ++d) {
          ae[d] = jb.be->a[d] + jb.be->e[d];
          aa[d] = jb.be->a[d];
          rr[d] = jb.be->r[d];
        }
        std::vector<Triple>* outv = &jobout[jj * kBuckets];
        const ScreenBound sb(c, L.maxb, tau, n > 0 ? ae.data() : rr.data(), D);
        // dz outermost: per target the triples of a term come in (dz, dy, dx) order
        const int Rz = sb.rz();
        for (int dz = -Rz; dz <= Rz; ++dz) {
          const int Ry = sb.ry(std::abs(dz));
          for (int dy = -Ry; dy <= Ry; ++dy) {
            const int Rx = sb.rx(std::abs(dy), std::abs(dz));
            for (int dx = -Rx; dx <= Rx; ++dx) {
              const double cN = screen_cn(c, n, ae.data(), aa.data(), rr.data(), std::abs(dx),
                                          std::abs(dy), std::abs(dz));
              if (cN * L.maxb < tau) continue;
              for (int64_t oi = 0; oi < L.np; ++oi) {
                int64_t p = L.order[oi];
                const double eta = cN * L.bn[p];
                if (!(eta >= tau)) break;
                int64_t tx = L.px[p] + dx, ty = L.py[p] + dy, tz = L.pz[p] + dz;
                if (tx < 0 || ty < 0 || tz < 0 || tx >= nb || ty >= nb || tz >= nb) continue;
                const int8_t low = (tiers && n > 0 && eta < tau_tier) ? 1 : 0;
                const uint64_t code = encode(n, tx, ty, tz);
                outv[target_bucket(n, code)].push_back({((uint64_t)n << 58) | code,
                                                        (int32_t)(L.ib + p), (int16_t)mu,
                                                        (int16_t)dx, (int16_t)dy, (int16_t)dz, low});
              }
            }
          }
        }
      });
      mark("enumerate");
      // group by target per (function, level, bucket) unit, largest units first
      units.clear();
      unit_lev.clear();
      for (size_t u = ua; u < ub; ++u) {
        const size_t jb0 = lu_j[u], je0 = lu_j[u + 1];
        for (int b = 0; b < kBuckets; ++b) {
          bool any = false;
          for (size_t q = jb0; q < je0 && !any; ++q) any = !jobout[(q - ja) * kBuckets + b].empty();
          if (!any) continue;
          Unit un;
          un.fn = lv[jobs[jb0].lev].fn;
          un.n = lv[jobs[jb0].lev].n;
          un.jb = jb0 - ja;
          un.je = je0 - ja;
          un.bucket = b;
          units.push_back(std::move(un));
          unit_lev.push_back(jobs[jb0].lev);
        }
      }
      std::vector<size_t> uorder(units.size());
      std::iota(uorder.begin(), uorder.end(), 0);
      {
        std::vector<size_t> usize(units.size(), 0);
        for (size_t i = 0; i < units.size(); ++i)
          for (size_t q = units[i].jb; q < units[i].je; ++q)
            usize[i] += jobout[q * kBuckets + units[i].bucket].size();
        std::stable_sort(uorder.begin(), uorder.end(),
                         [&](size_t a, size_t b) { return usize[a] > usize[b]; });
      }
      parallel_for(units.size(), [&](size_t ii, unsigned) {
        const size_t i = uorder[ii];
        group_unit(units[i], jobout, lv[unit_lev[i]], factored);
      });
      mark("group by target");
    };
    if (!pipelined) {
      enumerate_group(0, nlu);
      // the targets of each level-unit are the grouped target codes, in bucket order
      size_t u = 0;
      for (size_t q = 0; q < units.size(); ++q) {
        while (lu_j[u + 1] - j0 <= units[q].jb) ++u;
        for (uint64_t t : units[q].tcodes) lu_codes[u].push_back(t & ((1ULL << 58) - 1));
      }
    } else
    parallel_for(nlu, [&](size_t u, unsigned) {
      const LevelData& L = lv[jobs[lu_j[u]].lev];
      const Op& op = *ops[L.fn];
      const int n = L.n;
      const int64_t nb = (int64_t)1 << n;
      int Dm = 0;
      for (size_t j = lu_j[u]; j < lu_j[u + 1]; ++j) Dm = std::max(Dm, jobs[j].D);
      const size_t S1 = (size_t)Dm + 1;
      // max over the terms of c N, filled only where a term's pruning bound (ScreenBound)
      // can pass; the other entries stay 0 and would fail the test anyway.  lim_* record
      // the reach of the filled entries, so the scan below skips only zeros.
      std::vector<double> cn(S1 * S1 * S1, 0.0);   // [ax][ay][az]
      int lim_z = -1;
      std::vector<int> lim_y(S1, -1), lim_x(S1 * S1, -1);   // [az], [az][ay]
      for (size_t j = lu_j[u]; j < lu_j[u + 1]; ++j) {
        const Job& jb = jobs[j];
        const double c = std::fabs(op.c[jb.mu]);
        const int D = jb.D;
        std::vector<double> ae(D + 1), aa(D + 1), rr(D + 1);
        for (int d = 0; d <= D; ++d) {
          ae[d] = jb.be->a[d] + jb.be->e[d];
          aa[d] = jb.be->a[d];
          rr[d] = jb.be->r[d];
        }
        const ScreenBound sb(c, L.maxb, tau, n > 0 ? ae.data() : rr.data(), D);
        const int Rz = sb.rz();
        lim_z = std::max(lim_z, Rz);
        for (int az = 0; az <= Rz; ++az) {
          const int Ry = sb.ry(az);
          lim_y[az] = std::max(lim_y[az], Ry);
          for (int ay = 0; ay <= Ry; ++ay) {
            const int Rx = sb.rx(ay, az);
            lim_x[(size_t)az * S1 + ay] = std::max(lim_x[(size_t)az * S1 + ay], Rx);
            for (int ax = 0; ax <= Rx; ++ax) {
              double& m = cn[((size_t)ax * S1 + ay) * S1 + az];
              m = std::max(m, screen_cn(c, n, ae.data(), aa.data(), rr.data(), ax, ay, az));
            }
          }
        }
      }
      std::vector<uint64_t> codes;
      for (int dz = -lim_z; dz <= lim_z; ++dz)
        for (int dy = -lim_y[std::abs(dz)]; dy <= lim_y[std::abs(dz)]; ++dy)
          for (int dx = -lim_x[(size_t)std::abs(dz) * S1 + std::abs(dy)];
               dx <= lim_x[(size_t)std::abs(dz) * S1 + std::abs(dy)]; ++dx) {
            const double cN = cn[((size_t)std::abs(dx) * S1 + std::abs(dy)) * S1 + std::abs(dz)];
            if (cN * L.maxb < tau) continue;
            for (int64_t oi = 0; oi < L.np; ++oi) {
              const int64_t p = L.order[oi];
              if (!(cN * L.bn[p] >= tau)) break;
              const int64_t tx = L.px[p] + dx, ty = L.py[p] + dy, tz = L.pz[p] + dz;
              if (tx < 0 || ty < 0 || tz < 0 || tx >= nb || ty >= nb || tz >= nb) continue;
              codes.push_back(encode(n, tx, ty, tz));
            }
          }
      lu_weight[u] = (double)codes.size();
      radix_sort_unique(codes, 3 * n);
      lu_codes[u].swap(codes);
    });
    mark("target sets");
    // ---- 3. output trees of the sub-batch's functions
    parallel_for((size_t)(f1 - f0), [&](size_t ii, unsigned) {
      const int i = f0 + (int)ii;
      std::vector<uint64_t> tc;
      for (size_t u = 0; u < nlu; ++u) {
        const LevelData& L = lv[jobs[lu_j[u]].lev];
        if (L.fn != i) continue;
        for (uint64_t c : lu_codes[u]) tc.push_back(((uint64_t)L.n << 58) | c);
      }
      build_output_tree(ctx, plans[i], tc);
    });
    mark("output trees");
    // ---- 4. sub-batch data: level-n slots of the targets, sum-down entries, pointer tables
    std::vector<std::vector<int32_t>> sub_of_node(f1 - f0);
    int32_t nsub = 0;
    parallel_for((size_t)(f1 - f0), [&](size_t ii, unsigned) {
      sub_of_node[ii].assign((size_t)plans[f0 + (int)ii].out->nodes(), -1);
    });
    if (fused) {
      // slots numbered in unit order, each unit's targets in their sorted order: a unit's
      // first slot is the number of targets of the units before it (the units hold
      // disjoint target sets, so they are filled in parallel)
      std::vector<int64_t> uoff(nlu + 1, 0);
      for (size_t u = 0; u < nlu; ++u) {
        const LevelData& L = lv[jobs[lu_j[u]].lev];
        uoff[u + 1] = uoff[u] + (L.n == 0 ? 0 : (int64_t)lu_codes[u].size());
      }
      if (uoff[nlu] > INT32_MAX) fail(MRA_E_UNSUPPORTED, "too many level-n targets in one sub-batch");
      std::vector<char> missing(nlu, 0);
      parallel_for(nlu, [&](size_t u, unsigned) {
        const LevelData& L = lv[jobs[lu_j[u]].lev];
        if (L.n == 0) return;
        const Func& o = *plans[L.fn].out;
        int32_t slot = (int32_t)uoff[u];
        for (uint64_t c : lu_codes[u]) {
          const int64_t node = find_node(o, L.n, c);
          if (node < 0) {
            missing[u] = 1;
            return;
          }
          sub_of_node[L.fn - f0][node] = slot++;
        }
      });
      for (char m : missing)
        if (m) fail(MRA_E_INVALID, "internal plan error: target node");
      nsub = (int32_t)uoff[nlu];
    }
    mark("level-n slots");
    int out_maxlev = 0;
    for (int i = f0; i < f1; ++i) {
      in_leaves += (int64_t)plans[i].f->leaves.size();
      out_nodes += plans[i].out->nodes();
      out_leaves += (int64_t)plans[i].out->leaves.size();
      out_maxlev = std::max(out_maxlev, plans[i].out->nlev);
    }
    std::vector<NodeRef> sd_refs;
    std::vector<int64_t> sd_off(out_maxlev + 1, 0);
    for (int n = 0; n < out_maxlev; ++n) {
      for (int i = f0; i < f1; ++i) {
        const Func& o = *plans[i].out;
        if (n >= o.nlev) continue;
        for (int64_t q = o.inter_level_off[n]; q < o.inter_level_off[n + 1]; ++q)
          sd_refs.push_back({i, o.interior[q], o.first_child[o.interior[q]],
                             sub_of_node[i - f0][o.interior[q]]});
      }
      sd_off[n + 1] = (int64_t)sd_refs.size();
    }
    mark("sum-down lists");
    // device pointer tables (indexed by the batch position of a function; entries of other
    // sub-batches are not read)
    std::vector<double*> out_tab(nf, nullptr);
    std::vector<const double*> r_tab(nf), t_tab(nf), c_tab(nf);
    std::vector<const uint16_t*> l_tab(nf);
    std::vector<int64_t> out_len(nf, 0);
    size_t max_len = 0;
    for (int i = 0; i < nf; ++i) {
      r_tab[i] = plans[i].op->dR.p;
      t_tab[i] = plans[i].op->dT.p;
      c_tab[i] = plans[i].op->d_c.p;
      l_tab[i] = plans[i].op->dL.p;
      // the BF16 kernel addresses an operator's records with 32-bit byte offsets
      if (tiers && (double)plans[i].op->dL.n * sizeof(uint16_t) >= 2147483632.0)
        fail(MRA_E_UNSUPPORTED, "too many operator blocks for the low-precision tier");
    }
    for (int i = f0; i < f1; ++i) {
      Func& o = *plans[i].out;
      o.coeff.alloc(ctx, (size_t)o.nodes() * K3);
      o.device_leaves();
      out_tab[i] = o.coeff.p;
      out_len[i] = (int64_t)o.coeff.n;
      max_len = std::max(max_len, o.coeff.n);
    }
    mark("output storage");
    Arena& AS = ctx->arena[1 + (sb & 1)];
    AS.begin(ctx);
    const size_t o_out = AS.put(out_tab), o_r = AS.put(r_tab), o_t = AS.put(t_tab),
                 o_c = AS.put(c_tab), o_l = AS.put(l_tab), o_sd = AS.put(sd_refs),
                 o_olen = AS.put(out_len);
    const size_t o_subb = AS.scratch((size_t)nsub * K3 * sizeof(double));
    AS.commit();
    double* const* out_tab_d = AS.at<double*>(o_out);
    const double* const* r_tab_d = AS.at<const double*>(o_r);
    const double* const* t_tab_d = AS.at<const double*>(o_t);
    const double* const* c_tab_d = AS.at<const double*>(o_c);
    const uint16_t* const* l_tab_d = AS.at<const uint16_t*>(o_l);
    const NodeRef* sd_d = AS.at<NodeRef>(o_sd);
    double* subbuf_d = AS.scr_at<double>(o_subb);
    // outputs start at zero; so do the level-n slots (a target whose triples all run in the
    // low tier leaves its slot untouched)
    launch_zero_batch(out_tab_d + f0, AS.at<int64_t>(o_olen) + f0, f1 - f0, max_len, ctx->stream);
    launch_zero(subbuf_d, (size_t)nsub * K3, ctx->stream);
    mark("tables and zero fill");
    plan_ms += now_ms() - t_sb0;

    // ---- 5. chunks of level-units: enumerate, group, fill, upload and launch one chunk while
    // the device runs the previous ones.  A small first chunk starts the device early.
    std::vector<size_t> cb{0};
    if (pipelined) {
      double total = 0.0;
      for (double w : lu_weight) total += w;
      const double first = total / 8.0, rest = (total - first) / 3.0;
      double acc = 0.0, next = first;
      for (size_t u = 0; u < nlu; ++u) {
        acc += lu_weight[u];
        if (acc >= next && u + 1 < nlu && cb.size() < 4) {
          cb.push_back(u + 1);
          next = acc + rest;
        }
      }
      cb.push_back(nlu);
    } else {
      cb.push_back(nlu);
    }
    for (size_t ch = 0; ch + 1 < cb.size(); ++ch) {
      const size_t gc = cev.size();
      if (gc >= 2) hip_check(hipEventSynchronize(cev[gc - 2]->e[3]), "hipEventSynchronize");
      const double t_c0 = now_ms();
      t_mark = t_c0;
      if (pipelined) enumerate_group(cb[ch], cb[ch + 1]);
      // item offsets (per unit and target: FP64 items, then BF16 items), filled in parallel
      // over target chunks directly into the pinned upload buffer
      size_t n_items = 0, n_low = 0;
      for (Unit& u : units) {
        const size_t nt = u.tcodes.size();
        u.fpre.assign(nt + 1, 0);
        u.lpre.assign(nt + 1, 0);
        u.node.assign(nt, -1);
        for (size_t r = 0; r < nt; ++r) {
          u.fpre[r + 1] = u.fpre[r] + (u.tmid[r] - u.toff[r]);
          u.lpre[r + 1] = u.lpre[r] + (u.toff[r + 1] - u.tmid[r]);
        }
        u.item_base = n_items;
        u.low_base = n_low;
        n_items += (size_t)u.fpre[nt];
        n_low += (size_t)u.lpre[nt];
        const double per = f_ns + (u.n > 0 ? f_sub : 0.0);
        ntriples += (int64_t)u.sorted.size();
        ntargets += (int64_t)nt;
        flops += (double)u.sorted.size() * per;
        flops_low += (double)u.lpre[nt] * per;
      }
      if (n_items > (size_t)INT32_MAX || n_low > (size_t)INT32_MAX)
        fail(MRA_E_UNSUPPORTED, "too many triples for one apply");
      nlow += (int64_t)n_low;
      Arena& A1 = ctx->arena[3 + (gc & 1)];
      A1.begin(ctx);
      const size_t o_items = A1.reserve(n_items * sizeof(NSItem));
      const size_t o_litems = A1.reserve(n_low * sizeof(LowItem));
      NSItem* items_h = A1.host_at<NSItem>(o_items);
      LowItem* low_h = A1.host_at<LowItem>(o_litems);
      struct Task {
        size_t u;
        int64_t r0, r1;
      };
      std::vector<Task> tasks;
      for (size_t ui = 0; ui < units.size(); ++ui) {
        const Unit& u = units[ui];
        const int64_t nt = (int64_t)u.tcodes.size();
        for (int64_t r = 0; r < nt;) {
          int64_t e = r, cnt = 0;
          while (e < nt && cnt < 4096) cnt += u.toff[e + 1] - u.toff[e], ++e;
          tasks.push_back({ui, r, e});
          r = e;
        }
      }
      std::vector<double> task_eta(tasks.size(), 0.0), task_fk(tasks.size(), 0.0);
      // mode products the main kernel executes (before splitting long lists): per triple one
      // for a factored kernel, plus one per (term, dz, dy) and per (term, dz) group end
      const double fm = 2.0 * std::pow(2.0 * k, 4), fs = 2.0 * std::pow((double)k, 4);
      parallel_for(tasks.size(), [&](size_t ti, unsigned) {
        const Task& t = tasks[ti];
        Unit& u = units[t.u];
        const Plan& p = plans[u.fn];
        task_eta[ti] = fill_items(u, p, lv[unit_lev[t.u]], fu_index[u.fn], t.r0, t.r1, items_h,
                                  low_h, (int64_t)p.op->dR_blocks, (int64_t)p.op->dT_blocks,
                                  tiers ? (int64_t)p.op->dL_blocks : 0, (int64_t)fu_refs.size());
        const double per = fm + (fused && u.n > 0 ? fs : 0.0);
        double acc = 0.0;
        for (int64_t r = t.r0; r < t.r1; ++r) {
          const int64_t b = (int64_t)u.item_base + u.fpre[r], e = (int64_t)u.item_base + u.fpre[r + 1];
          int64_t prods = e - b;
          if (factored)
            for (int64_t q = b; q < e; ++q) {
              const bool last = q + 1 == e;
              const NSItem& a = items_h[q];
              if (last || items_h[q + 1].rz != a.rz || items_h[q + 1].ry != a.ry) ++prods;
              if (last || items_h[q + 1].rz != a.rz) ++prods;
            }
          else
            prods *= 3;
          acc += (double)prods * per;
        }
        task_fk[ti] = acc;
      });
      for (double v : task_fk) flops_kernel += v;   // fixed order
      for (double e : task_eta) eta_low += e;   // fixed order
      mark("work items");
      // the items are final: their copy to the device runs while the target ranges are built
      // (device room for the lists that follow is reserved from an upper bound on their size)
      {
        size_t nt_all = 0;
        for (const Unit& u : units) nt_all += u.tcodes.size();
        const size_t lists = 2 * ((3 * nt_all + n_items / 24 + 16) * sizeof(TargetRange) +
                                  (nt_all + 16) * sizeof(SplitTarget) + 4096);
        A1.prepare_device(A1.used + lists);
        A1.commit_upto(A1.used);
      }
      mark("items upload issued");
      // target ranges: split long lists, longest first
      std::vector<TargetRange> tgt_sub, work, low_work;
      std::vector<SplitTarget> splits;
      const int64_t div = std::max(1, ctx->sched_split_div);
      const int64_t chunk = std::max<int64_t>(24, ((int64_t)n_items + div - 1) / div);
      int32_t npartials = 0;
      for (const Unit& u : units) {
        const int i = u.fn;
        const Func& o = *plans[i].out;
        for (size_t r = 0; r < u.tcodes.size(); ++r) {
          const int32_t node = u.node[r], fc = o.first_child[node];
          const int32_t lb = (int32_t)(u.low_base + u.lpre[r]), le = (int32_t)(u.low_base + u.lpre[r + 1]);
          if (le > lb) low_work.push_back({i, node, fc, lb, le, -1, -1});
          const int32_t b = (int32_t)(u.item_base + u.fpre[r]), e = (int32_t)(u.item_base + u.fpre[r + 1]);
          if (e == b) continue;
          int32_t sub = -1;
          if (u.n > 0) {
            if (fused) {
              sub = sub_of_node[i - f0][node];
              if (sub < 0) fail(MRA_E_INVALID, "internal plan error: target outside the target set");
            } else {
              tgt_sub.push_back({i, node, fc, b, e, -1, -1});
            }
          }
          const int64_t len = e - b;
          if (len <= chunk) {
            work.push_back({i, node, fc, b, e, -1, sub});
            continue;
          }
          const int32_t parts = (int32_t)((len + chunk - 1) / chunk);
          for (int32_t q = 0; q < parts; ++q) {
            const int32_t qb = b + (int32_t)(q * len / parts), qe = b + (int32_t)((q + 1) * len / parts);
            work.push_back({i, node, fc, qb, qe, npartials + q, sub});
            // a part ends its groups: its last triple closes the y- and z-groups it is in
            if (factored && q + 1 < parts) {
              const NSItem& a = items_h[qe - 1];
              const NSItem& nb = items_h[qe];
              const double per = fm + (sub >= 0 ? fs : 0.0);
              if (nb.rz == a.rz && nb.ry == a.ry) flops_kernel += per;
              if (nb.rz == a.rz) flops_kernel += per;
            }
          }
          splits.push_back({i, fc, npartials, parts, sub});
          npartials += parts;
        }
      }
      auto by_len = [](const TargetRange& a, const TargetRange& b) {
        return (a.end - a.beg) > (b.end - b.beg);
      };
      std::stable_sort(work.begin(), work.end(), by_len);
      std::stable_sort(tgt_sub.begin(), tgt_sub.end(), by_len);
      std::stable_sort(low_work.begin(), low_work.end(), by_len);
      if (timing && !low_work.empty()) {
        int64_t tot = 0;
        for (const TargetRange& t : low_work) tot += t.end - t.beg;
        std::fprintf(stderr, "[mra] low-tier lists: %zu targets, %lld triples, longest %d, 10th %d\n",
                     low_work.size(), (long long)tot, low_work[0].end - low_work[0].beg,
                     low_work[std::min<size_t>(9, low_work.size() - 1)].end -
                         low_work[std::min<size_t>(9, low_work.size() - 1)].beg);
      }
      mark("target ranges");
      const size_t o_work = A1.put(work), o_sub = A1.put(tgt_sub), o_spl = A1.put(splits),
                   o_lwork = A1.put(low_work);
      const size_t o_part = A1.scratch((size_t)npartials * 9 * K3 * sizeof(double));  // (2k)^3 + k^3
      const size_t o_cnt = A1.scratch(256);   // work counter of the persistent kernel
      A1.commit();
      const NSItem* items_d = A1.at<NSItem>(o_items);
      const TargetRange* work_d = A1.at<TargetRange>(o_work);
      const TargetRange* sub_d = A1.at<TargetRange>(o_sub);
      const SplitTarget* splits_d = A1.at<SplitTarget>(o_spl);
      const LowItem* low_items_d = A1.at<LowItem>(o_litems);
      const TargetRange* low_work_d = A1.at<TargetRange>(o_lwork);
      double* partials_d = A1.scr_at<double>(o_part);
      int* counter_d = A1.scr_at<int>(o_cnt);
      mark("ranges + uploads");
      plan_ms += now_ms() - t_c0;
      // device work of the chunk
      cev.push_back(std::make_unique<Events>());
      hipEvent_t* E = cev.back()->e;
      hip_check(hipEventRecord(E[0], ctx->stream), "event");
      launch_apply_ns(k, in_tab_d, out_tab_d, items_d, work_d, (int)work.size(), r_tab_d,
                      t_tab_d, c_tab_d, partials_d, subbuf_d, counter_d, ctx->stream, slabs_d);
      hip_check(hipEventRecord(E[1], ctx->stream), "event");
      launch_reduce_partials(k, partials_d, out_tab_d, subbuf_d, splits_d,
                             (int)splits.size(), ctx->stream);
      launch_apply_std(k, in_tab_d, out_tab_d, items_d, sub_d, (int)tgt_sub.size(),
                       t_tab_d, c_tab_d, -1.0, ctx->stream);
      hip_check(hipEventRecord(E[2], ctx->stream), "event");
      if (!low_work.empty()) {
        any_low = true;
        ++n_low_launch;
        launch_apply_low(k, mirror_d, out_tab_d, low_items_d, low_work_d,
                         (int)low_work.size(), l_tab_d, c_tab_d, counter_d + 2, ctx->stream);
      }
      hip_check(hipEventRecord(E[3], ctx->stream), "event");
    }
    // ---- 6. sum-down of the sub-batch
    sev.push_back(std::make_unique<Events>());
    hipEvent_t* ES = sev.back()->e;
    hip_check(hipEventRecord(ES[0], ctx->stream), "event");
    for (int n = 0; n < out_maxlev; ++n) {
      int64_t b = sd_off[n], e = sd_off[n + 1];
      if (e > b)
        launch_sum_down(k, out_tab_d, sd_d + b, (int)(e - b), subbuf_d, h0p, h1p, ctx->stream);
    }
    hip_check(hipEventRecord(ES[1], ctx->stream), "event");
  }
  const double t_issued = now_ms();
  ctx->sync();
  if (timing)
    std::fprintf(stderr, "[mra] %-28s %8.3f ms\n[mra] %-28s %8.3f ms\n", "after plan to last launch",
                 t_issued - t_mark, "final wait", now_ms() - t_issued);
  for (int i = 0; i < nf; ++i) plans[i].out->interior_valid = false;

  float ms_f = 0;
  double ms_a = 0, ms_s = 0, ms_main = 0, ms_low = 0;
  hip_check(hipEventElapsedTime(&ms_f, ctx->ev[0], ctx->ev[1]), "elapsed");
  for (const auto& ce : cev) {
    float a = 0, m = 0, l = 0;
    hip_check(hipEventElapsedTime(&a, ce->e[0], ce->e[3]), "elapsed");
    hip_check(hipEventElapsedTime(&m, ce->e[0], ce->e[1]), "elapsed");
    hip_check(hipEventElapsedTime(&l, ce->e[2], ce->e[3]), "elapsed");
    ms_a += a;
    ms_main += m;
    ms_low += l;
  }
  for (const auto& se : sev) {
    float d = 0;
    hip_check(hipEventElapsedTime(&d, se->e[0], se->e[1]), "elapsed");
    ms_s += d;
  }
  mra_apply_stats& st = ctx->stats;
  st = mra_apply_stats{};
  st.triples = ntriples;
  st.targets = ntargets;
  st.in_leaves = in_leaves;
  st.out_nodes = out_nodes;
  st.out_leaves = out_leaves;
  st.useful_flops = flops;
  st.ms_filter = ms_f;
  st.ms_plan = plan_ms;
  st.ms_apply = ms_a;
  st.ms_main_kernel = ms_main;
  st.ms_sumdown = ms_s;
  st.triples_low = nlow;
  st.flops_low = flops_low;
  st.flops_kernel = flops_kernel;
  st.eta_low = eta_low;
  st.ms_low_kernel = any_low ? ms_low : 0.0;
  st.launches_main = (int64_t)cev.size();
  st.launches_low = n_low_launch;
  if (timing) std::fprintf(stderr, "[mra] %-28s %8.3f ms\n", "host total", now_ms() - t_entry);
}

// Filter-up of one function (used by mra_inner); returns nothing but marks it valid.
void filter_up_function(Ctx* ctx, Func& f) {
  if (f.interior_valid) return;
  std::vector<double> h0v, h1v;
  two_scale_filters(f.k, h0v, h1v);
  DevArray<double> h0, h1;
  h0.upload(ctx, h0v);
  h1.upload(ctx, h1v);
  std::vector<double*> tab{f.coeff.p};
  DevArray<double*> d_tab;
  d_tab.upload(ctx, tab);
  std::vector<NodeRef> refs;
  std::vector<int64_t> off;
  off.push_back(0);
  for (int n = f.nlev - 1; n >= 0; --n) {
    for (int64_t q = f.inter_level_off[n]; q < f.inter_level_off[n + 1]; ++q)
      refs.push_back({0, f.interior[q], f.first_child[f.interior[q]], -1});
    off.push_back((int64_t)refs.size());
  }
  DevArray<NodeRef> d_refs;
  d_refs.upload(ctx, refs);
  DevArray<double> d_bn2;
  d_bn2.alloc(ctx, std::max<size_t>(1, refs.size()));
  for (size_t j = 0; j + 1 < off.size(); ++j)
    if (off[j + 1] > off[j])
      launch_filter_up(f.k, d_tab.p, d_refs.p + off[j], (int)(off[j + 1] - off[j]), h0.p, h1.p,
                       d_bn2.p + off[j], nullptr, ctx->stream);
  ctx->sync();
  f.interior_valid = true;
}

}  // namespace mra
