// C ABI of libmra: contexts, functions, operators, the apply planner and reductions.
//
// mra_apply (non-standard form, Sec. 2.2-2.3) runs these steps on the context's stream:
//   1. filter-up (device): s_P and ||B_P||_F for every refined box, bottom-up;
//   2. screening (host, from the norms): triples (P, delta, mu) with
//      eta = |c_mu| N(delta) ||B_P||_F >= tau_drop, targets inside the cell;
//   3. output tree (targets, their children, ancestors, closed under siblings) and the
//      target-sorted work list; operator blocks missing from the cache are computed;
//   4. transform-and-accumulate (device): children blocks of every target, and the level-n
//      subtraction for targets below the root;
//   5. sum-down (device), level by level.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "mra_internal.hpp"

struct mra_ctx {
  mra::Ctx c;
};
struct mra_func {
  mra::Func f;
};
struct mra_op {
  mra::Op o;
};

namespace mra {

void fail(mra_status code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(MRA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* Ctx::dalloc(size_t bytes) {
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  if (alloc) {
    p = alloc(bytes, user);
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  }
  if (!p) fail(MRA_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  return p;
}

void Ctx::dfree(void* p) {
  if (!p) return;
  if (free_fn)
    free_fn(p, user);
  else
    (void)hipFree(p);
}

void Ctx::sync() { hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

// ------------------------------------------------------------------------------- pool
namespace {
thread_local bool t_in_pool = false;   // set on pool workers and on a caller inside run()
}

Pool& Pool::get() {
  static Pool pool;
  return pool;
}

Pool::Pool() {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned n = std::min(16u, hw);
  for (unsigned i = 1; i < n; ++i) th_.emplace_back([this, i] { loop(i); });
}

Pool::~Pool() {
  {
    std::lock_guard<std::mutex> lk(m_);
    stop_.store(true);
  }
  cv_.notify_all();
  for (auto& t : th_) t.join();
}

void Pool::work(unsigned id) {
  for (;;) {
    const size_t i = next_.fetch_add(1, std::memory_order_relaxed);
    if (i >= count_) break;
    try {
      (*fn_)(i, id);
    } catch (...) {
      std::lock_guard<std::mutex> lk(m_);
      if (!err_) err_ = std::current_exception();
    }
  }
}

// Workers spin briefly on the generation counter before sleeping, because the planner
// issues its loops in quick succession.
void Pool::loop(unsigned id) {
  t_in_pool = true;
  uint64_t seen = 0;
  for (;;) {
    for (int spin = 0; spin < 4000 && gen_.load(std::memory_order_acquire) == seen &&
                       !stop_.load(std::memory_order_relaxed);
         ++spin)
      std::this_thread::yield();
    if (gen_.load(std::memory_order_acquire) == seen) {
      std::unique_lock<std::mutex> lk(m_);
      cv_.wait(lk, [&] { return stop_.load() || gen_.load() != seen; });
    }
    if (stop_.load()) return;
    seen = gen_.load(std::memory_order_acquire);
    work(id);
    if (busy_.fetch_sub(1, std::memory_order_acq_rel) == 1) {
      std::lock_guard<std::mutex> lk(m_);
      done_.notify_one();
    }
  }
}

void Pool::run(size_t count, const std::function<void(size_t, unsigned)>& fn) {
  if (count == 0) return;
  if (th_.empty() || count == 1 || t_in_pool) {   // nested calls run serially
    for (size_t i = 0; i < count; ++i) fn(i, 0);
    return;
  }
  struct Flag {
    Flag() { t_in_pool = true; }
    ~Flag() { t_in_pool = false; }
  } flag;
  {
    std::lock_guard<std::mutex> lk(m_);
    fn_ = &fn;
    count_ = count;
    next_.store(0, std::memory_order_relaxed);
    busy_.store((unsigned)th_.size(), std::memory_order_relaxed);
    err_ = nullptr;
    gen_.fetch_add(1, std::memory_order_release);
  }
  cv_.notify_all();
  work(0);
  for (int spin = 0; spin < 4000 && busy_.load(std::memory_order_acquire) != 0; ++spin)
    std::this_thread::yield();
  std::exception_ptr e;
  {
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [&] { return busy_.load() == 0; });
    e = err_;
    fn_ = nullptr;
  }
  if (e) std::rethrow_exception(e);
}

// ------------------------------------------------------------------------------ arena
Arena::~Arena() {
  if (host) (void)hipHostFree(host);
  if (ctx) {
    ctx->dfree(dev);
    ctx->dfree(scr);
  }
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t Arena::reserve(size_t bytes) {
  const size_t off = used;
  const size_t end = align256(off + bytes);
  if (end > host_cap) {
    // host regions handed out earlier keep their offsets; their contents move with the buffer
    // (after copies already issued from the old buffer have finished)
    if (committed) ctx->sync();
    size_t cap = std::max<size_t>(end, host_cap + host_cap / 2);
    cap = std::max<size_t>(cap, (size_t)1 << 20);
    void* p = nullptr;
    hip_check(hipHostMalloc(&p, cap, hipHostMallocDefault), "hipHostMalloc");
    if (host) {
      std::memcpy(p, host, used);
      (void)hipHostFree(host);
    }
    host = static_cast<char*>(p);
    host_cap = cap;
  }
  used = end;
  return off;
}

size_t Arena::put_bytes(const void* src, size_t bytes) {
  const size_t off = reserve(bytes);
  if (bytes) std::memcpy(host + off, src, bytes);
  return off;
}

size_t Arena::scratch(size_t bytes) {
  const size_t off = scr_used;
  scr_used = align256(off + bytes);
  return off;
}

static void arena_grow(Ctx* ctx, char*& buf, size_t& cap, size_t need) {
  if (need <= cap) return;
  ctx->sync();   // nothing may still use the old buffer
  ctx->dfree(buf);
  buf = nullptr;
  cap = 0;
  size_t c = std::max<size_t>(need, (size_t)1 << 20);
  buf = static_cast<char*>(ctx->dalloc(c));
  cap = c;
}

void Arena::prepare_device(size_t bytes) {
  if (bytes > dev_cap) {
    arena_grow(ctx, dev, dev_cap, bytes);
    committed = 0;   // a new buffer holds nothing yet
  }
}

void Arena::commit_upto(size_t end) {
  end = std::min(end, used);
  if (end <= committed) return;
  prepare_device(used);
  hip_check(hipMemcpyAsync(dev + committed, host + committed, end - committed,
                           hipMemcpyHostToDevice, ctx->stream),
            "hipMemcpyAsync H2D");
  committed = end;
}

void Arena::commit() {
  if (used > dev_cap) {
    arena_grow(ctx, dev, dev_cap, used);
    committed = 0;
  }
  arena_grow(ctx, scr, scr_cap, scr_used);
  commit_upto(used);
}

// ------------------------------------------------------------------------ block cache
static void transpose_into(int m, const double* a, double* out) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) out[j * m + i] = a[i * m + j];
}

const BlockEntry& Op::ensure(int level, int mu, int D) {
  // direct index in front of the map (its nodes never move)
  const size_t M = c.size(), slot = (size_t)level * M + (size_t)mu;
  if (slot < entry_at.size() && entry_at[slot] && entry_at[slot]->D >= D) return *entry_at[slot];
  BlockEntry& e = entries[{level, mu}];
  if (entry_at.size() <= slot) entry_at.resize((size_t)(level + 1) * M, nullptr);
  entry_at[slot] = &e;
  if (e.D >= D) return e;
  const int K2 = k * k, N = 2 * k, N2 = N * N;
  double W = ctx->width();
  double h = W / std::ldexp(1.0, level), hf = W / std::ldexp(1.0, level + 1);
  double texp = t[mu];
  // fine blocks t^{n+1, d} for d in [-2D-1, 2D+1] (t^{-d} = (t^d)^T)
  int F = 2 * D + 1;
  std::vector<double> fine((size_t)(2 * F + 1) * K2);
  for (int d = 0; d <= F; ++d) {
    block_t(k, hf, d, texp, &fine[(size_t)(d + F) * K2]);
    if (d > 0) transpose_into(k, &fine[(size_t)(d + F) * K2], &fine[(size_t)(F - d) * K2]);
  }
  std::vector<double> coarse((size_t)(2 * D + 1) * K2);
  for (int d = 0; d <= D; ++d) {
    block_t(k, h, d, texp, &coarse[(size_t)(d + D) * K2]);
    if (d > 0) transpose_into(k, &coarse[(size_t)(d + D) * K2], &coarse[(size_t)(D - d) * K2]);
  }
  std::vector<double> h0, h1;
  two_scale_filters(k, h0, h1);
  e.D = D;
  e.a.assign(D + 1, 0.0);
  e.e.assign(D + 1, 0.0);
  e.r.assign(D + 1, 0.0);
  e.r_base = (int64_t)(hR.size() / N2);
  e.t_base = (int64_t)(hT.size() / K2);
  std::vector<double> R(N2), P(N2), tmp(N2);
  for (int d = -D; d <= D; ++d) {
    // R rows (b, i) target child, columns (a, j) source child: block t^{n+1, 2d + b - a}
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const double* src = &fine[(size_t)(2 * d + b - a + F) * K2];
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < k; ++j) R[(b * k + i) * N + a * k + j] = src[i * k + j];
      }
    const double* tc = &coarse[(size_t)(d + D) * K2];
    size_t off = hR.size();
    hR.resize(off + N2);
    transpose_into(N, R.data(), &hR[off]);
    size_t offt = hT.size();
    hT.resize(offt + K2);
    transpose_into(k, tc, &hT[offt]);
    if (d >= 0) {
      // P = H^T t H with H = [h0 | h1] (k x 2k)
      for (int X = 0; X < N; ++X)
        for (int j = 0; j < k; ++j) {
          double s = 0.0;
          for (int i = 0; i < k; ++i) {
            double hix = X < k ? h0[i * k + X] : h1[i * k + X - k];
            s += hix * tc[i * k + j];
          }
          tmp[X * k + j] = s;   // (H^T t)[X][j]
        }
      for (int X = 0; X < N; ++X)
        for (int Y = 0; Y < N; ++Y) {
          double s = 0.0;
          for (int j = 0; j < k; ++j) {
            double hjy = Y < k ? h0[j * k + Y] : h1[j * k + Y - k];
            s += tmp[X * k + j] * hjy;
          }
          P[X * N + Y] = R[X * N + Y] - s;
        }
      e.a[d] = spectral_norm(k, tc);
      e.e[d] = spectral_norm(N, P.data());
      e.r[d] = spectral_norm(N, R.data());
    }
  }
  return e;
}

uint16_t bf16_bits(double v) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, sizeof u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Slot s of a permuted row holds column 4g + j (j < 4) or 16 + 4g + j - 4 (j >= 4),
// g = s / 8, j = s % 8: the row order of two stacked 16-row results of a BF16 matrix-core
// product, so that such a result can be fed back as the contracted operand unchanged.
static int low_perm(int s) {
  const int g = s / 8, j = s % 8;
  return j < 4 ? 4 * g + j : 16 + 4 * g + j - 4;
}

void Op::ensure_low() {
  const int N = 2 * k, K2 = k * k, N2 = N * N, UP = low_up(k);
  const size_t REC = low_record(k);
  const size_t nb = hR.size() / N2;
  if (hL_blocks >= nb) return;
  std::vector<double> h0, h1;
  two_scale_filters(k, h0, h1);
  std::vector<double> H((size_t)k * N);   // H[i][X] = [h0 | h1]
  for (int i = 0; i < k; ++i)
    for (int X = 0; X < N; ++X) H[i * N + X] = X < k ? h0[i * k + X] : h1[i * k + X - k];
  hL.resize(nb * REC);
  const size_t first = hL_blocks;
  auto one = [&](size_t b) {
    std::vector<double> R(N2), P(N2), E(N2), Ht((size_t)N * k);
    const double* RT = &hR[b * N2];   // RT[i][a] = R[a][i]
    const double* tT = &hT[b * K2];   // tT[j][i] = t[i][j]
    for (int a = 0; a < N; ++a)
      for (int i = 0; i < N; ++i) R[a * N + i] = RT[i * N + a];
    for (int X = 0; X < N; ++X)       // (H^T t)[X][j]
      for (int j = 0; j < k; ++j) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += H[i * N + X] * tT[j * k + i];
        Ht[X * k + j] = s;
      }
    for (int X = 0; X < N; ++X)
      for (int Y = 0; Y < N; ++Y) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += Ht[X * k + j] * H[j * N + Y];
        P[X * N + Y] = s;
        E[X * N + Y] = R[X * N + Y] - s;
      }
    const double* mats[3] = {R.data(), E.data(), P.data()};
    uint16_t* rec = &hL[b * REC];
    for (int m = 0; m < 3; ++m) {
      uint16_t* u = rec + (size_t)m * N * UP;
      uint16_t* v = rec + (size_t)3 * N * UP + (size_t)m * N * 32;
      for (int row = 0; row < N; ++row) {
        for (int col = 0; col < UP; ++col)
          u[row * UP + col] = col < N ? bf16_bits(mats[m][row * N + col]) : 0;
        for (int sl = 0; sl < 32; ++sl) {
          const int col = low_perm(sl);
          v[row * 32 + sl] = col < N ? bf16_bits(mats[m][row * N + col]) : 0;
        }
      }
    }
  };
  const size_t count = nb - first, per = 64;
  Pool::get().run((count + per - 1) / per, [&](size_t c, unsigned) {
    for (size_t b = first + c * per; b < std::min(nb, first + (c + 1) * per); ++b) one(b);
  });
  hL_blocks = nb;
}

void Op::sync_device() {
  const size_t N2 = (size_t)4 * k * k, K2 = (size_t)k * k;
  size_t nR = hR.size() / N2, nT = hT.size() / K2;
  if (nR == dR_blocks && nT == dT_blocks && hL_blocks == dL_blocks) return;
  // grow: re-upload everything (blocks are appended; kernels in flight use the old copy,
  // so synchronise before freeing it)
  ctx->sync();
  if (nR != dR_blocks || nT != dT_blocks) {
    dR.upload(ctx, hR);
    dT.upload(ctx, hT);
    dR_blocks = nR;
    dT_blocks = nT;
  }
  if (hL_blocks != dL_blocks) {
    std::vector<uint16_t> part(hL.begin(), hL.begin() + hL_blocks * low_record(k));
    dL.upload(ctx, part);
    dL_blocks = hL_blocks;
  }
}

// ------------------------------------------------------------------------ helpers
static double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Bit b of v (v < 2^21) moved to bit 3b, and back: the usual shift-and-mask spreading.
static inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
static inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ULL;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
  v = (v ^ (v >> 32)) & 0x1fffffULL;
  return v;
}
static void decode(uint64_t code, int n, int64_t& x, int64_t& y, int64_t& z) {
  const uint64_t c = n >= 21 ? code : code & ((1ULL << (3 * n)) - 1);
  x = (int64_t)compact3(c >> 2);
  y = (int64_t)compact3(c >> 1);
  z = (int64_t)compact3(c);
}

static uint64_t encode(int n, int64_t x, int64_t y, int64_t z) {
  const uint64_t m = n >= 21 ? 0x1fffffULL : (1ULL << n) - 1;
  return spread3((uint64_t)x & m) << 2 | spread3((uint64_t)y & m) << 1 | spread3((uint64_t)z & m);
}

static int64_t find_node(const Func& f, int n, uint64_t code) {
  if (n >= f.nlev) return -1;
  auto beg = f.code.begin() + f.level_off[n], end = f.code.begin() + f.level_off[n + 1];
  auto it = std::lower_bound(beg, end, code);
  if (it == end || *it != code) return -1;
  return it - f.code.begin();
}

// ------------------------------------------------------------------------ apply (std)
static void apply_standard(Ctx* ctx, Op& op, Func& f, int radius, Func& out) {
  const int k = f.k;
  if (f.leaves.empty()) fail(MRA_E_INVALID, "empty function");
  int L = f.level_of(f.leaves[0]);
  for (int32_t l : f.leaves)
    if (f.level_of(l) != L) fail(MRA_E_INVALID, "standard form needs a uniform tree");
  if (radius < 0) fail(MRA_E_INVALID, "disp_radius must be >= 0");
  const int64_t nb = (int64_t)1 << L;
  const int M = (int)op.c.size();
  int D = (int)std::min<int64_t>(radius, nb - 1);
  for (int mu = 0; mu < M; ++mu) op.ensure(L, mu, D);
  double t_plan0 = now_ms();
  // output: same structure
  out.ctx = ctx;
  out.k = k;
  out.nlev = f.nlev;
  out.level_off = f.level_off;
  out.code = f.code;
  out.first_child = f.first_child;
  out.finalize_structure();
  // the level is complete (all nb^3 boxes present), so its codes are 0 .. nb^3 - 1 in order
  // and the node of Morton code c is level_off[L] + c
  if (f.level_off[L + 1] - f.level_off[L] != nb * nb * nb)
    fail(MRA_E_INVALID, "standard form needs a complete uniform level");
  std::vector<int64_t> tb(M);   // t block of displacement 0 per term
  for (int mu = 0; mu < M; ++mu) {
    const BlockEntry& be = op.entries.at({L, mu});
    tb[mu] = be.t_base + be.D;
  }
  op.sync_device();
  // items per target (displacements that stay in the cube, times the terms), then the
  // items themselves in parallel, in (dx, dy, dz, mu) order per target
  const size_t nt = f.leaves.size();
  auto span = [&](int64_t x) { return std::min<int64_t>(x, D) + std::min<int64_t>(nb - 1 - x, D) + 1; };
  std::vector<int64_t> start(nt + 1, 0);
  std::vector<TargetRange> tgt(nt);
  for (size_t q = 0; q < nt; ++q) {
    int64_t x, y, z;
    decode(f.code[f.leaves[q]], L, x, y, z);
    start[q + 1] = start[q] + span(x) * span(y) * span(z) * M;
  }
  if (start[nt] > INT32_MAX) fail(MRA_E_UNSUPPORTED, "standard form: too many items");
  // the items are written straight into the context's pinned staging buffer and copied
  // with the tables in one asynchronous transfer
  Arena& A = ctx->arena[1];
  A.begin(ctx);
  const size_t o_items = A.reserve((size_t)start[nt] * sizeof(NSItem));
  NSItem* const items = A.host_at<NSItem>(o_items);
  const size_t nitems = (size_t)start[nt];
  std::atomic<bool> bad{false};
  Pool::get().run(nt, [&](size_t q, unsigned) {
    const int32_t T = f.leaves[q];
    int64_t x, y, z;
    decode(f.code[T], L, x, y, z);
    tgt[q] = TargetRange{0, T, -1, (int32_t)start[q], (int32_t)start[q + 1], -1, -1};
    NSItem* out_it = items + start[q];
    for (int dx = -D; dx <= D; ++dx)
      for (int dy = -D; dy <= D; ++dy)
        for (int dz = -D; dz <= D; ++dz) {
          const int64_t sx = x - dx, sy = y - dy, sz = z - dz;
          if (sx < 0 || sy < 0 || sz < 0 || sx >= nb || sy >= nb || sz >= nb) continue;
          const int64_t S = f.level_off[L] + (int64_t)encode(L, sx, sy, sz);
          for (int mu = 0; mu < M; ++mu) {
            NSItem it{};
            it.src = (int32_t)S;
            it.src_fc = -1;
            it.mu = mu;
            it.tx = (int32_t)(tb[mu] + dx);
            it.ty = (int32_t)(tb[mu] + dy);
            it.tz = (int32_t)(tb[mu] + dz);
            if (it.src >= f.nodes() || it.tx < 0 || it.ty < 0 || it.tz < 0 ||
                it.tx >= (int64_t)op.dT_blocks || it.ty >= (int64_t)op.dT_blocks ||
                it.tz >= (int64_t)op.dT_blocks)
              bad = true;
            *out_it++ = it;
          }
        }
    if (out_it != items + start[q + 1]) bad = true;
  });
  if (bad) fail(MRA_E_INVALID, "internal plan error: standard-form item");
  out.coeff.alloc(ctx, (size_t)out.nodes() * k * k * k);
  out.device_leaves();
  std::vector<const double*> in_tab{f.coeff.p}, t_tab{op.dT.p}, c_tab{op.d_c.p};
  std::vector<double*> out_tab{out.coeff.p};
  const size_t o_tgt = A.put(tgt), o_in = A.put(in_tab), o_t = A.put(t_tab),
               o_c = A.put(c_tab), o_out = A.put(out_tab);
  A.commit();
  double t_plan1 = now_ms();
  launch_zero(out.coeff.p, out.coeff.n, ctx->stream);
  hip_check(hipEventRecord(ctx->ev[2], ctx->stream), "event");
  launch_apply_std(k, A.at<const double*>(o_in), A.at<double*>(o_out), A.at<NSItem>(o_items),
                   A.at<TargetRange>(o_tgt), (int)tgt.size(), A.at<const double*>(o_t),
                   A.at<const double*>(o_c), 1.0, ctx->stream,
                   (int)std::min<int64_t>((int64_t)op.dT_blocks * k * k, INT32_MAX));
  hip_check(hipEventRecord(ctx->ev[3], ctx->stream), "event");
  ctx->sync();
  float ms_a = 0;
  hip_check(hipEventElapsedTime(&ms_a, ctx->ev[2], ctx->ev[3]), "elapsed");
  mra_apply_stats& st = ctx->stats;
  st = mra_apply_stats{};
  st.triples = (int64_t)nitems;
  st.targets = (int64_t)tgt.size();
  st.in_leaves = (int64_t)f.leaves.size();
  st.out_nodes = out.nodes();
  st.out_leaves = (int64_t)out.leaves.size();
  st.useful_flops = (double)nitems * 6.0 * std::pow((double)k, 4);
  st.flops_kernel = st.useful_flops;
  st.ms_plan = t_plan1 - t_plan0;
  st.ms_apply = ms_a;
  st.ms_main_kernel = ms_a;
  st.launches_main = 1;
}

// ------------------------------------------------------------------------ reductions
// Fixed-order reduction over leaves: 2048 workgroup partials, summed in order on the host.
// la_dev (optional) is a device copy of la.
static double reduce(Ctx* ctx, int k, const double* a, const double* b,
                     const std::vector<int32_t>& la, const std::vector<int32_t>* lb,
                     const std::vector<double>* w, int mode, const int32_t* la_dev = nullptr) {
  if (la.empty()) return 0.0;
  const int nblocks = 2048;
  DevArray<int32_t> d_la, d_lb;
  DevArray<double> d_w;
  if (!la_dev) {
    d_la.upload(ctx, la);
    la_dev = d_la.p;
  }
  if (lb) d_lb.upload(ctx, *lb);
  if (w) d_w.upload(ctx, *w);
  if (!ctx->red_part) ctx->red_part = static_cast<double*>(ctx->dalloc(nblocks * sizeof(double)));
  launch_leaf_reduce(k, a, b, la_dev, lb ? d_lb.p : nullptr, w ? d_w.p : nullptr,
                     (int)la.size(), mode, ctx->red_part, nblocks, ctx->stream);
  std::vector<double> part(nblocks);
  hip_check(hipMemcpyAsync(part.data(), ctx->red_part, nblocks * sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync D2H");
  ctx->sync();
  double s = 0.0;
  for (double v : part) s += v;
  return s;
}

}  // namespace mra

// =========================================================================== C ABI
using namespace mra;

#define MRA_TRY(ctxptr, ...)                                   \
  try {                                                        \
    __VA_ARGS__;                                               \
    return MRA_OK;                                             \
  } catch (const Error& e) {                                   \
    if (ctxptr) (ctxptr)->err = e.msg;                         \
    return e.code;                                             \
  } catch (const std::bad_alloc&) {                            \
    if (ctxptr) (ctxptr)->err = "host allocation failed";      \
    return MRA_E_NOMEM;                                        \
  } catch (const std::exception& e) {                          \
    if (ctxptr) (ctxptr)->err = e.what();                      \
    return MRA_E_INVALID;                                      \
  }

extern "C" {

static thread_local std::string g_create_error;

mra_status mra_ctx_create(int device, void* stream, mra_alloc_fn alloc, mra_free_fn free_fn,
                          void* user, double cell_lo, double cell_hi, mra_ctx** out) {
  g_create_error.clear();
  if (!out || !(cell_hi > cell_lo) || ((alloc == nullptr) != (free_fn == nullptr))) {
    g_create_error = "mra_ctx_create: bad arguments";
    return MRA_E_INVALID;
  }
  mra_ctx* h = nullptr;
  try {
    h = new mra_ctx();
    Ctx& c = h->c;
    c.device = device;
    c.stream = (hipStream_t)stream;
    c.alloc = alloc;
    c.free_fn = free_fn;
    c.user = user;
    c.lo = cell_lo;
    c.hi = cell_hi;
    hip_check(hipSetDevice(device), "hipSetDevice");
    for (auto& e : c.ev) hip_check(hipEventCreate(&e), "hipEventCreate");
    static_scratch_init(device);   // this device's address of the allocation-free scratch
    *out = h;
    return MRA_OK;
  } catch (const Error& e) {
    delete h;
    g_create_error = e.msg;
    return e.code;
  } catch (...) {
    delete h;
    g_create_error = "mra_ctx_create: allocation failed";
    return MRA_E_NOMEM;
  }
}

mra_status mra_ctx_free(mra_ctx* ctx) {
  if (!ctx) return MRA_E_INVALID;
  for (auto& e : ctx->c.ev)
    if (e) (void)hipEventDestroy(e);
  ctx->c.dfree(ctx->c.red_part);
  delete ctx;
  return MRA_OK;
}

const char* mra_last_error(const mra_ctx* ctx) {
  return ctx ? ctx->c.err.c_str() : g_create_error.c_str();
}

namespace {
void need_scaling(const mra::Func& f, const char* what) {
  if (f.wavelet_form)
    mra::fail(MRA_E_INVALID, std::string(what) + ": the function is in wavelet form");
}
}  // namespace

mra_status mra_project(mra_ctx* ctx, const mra_gaussian* g, int ng,
                       const mra_project_params* p, mra_func** out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!g || ng < 1 || !p || !out) fail(MRA_E_INVALID, "mra_project: bad arguments");
    if (p->k < 2 || p->k > kMaxK) fail(MRA_E_INVALID, "k must be in [2, 14]");
    if (!(p->thresh > 0.0)) fail(MRA_E_INVALID, "thresh must be > 0");
    if (p->initial_level < 0 || p->max_level > kMaxLevel || p->initial_level > p->max_level)
      fail(MRA_E_INVALID, "need 0 <= initial_level <= max_level <= 20");
    for (int i = 0; i < ng; ++i)
      if (!(g[i].expnt > 0.0)) fail(MRA_E_INVALID, "Gaussian exponents must be > 0");
    if (ng > 4096) fail(MRA_E_UNSUPPORTED, "mra_project takes at most 4096 Gaussians");
    std::unique_ptr<mra_func> h(new mra_func());
    project_gaussians_device(c, g, ng, p->k, p->thresh, p->initial_level, p->max_level, h->f);
    h->f.device_leaves();
    c->sync();
    *out = h.release();
  });
}

mra_status mra_func_info(const mra_func* f, int* k, int64_t* nodes, int64_t* leaves,
                         int* max_level) {
  if (!f) return MRA_E_INVALID;
  if (k) *k = f->f.k;
  if (nodes) *nodes = f->f.nodes();
  if (leaves) *leaves = (int64_t)f->f.leaves.size();
  if (max_level) *max_level = f->f.nlev - 1;
  return MRA_OK;
}

mra_status mra_func_export(mra_ctx* ctx, const mra_func* fh, int64_t cap, uint64_t* keys,
                           double* coeffs, int64_t* nleaves) {
  if (!ctx || !fh) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    const Func& f = fh->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    need_scaling(f, "mra_func_export");
    int64_t nl = (int64_t)f.leaves.size();
    if (nleaves) *nleaves = nl;
    if (keys || coeffs) {
      if (cap < nl) fail(MRA_E_INVALID, "export capacity too small");
      const size_t k3 = (size_t)f.k * f.k * f.k;
      std::vector<double> all;
      if (coeffs) {
        all.resize((size_t)f.nodes() * k3);
        hip_check(hipMemcpyAsync(all.data(), f.coeff.p, all.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream),
                  "hipMemcpyAsync D2H");
        c->sync();
      }
      for (int64_t i = 0; i < nl; ++i) {
        int32_t node = f.leaves[i];
        int n = f.level_of(node);
        if (keys) keys[i] = (1ULL << (3 * n)) | f.code[node];
        if (coeffs) std::memcpy(coeffs + i * k3, all.data() + (size_t)node * k3, k3 * sizeof(double));
      }
    }
  });
}

mra_status mra_func_free(mra_func* f) {
  if (!f) return MRA_E_INVALID;
  delete f;
  return MRA_OK;
}

mra_status mra_func_repr(const mra_func* f, int* repr) {
  if (!f || !repr) return MRA_E_INVALID;
  *repr = f->f.wavelet_form ? MRA_REPR_WAVELET : MRA_REPR_SCALING;
  return MRA_OK;
}

mra_status mra_compress(mra_ctx* ctx, const mra_func* fh, mra_func** out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !out) fail(MRA_E_INVALID, "mra_compress: bad arguments");
    const Func& f = fh->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    need_scaling(f, "mra_compress");
    std::unique_ptr<mra_func> h(new mra_func());
    compress_function(c, f, h->f);
    *out = h.release();
  });
}

mra_status mra_reconstruct(mra_ctx* ctx, const mra_func* ch, mra_func** out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!ch || !out) fail(MRA_E_INVALID, "mra_reconstruct: bad arguments");
    const Func& f = ch->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    if (!f.wavelet_form) fail(MRA_E_INVALID, "mra_reconstruct: the function is in scaling form");
    std::unique_ptr<mra_func> h(new mra_func());
    reconstruct_function(c, f, h->f);
    h->f.device_leaves();
    c->sync();
    *out = h.release();
  });
}

mra_status mra_truncate(mra_ctx* ctx, const mra_func* fh, double tol, mra_func** out,
                        double* removed2) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !out || !(tol >= 0.0)) fail(MRA_E_INVALID, "mra_truncate: bad arguments");
    const Func& f = fh->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    need_scaling(f, "mra_truncate");
    std::unique_ptr<mra_func> h(new mra_func());
    double rem = 0.0;
    truncate_function(c, f, tol, h->f, rem);
    if (removed2) *removed2 = rem;
    *out = h.release();
  });
}

mra_status mra_func_export_nodes(mra_ctx* ctx, const mra_func* fh, int64_t cap,
                                 uint64_t* keys, double* coeffs, int64_t* nnodes) {
  if (!ctx || !fh) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    Func& f = const_cast<mra_func*>(fh)->f;   // scaling form: interior slabs are filled
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    const int64_t nn = f.nodes();
    if (nnodes) *nnodes = nn;
    if (keys || coeffs) {
      if (cap < nn) fail(MRA_E_INVALID, "export capacity too small");
      if (coeffs) {
        if (!f.wavelet_form) filter_up_function(c, f);
        hip_check(hipMemcpyAsync(coeffs, f.coeff.p, (size_t)nn * f.k * f.k * f.k * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream),
                  "hipMemcpyAsync D2H");
        c->sync();
      }
      if (keys)
        for (int64_t i = 0; i < nn; ++i)
          keys[i] = (1ULL << (3 * f.level_of(i))) | f.code[i];
    }
  });
}

static mra_status make_op(mra_ctx* ctx, int k, const std::vector<double>& cc,
                          const std::vector<double>& tt, mra_op** out) {
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (k < 2 || k > kMaxK) fail(MRA_E_INVALID, "k must be in [2, 14]");
    if (cc.empty() || cc.size() > 32767) fail(MRA_E_INVALID, "need 1 <= M <= 32767 terms");
    for (double t : tt)
      if (!(t > 0.0)) fail(MRA_E_INVALID, "operator exponents must be > 0");
    std::unique_ptr<mra_op> h(new mra_op());
    h->o.ctx = c;
    h->o.k = k;
    h->o.c = cc;
    h->o.t = tt;
    h->o.d_c.upload(c, cc);
    c->sync();
    *out = h.release();
  });
}

mra_status mra_op_coulomb(mra_ctx* ctx, int k, double lo, double eps, mra_op** out) {
  if (!ctx || !out) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  std::vector<double> cc, tt;
  try {
    fit_coulomb(lo, eps, std::sqrt(3.0) * c->width(), cc, tt);
  } catch (const Error& e) {
    c->err = e.msg;
    return e.code;
  }
  return make_op(ctx, k, cc, tt, out);
}

mra_status mra_op_bsh(mra_ctx* ctx, int k, double mu, double lo, double eps, mra_op** out) {
  if (!ctx || !out) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  std::vector<double> cc, tt;
  try {
    fit_bsh(mu, lo, eps, std::sqrt(3.0) * c->width(), cc, tt);
  } catch (const Error& e) {
    c->err = e.msg;
    return e.code;
  }
  return make_op(ctx, k, cc, tt, out);
}

mra_status mra_op_gaussians(mra_ctx* ctx, int k, int M, const double* cv, const double* tv,
                            mra_op** out) {
  if (!ctx || !out || M < 1 || !cv || !tv) {
    if (ctx) ctx->c.err = "mra_op_gaussians: bad arguments";
    return MRA_E_INVALID;
  }
  return make_op(ctx, k, std::vector<double>(cv, cv + M), std::vector<double>(tv, tv + M), out);
}

mra_status mra_op_terms(const mra_op* op, int* M, double* c, double* t) {
  if (!op) return MRA_E_INVALID;
  if (M) *M = (int)op->o.c.size();
  if (c) std::copy(op->o.c.begin(), op->o.c.end(), c);
  if (t) std::copy(op->o.t.begin(), op->o.t.end(), t);
  return MRA_OK;
}

mra_status mra_op_free(mra_op* op) {
  if (!op) return MRA_E_INVALID;
  delete op;
  return MRA_OK;
}

namespace {
void check_nonstandard(int k, const mra_apply_params& p) {
  using namespace mra;
  if (k > 10 && k != 12 && k != 14)
    fail(MRA_E_UNSUPPORTED, "non-standard apply is built for k <= 10, 12 and 14");
  if (!(p.tau_drop >= 0.0)) fail(MRA_E_INVALID, "tau_drop must be >= 0");
  if (!(p.tau_tier >= 0.0)) fail(MRA_E_INVALID, "tau_tier must be >= 0");
  if (p.tau_tier > 0.0) {
    if (p.low_precision != MRA_LOW_BF16) fail(MRA_E_INVALID, "unknown low_precision");
    if (!low_kernel_available(k))
      fail(MRA_E_UNSUPPORTED, "the low-precision tier is built for k = 10, 12, 14");
  }
}
}  // namespace

mra_status mra_apply(mra_ctx* ctx, const mra_op* oph, const mra_func* fh,
                     const mra_apply_params* p, mra_func** out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!oph || !fh || !p || !out) fail(MRA_E_INVALID, "mra_apply: bad arguments");
    Op& op = const_cast<mra_op*>(oph)->o;          // the block cache is mutable state
    Func& f = const_cast<mra_func*>(fh)->f;        // refined-box slabs are workspace
    if (op.ctx != c || f.ctx != c) fail(MRA_E_MISMATCH, "handles belong to another context");
    if (op.k != f.k) fail(MRA_E_MISMATCH, "operator and function have different k");
    need_scaling(f, "mra_apply");
    std::unique_ptr<mra_func> h(new mra_func());
    if (p->form == MRA_FORM_STANDARD) {
      apply_standard(c, op, f, p->disp_radius, h->f);
    } else if (p->form == MRA_FORM_NONSTANDARD) {
      check_nonstandard(f.k, *p);
      apply_nonstandard_batch(c, {&op}, {&f}, p->tau_drop, p->tau_tier, {&h->f});
    } else {
      fail(MRA_E_INVALID, "unknown form");
    }
    *out = h.release();
  });
}

mra_status mra_apply_batch(mra_ctx* ctx, int n, const mra_op* const* ophs,
                           const mra_func* const* fhs, const mra_apply_params* p,
                           mra_func** outs) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (n < 1 || !ophs || !fhs || !p || !outs) fail(MRA_E_INVALID, "mra_apply_batch: bad arguments");
    if (p->form != MRA_FORM_NONSTANDARD) fail(MRA_E_UNSUPPORTED, "batches use the non-standard form");
    std::vector<Op*> ops(n);
    std::vector<Func*> funcs(n);
    for (int i = 0; i < n; ++i) {
      if (!ophs[i] || !fhs[i]) fail(MRA_E_INVALID, "mra_apply_batch: null handle");
      ops[i] = &const_cast<mra_op*>(ophs[i])->o;
      funcs[i] = &const_cast<mra_func*>(fhs[i])->f;
      if (ops[i]->ctx != c || funcs[i]->ctx != c)
        fail(MRA_E_MISMATCH, "handles belong to another context");
      if (ops[i]->k != funcs[i]->k || funcs[i]->k != funcs[0]->k)
        fail(MRA_E_MISMATCH, "all operators and functions of a batch need the same k");
      for (int j = 0; j < i; ++j)
        if (funcs[j] == funcs[i]) fail(MRA_E_INVALID, "a function appears twice in the batch");
      need_scaling(*funcs[i], "mra_apply_batch");
    }
    check_nonstandard(funcs[0]->k, *p);
    std::vector<std::unique_ptr<mra_func>> hs(n);
    std::vector<Func*> outf(n);
    for (int i = 0; i < n; ++i) {
      hs[i].reset(new mra_func());
      outf[i] = &hs[i]->f;
    }
    apply_nonstandard_batch(c, ops, funcs, p->tau_drop, p->tau_tier, outf);
    for (int i = 0; i < n; ++i) outs[i] = hs[i].release();
  });
}

mra_status mra_norm2(mra_ctx* ctx, const mra_func* fh, double* out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !out) fail(MRA_E_INVALID, "mra_norm2: bad arguments");
    const Func& f = fh->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    if (f.wavelet_form) {   // every slab: s_0 and the D_P pieces
      std::vector<int32_t> all(f.nodes());
      for (int64_t i = 0; i < f.nodes(); ++i) all[i] = (int32_t)i;
      *out = std::sqrt(reduce(c, f.k, f.coeff.p, nullptr, all, nullptr, nullptr, 0));
      return MRA_OK;
    }
    Func& fm = const_cast<mra_func*>(fh)->f;   // device leaf list is made on first use
    double s = reduce(c, f.k, f.coeff.p, nullptr, f.leaves, nullptr, nullptr, 0,
                      fm.device_leaves());
    *out = std::sqrt(s);
  });
}

mra_status mra_norm2_noalloc(mra_ctx* ctx, const mra_func* fh, double* out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !out) fail(MRA_E_INVALID, "mra_norm2_noalloc: bad arguments");
    const Func& f = fh->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    need_scaling(f, "mra_norm2_noalloc");
    if (f.d_leaves.n != f.leaves.size())
      fail(MRA_E_INVALID, "mra_norm2_noalloc: the function's leaf list is not on the device");
    const double s = norm2_noalloc(c->device, f.k, f.coeff.p, f.d_leaves.p,
                                   (int64_t)f.leaves.size(), c->stream);
    *out = std::sqrt(s);
  });
}

mra_status mra_trace(mra_ctx* ctx, const mra_func* fh, double* out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !out) fail(MRA_E_INVALID, "mra_trace: bad arguments");
    const Func& f = fh->f;
    if (f.ctx != c) fail(MRA_E_MISMATCH, "function belongs to another context");
    need_scaling(f, "mra_trace");
    std::vector<double> w(f.leaves.size());
    for (size_t i = 0; i < f.leaves.size(); ++i)
      w[i] = std::pow(c->width() / std::ldexp(1.0, f.level_of(f.leaves[i])), 1.5);
    *out = reduce(c, f.k, f.coeff.p, nullptr, f.leaves, nullptr, &w, 1);
  });
}

mra_status mra_inner(mra_ctx* ctx, const mra_func* fh, const mra_func* gh, double* out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !gh || !out) fail(MRA_E_INVALID, "mra_inner: bad arguments");
    Func& f = const_cast<mra_func*>(fh)->f;
    Func& g = const_cast<mra_func*>(gh)->f;
    if (f.ctx != c || g.ctx != c) fail(MRA_E_MISMATCH, "handles belong to another context");
    if (f.k != g.k) fail(MRA_E_MISMATCH, "functions have different k");
    need_scaling(f, "mra_inner");
    need_scaling(g, "mra_inner");
    filter_up_function(c, f);
    filter_up_function(c, g);
    // pair the leaves of the intersection of the two trees: boxes present in both where at
    // least one of the two is a leaf (the other side holds its filtered coefficients).
    std::vector<int32_t> la, lb;
    for (int n = 0; n < std::min(f.nlev, g.nlev); ++n) {
      for (int64_t i = f.level_off[n]; i < f.level_off[n + 1]; ++i) {
        int64_t j = find_node(g, n, f.code[i]);
        if (j < 0) continue;
        if (f.first_child[i] < 0 || g.first_child[j] < 0) {
          la.push_back((int32_t)i);
          lb.push_back((int32_t)j);
        }
      }
    }
    *out = reduce(c, f.k, f.coeff.p, g.coeff.p, la, &lb, nullptr, 2);
  });
}

mra_status mra_distance(mra_ctx* ctx, const mra_func* fh, const mra_func* gh, double* out) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  MRA_TRY(c, {
    if (!fh || !gh || !out) fail(MRA_E_INVALID, "mra_distance: bad arguments");
    Func& f = const_cast<mra_func*>(fh)->f;
    Func& g = const_cast<mra_func*>(gh)->f;
    if (f.ctx != c || g.ctx != c) fail(MRA_E_MISMATCH, "handles belong to another context");
    if (f.k != g.k) fail(MRA_E_MISMATCH, "functions have different k");
    need_scaling(f, "mra_distance");
    need_scaling(g, "mra_distance");
    if (f.code != g.code || f.first_child != g.first_child)
      fail(MRA_E_MISMATCH, "mra_distance: the two functions have different trees");
    double s = reduce(c, f.k, f.coeff.p, g.coeff.p, f.leaves, &g.leaves, nullptr, 3,
                      f.device_leaves());
    *out = std::sqrt(s);
  });
}

mra_status mra_set_schedule(mra_ctx* ctx, const mra_schedule* sch) {
  if (!ctx || !sch || sch->sub_batches < 0 || sch->sub_batches > 64 || sch->split_div < 1)
    return MRA_E_INVALID;
  ctx->c.sched_sub_batches = sch->sub_batches;
  ctx->c.sched_split_div = sch->split_div;
  return MRA_OK;
}

mra_status mra_get_schedule(const mra_ctx* ctx, mra_schedule* sch) {
  if (!ctx || !sch) return MRA_E_INVALID;
  sch->sub_batches = ctx->c.sched_sub_batches;
  sch->split_div = ctx->c.sched_split_div;
  return MRA_OK;
}

namespace {
// The autotuner's cache: a JSON object of  "key": {"sub_batches": S, "split_div": D, "ms": t}.
struct TuneEntry {
  std::string key;
  int sb = 0, div = 512;
  double ms = 0.0;
};
std::vector<TuneEntry> read_tune_cache(const char* path) {
  std::vector<TuneEntry> out;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return out;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, got);
  std::fclose(fp);
  size_t pos = 0;
  auto num_after = [&](size_t from, size_t end, const char* name, double& v) {
    const size_t q = text.find(name, from);
    if (q == std::string::npos || q > end) return false;
    const size_t c = text.find(':', q);
    if (c == std::string::npos || c > end) return false;
    v = std::strtod(text.c_str() + c + 1, nullptr);
    return true;
  };
  while (true) {
    const size_t k0 = text.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = text.find('"', k0 + 1);
    const size_t ob = text.find('{', k1);
    const size_t cb = text.find('}', ob);
    if (k1 == std::string::npos || ob == std::string::npos || cb == std::string::npos) break;
    TuneEntry e;
    e.key = text.substr(k0 + 1, k1 - k0 - 1);
    double sb = -1, div = -1, ms = 0;
    if (num_after(ob, cb, "\"sub_batches\"", sb) && num_after(ob, cb, "\"split_div\"", div)) {
      num_after(ob, cb, "\"ms\"", ms);
      e.sb = (int)sb;
      e.div = (int)div;
      e.ms = ms;
      if (e.sb >= 0 && e.div >= 1) out.push_back(e);
    }
    pos = cb + 1;
  }
  return out;
}
void write_tune_cache(const char* path, const std::vector<TuneEntry>& es) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) fail(MRA_E_INVALID, std::string("mra_autotune_batch: cannot write ") + path);
  std::fprintf(fp, "{\n");
  for (size_t i = 0; i < es.size(); ++i)
    std::fprintf(fp, "  \"%s\": {\"sub_batches\": %d, \"split_div\": %d, \"ms\": %.3f}%s\n",
                 es[i].key.c_str(), es[i].sb, es[i].div, es[i].ms, i + 1 < es.size() ? "," : "");
  std::fprintf(fp, "}\n");
  std::fclose(fp);
  if (std::rename(tmp.c_str(), path) != 0)
    fail(MRA_E_INVALID, std::string("mra_autotune_batch: cannot replace ") + path);
}
}  // namespace

mra_status mra_autotune_batch(mra_ctx* ctx, int n, const mra_op* const* ophs,
                              const mra_func* const* fhs, const mra_apply_params* p,
                              const char* cache_path, mra_schedule* best, double* times_ms) {
  if (!ctx) return MRA_E_INVALID;
  Ctx* c = &ctx->c;
  const int old_sb = c->sched_sub_batches, old_div = c->sched_split_div;
  MRA_TRY(c, {
    if (n < 1 || !ophs || !fhs || !p || !best) fail(MRA_E_INVALID, "mra_autotune_batch: bad arguments");
    if (p->form != MRA_FORM_NONSTANDARD) fail(MRA_E_UNSUPPORTED, "batches use the non-standard form");
    if (!fhs[0]) fail(MRA_E_INVALID, "mra_autotune_batch: null handle");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, c->device), "hipGetDeviceProperties");
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    const std::string key = arch + "/k" + std::to_string(fhs[0]->f.k) +
                            (p->tau_tier > 0.0 ? "/tiered" : "/fp64");
    const int cand_sb[3] = {1, 2, 4}, cand_div[3] = {256, 512, 1024};
    std::vector<TuneEntry> cache;
    if (cache_path) {
      cache = read_tune_cache(cache_path);
      for (const TuneEntry& e : cache)
        if (e.key == key) {
          c->sched_sub_batches = e.sb;
          c->sched_split_div = e.div;
          best->sub_batches = e.sb;
          best->split_div = e.div;
          if (times_ms)
            for (int q = 0; q < 9; ++q) times_ms[q] = -1.0;
          return MRA_OK;
        }
    }
    std::vector<mra_func*> outs(n, nullptr);
    auto run = [&]() {
      const auto t0 = std::chrono::steady_clock::now();
      const mra_status rc = mra_apply_batch(ctx, n, ophs, fhs, p, outs.data());
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (rc != MRA_OK) {
        c->sched_sub_batches = old_sb;
        c->sched_split_div = old_div;
        fail(rc, c->err);
      }
      for (mra_func*& o : outs) {
        mra_func_free(o);
        o = nullptr;
      }
      return ms;
    };
    run();   // block caches, pinned arenas and planner buffers settle; not timed
    double t[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        c->sched_sub_batches = cand_sb[a];
        c->sched_split_div = cand_div[b];
        t[3 * a + b] = run();
        if (times_ms) times_ms[3 * a + b] = t[3 * a + b];
      }
    // the first candidate (fewest sub-batches, then shortest split) within 1% of the
    // fastest: differences below that are timing noise, and a stable pick keeps the
    // schedule, and the profiles taken under it, the same from run to run
    double fastest = 1e300;
    for (double v : t) fastest = std::min(fastest, v);
    int bsb = old_sb, bdiv = old_div;
    double best_ms = 1e300;
    for (int q = 0; q < 9; ++q)
      if (t[q] <= 1.01 * fastest) {
        bsb = cand_sb[q / 3];
        bdiv = cand_div[q % 3];
        best_ms = t[q];
        break;
      }
    c->sched_sub_batches = bsb;
    c->sched_split_div = bdiv;
    best->sub_batches = bsb;
    best->split_div = bdiv;
    if (cache_path) {
      TuneEntry e;
      e.key = key;
      e.sb = bsb;
      e.div = bdiv;
      e.ms = best_ms;
      cache.push_back(e);
      write_tune_cache(cache_path, cache);
    }
  });
}

mra_status mra_last_stats(const mra_ctx* ctx, mra_apply_stats* out) {
  if (!ctx || !out) return MRA_E_INVALID;
  *out = ctx->c.stats;
  return MRA_OK;
}

// ----------------------------------------------------------------- host-only helpers
mra_status mra_host_fit(int kind, double mu, double lo, double eps, double r_hi, int cap,
                        double* c, double* t, int* M) {
  try {
    std::vector<double> cc, tt;
    if (kind == 0)
      fit_coulomb(lo, eps, r_hi, cc, tt);
    else
      fit_bsh(mu, lo, eps, r_hi, cc, tt);
    if (M) *M = (int)cc.size();
    if (c || t) {
      if (cap < (int)cc.size()) return MRA_E_INVALID;
      if (c) std::copy(cc.begin(), cc.end(), c);
      if (t) std::copy(tt.begin(), tt.end(), t);
    }
    return MRA_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

mra_status mra_host_block(int k, double h, int delta, double texp, double* out) {
  if (k < 2 || k > kMaxK || !(h > 0) || !(texp > 0) || !out) return MRA_E_INVALID;
  try {
    block_t(k, h, delta, texp, out);
    return MRA_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

mra_status mra_host_filters(int k, double* h0, double* h1) {
  if (k < 2 || k > kMaxK || !h0 || !h1) return MRA_E_INVALID;
  std::vector<double> a, b;
  two_scale_filters(k, a, b);
  std::copy(a.begin(), a.end(), h0);
  std::copy(b.begin(), b.end(), h1);
  return MRA_OK;
}

mra_status mra_host_spectral_norm(int m, const double* a, double* out) {
  if (m < 1 || !a || !out) return MRA_E_INVALID;
  *out = spectral_norm(m, a);
  return MRA_OK;
}

mra_status mra_host_project(double cell_lo, double cell_hi, const mra_gaussian* g, int ng,
                            const mra_project_params* p, int64_t cap, uint64_t* keys,
                            double* coeffs, int64_t* nleaves) {
  if (!g || ng < 1 || !p || !(cell_hi > cell_lo)) return MRA_E_INVALID;
  if (p->k < 2 || p->k > kMaxK || !(p->thresh > 0) || p->initial_level < 0 ||
      p->max_level > kMaxLevel || p->initial_level > p->max_level)
    return MRA_E_INVALID;
  try {
    Ctx c;
    c.lo = cell_lo;
    c.hi = cell_hi;
    Func f;
    std::vector<double> coef;
    project_gaussians(&c, g, ng, p->k, p->thresh, p->initial_level, p->max_level, f, coef);
    int64_t nl = (int64_t)f.leaves.size();
    if (nleaves) *nleaves = nl;
    if (keys || coeffs) {
      if (cap < nl) return MRA_E_INVALID;
      const size_t k3 = (size_t)p->k * p->k * p->k;
      for (int64_t i = 0; i < nl; ++i) {
        int32_t node = f.leaves[i];
        int n = f.level_of(node);
        if (keys) keys[i] = (1ULL << (3 * n)) | f.code[node];
        if (coeffs) std::memcpy(coeffs + i * k3, coef.data() + (size_t)node * k3, k3 * 8);
      }
    }
    return MRA_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

}  // extern "C"
