// Internal declarations of libmra (host planner + device kernels).
//
// Layout of a function in HBM ("flat octree"): nodes are stored level by level (level 0
// first); inside a level they are sorted by their Morton code (interleave(lx, ly, lz), x in
// the highest bit of each bit triple).  Every node owns one k^3 FP64 slab, row-major
// [i][j][m].  A refined node has all 8 children, and because their codes are
// 8*parent + c (c = 4bx + 2by + bz) they are 8 consecutive nodes of the next level: the
// (2k)^3 "children block" of a node is 8 consecutive slabs.  Leaves hold the function;
// slabs of refined nodes are workspace (filtered scaling coefficients when valid).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mra.h"

namespace mra {

constexpr int kMaxK = 14;
constexpr int kMaxLevel = 20;

// ----------------------------------------------------------------------------- errors
struct Error {
  mra_status code;
  std::string msg;
};
[[noreturn]] void fail(mra_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what);

// ------------------------------------------------------------------------ host threads
// Persistent workers for the planner's data-parallel loops (created once per process, at
// most 16 including the calling thread).  run(count, fn) calls fn(i, worker) for every
// i < count, the caller taking part as worker 0, and returns when all calls are done; the
// first exception thrown by fn is rethrown on the caller.  Not reentrant.
class Pool {
 public:
  static Pool& get();
  unsigned workers() const { return (unsigned)th_.size() + 1; }
  void run(size_t count, const std::function<void(size_t, unsigned)>& fn);
  ~Pool();

 private:
  Pool();
  void loop(unsigned id);
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_, done_;
  const std::function<void(size_t, unsigned)>* fn_ = nullptr;
  size_t count_ = 0;
  std::atomic<size_t> next_{0};
  std::atomic<unsigned> busy_{0};
  std::atomic<uint64_t> gen_{0};
  std::atomic<bool> stop_{false};
  std::exception_ptr err_;
  void work(unsigned id);
};

// ------------------------------------------------------------------------- quadrature
struct GLRule {
  std::vector<double> x, w;  // on [0, 1]
};
const GLRule& gauss_legendre01(int n);
// phi_i(x) = sqrt(2i+1) P_i(2x-1) on [0,1], 0 outside; out[0..k-1]
void scaling_functions(int k, double x, double* out);
// two-scale filters h0, h1 (row-major k x k): parent s = h0 s_left + h1 s_right
void two_scale_filters(int k, std::vector<double>& h0, std::vector<double>& h1);

// ------------------------------------------------------------------------ operator fit
double erfc_inverse(double p);
void fit_coulomb(double r_lo, double eps, double r_hi, std::vector<double>& c,
                 std::vector<double>& t);
void fit_bsh(double mu, double r_lo, double eps, double r_hi, std::vector<double>& c,
             std::vector<double>& t);

// ------------------------------------------------------------------------ 1D blocks
// t^{n,delta} for the kernel exp(-texp r^2) on boxes of width h (row-major k x k,
// rows = target index).
void block_t(int k, double h, int delta, double texp, double* out);
// Spectral norm of a row-major m x m matrix.
double spectral_norm(int m, const double* a);
// Rigorous bounds used to enumerate candidate displacements.
double e_bound(int k, double h, double beta);
double decay_bound(double h, double beta, int delta);

// Per (level, term) cache entry: blocks for delta in [-D, D] and 1D norms for 0..D.
struct BlockEntry {
  int D = -1;
  std::vector<double> a, e, r;   // size D+1
  int64_t r_base = -1;           // index of the R block of delta = -D in the device R array
  int64_t t_base = -1;           // index of the t block of delta = -D in the device t array
};

// ------------------------------------------------------------------------- context
struct Ctx;
// Reusable staging of the per-apply arrays: host arrays are packed into one pinned buffer
// and copied with a single asynchronous transfer into one device buffer; scratch regions
// (no host contents) live in a second device buffer.  Both grow on demand and are reused
// by the next apply on the context, which may start only after the previous one has been
// synchronised (every apply ends with a stream synchronisation).
struct Arena {
  Ctx* ctx = nullptr;
  char* host = nullptr;
  size_t host_cap = 0;
  char* dev = nullptr;
  size_t dev_cap = 0;
  char* scr = nullptr;
  size_t scr_cap = 0;
  size_t used = 0, scr_used = 0;
  size_t committed = 0;                               // bytes already copied to the device
  ~Arena();
  void begin(Ctx* c) {
    ctx = c;
    used = scr_used = committed = 0;
  }
  size_t put_bytes(const void* src, size_t bytes);    // returns the device offset
  size_t reserve(size_t bytes);                       // host region filled by the caller
  template <class T>
  T* host_at(size_t off) const { return reinterpret_cast<T*>(host + off); }
  template <class T>
  size_t put(const std::vector<T>& v) { return put_bytes(v.data(), v.size() * sizeof(T)); }
  size_t scratch(size_t bytes);                       // device-only region, offset
  void commit();                                      // grow device buffers, copy the rest
  // device capacity for `bytes` of uploads, so that a prefix can be copied before the rest
  // of the arena is filled (commit() re-copies everything if the estimate was short)
  void prepare_device(size_t bytes);
  void commit_upto(size_t end);                       // copy [committed, end) now
  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(dev + off); }
  template <class T>
  T* scr_at(size_t off) const { return reinterpret_cast<T*>(scr + off); }
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  mra_alloc_fn alloc = nullptr;
  mra_free_fn free_fn = nullptr;
  void* user = nullptr;
  double lo = 0, hi = 1;
  std::string err;
  mra_apply_stats stats{};
  hipEvent_t ev[8]{};
  Arena arena[5];                      // filter-up; tables of alternate sub-batches; alternate chunks
  double* red_part = nullptr;          // 2048 partial sums of the leaf reductions
  // schedule of the batched apply (mra_set_schedule / mra_autotune_batch): number of
  // pipelined sub-batches (0: 4 for >= 8 functions, 2 for >= 2, else 1) and the divisor D of
  // the split length max(24, items / D) of long target lists
  int sched_sub_batches = 0;
  int sched_split_div = 512;

  double width() const { return hi - lo; }
  void* dalloc(size_t bytes);
  void dfree(void* p);
  void sync();
};

template <class T>
struct DevArray {
  Ctx* ctx = nullptr;
  T* p = nullptr;
  size_t n = 0;
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  ~DevArray() { reset(); }
  void reset() {
    if (p && ctx) ctx->dfree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(Ctx* c, size_t count) {
    reset();
    ctx = c;
    n = count;
    if (count) p = static_cast<T*>(c->dalloc(count * sizeof(T)));
  }
  void upload(Ctx* c, const std::vector<T>& v) {
    alloc(c, v.size());
    if (!v.empty())
      hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice,
                               c->stream),
                "hipMemcpyAsync H2D");
  }
};

// ------------------------------------------------------------------------- function
struct Func {
  Ctx* ctx = nullptr;
  int k = 0;
  int nlev = 0;                        // levels 0 .. nlev-1 are present
  std::vector<int64_t> level_off;      // nlev + 1
  std::vector<uint64_t> code;          // per node, sorted within level
  std::vector<int32_t> first_child;    // per node, -1 for leaves
  std::vector<int32_t> leaves;         // leaf node indices (level-major, sorted)
  std::vector<int32_t> interior;       // refined node indices (level-major, sorted)
  std::vector<int64_t> inter_level_off;  // nlev + 1 offsets into `interior`
  DevArray<double> coeff;              // nodes * k^3
  DevArray<int32_t> d_leaves;          // device copy of `leaves`, made on first use
  bool interior_valid = false;
  bool wavelet_form = false;           // slabs hold s_0 and the D_P pieces (Sec. 2.2)

  int64_t nodes() const { return (int64_t)code.size(); }
  int level_of(int64_t node) const;
  void finalize_structure();           // leaves / interior lists from first_child
  const int32_t* device_leaves();
};

// Build the node arrays of a full octree from per-level sorted codes.
void build_tree(Func& f, const std::vector<std::vector<uint64_t>>& levels);

// Wavelet form (Sec. 2.2): out is a new function; the input is left unchanged.
void compress_function(Ctx* ctx, const Func& f, Func& out);
void reconstruct_function(Ctx* ctx, const Func& c, Func& out);
// Drops D_P of refined boxes whose children are leaves while ||D_P|| <= tol, bottom-up;
// removed2 = sum of the dropped ||D_P||^2 (the squared L2 error, by orthogonality).
void truncate_function(Ctx* ctx, const Func& f, double tol, Func& out, double& removed2);

// ------------------------------------------------------------------------- operator
struct Op {
  Ctx* ctx = nullptr;
  int k = 0;
  std::vector<double> c, t;
  std::map<std::pair<int, int>, BlockEntry> entries;   // (level, mu)
  std::vector<BlockEntry*> entry_at;                   // [level * M + mu] -> entries' node
  std::vector<double> hR, hT;                          // host mirror of device blocks
  DevArray<double> dR, dT;                             // transposed blocks
  size_t dR_blocks = 0, dT_blocks = 0;                 // blocks resident on device
  DevArray<double> d_c;
  // Low-precision tier: per R block index b one record of BF16 matrices (rows = output
  // index) in the lane order of the BF16 matrix-core operands, built from hR[b], hT[b]:
  //   U(R), U(E), U(P): N x UP rows, UP = 8 ceil(N/8) columns, zero padded;
  //   V(R), V(E), V(P): N x 32, column slot s holds column perm(s), where slot 8g + j
  //   is column 4g + j (j < 4) or 16 + 4g + j - 4 (j >= 4), zero where that is >= N;
  // N = 2k, P = H^T t H, E = R - P.
  std::vector<uint16_t> hL;
  DevArray<uint16_t> dL;
  size_t hL_blocks = 0, dL_blocks = 0;
  // Make sure (level, mu) has blocks and norms for |delta| <= D.  Returns the entry.
  const BlockEntry& ensure(int level, int mu, int D);
  void ensure_low();                                   // BF16 records for every R block
  void sync_device();                                  // upload blocks added since last call
};
// BF16 record geometry of the low tier for wavelet order k.
inline int low_up(int k) { return (2 * k + 7) / 8 * 8; }
inline size_t low_record(int k) { return (size_t)3 * 2 * k * low_up(k) + (size_t)3 * 2 * k * 32; }
// FP64 -> FP32 (round to nearest even) -> BF16 (round to nearest even), finite inputs.
uint16_t bf16_bits(double v);

// ------------------------------------------------------------------------- projection
void project_gaussians(Ctx* ctx, const mra_gaussian* g, int ng, int k, double thresh,
                       int initial_level, int max_level, Func& out,
                       std::vector<double>& leaf_coeffs);
// The same projection with the integrals, coefficients and refinement tests on the device;
// out.coeff receives the leaf slabs (interior slabs zero).
void project_gaussians_device(Ctx* ctx, const mra_gaussian* g, int ng, int k, double thresh,
                              int initial_level, int max_level, Func& out);

// ------------------------------------------------------------------------- device side
struct NSItem {          // one kept (source, displacement, term) triple of a target
  int32_t src;           // input node P (its slab holds s_P)
  int32_t src_fc;        // first child of P (children block B_P)
  int32_t mu;
  int32_t rx, ry, rz;    // R block indices (transposed (2k)^2 blocks)
  int32_t tx, ty, tz;    // t block indices (transposed k^2 blocks)
  int32_t slot;          // filter-up slot of P: its children block in slab order (k = 14)
};
struct LowItem {         // one kept triple of the low-precision tier
  int32_t slot;          // BF16 copy of the children block B_P (filter-up order)
  int32_t mu;
  int32_t rx, ry, rz;    // R block indices (BF16 records)
};
struct TargetRange {
  int32_t fn;            // function of the batch (index into the pointer tables)
  int32_t node;          // output node T (its slab gets the level-n part)
  int32_t fc;            // first child of T in the output (children block)
  int32_t beg, end;      // items
  int32_t partial;       // -1: accumulate into the output; else slot of a partial block
  int32_t sub;           // >= 0: slot (k^3 doubles) receiving the level-n subtraction of T
};
struct SplitTarget {     // a target whose list was split over several workgroups
  int32_t fn;
  int32_t fc;            // first child of T in the output
  int32_t first, count;  // partial slots ((2k)^3 + k^3 doubles each), summed in this order
  int32_t sub;           // >= 0: level-n subtraction slot of T
};
// A refined node for filter-up / sum-down.  The level-n subtraction of a target is kept in
// a slot of its own (sub >= 0) and added by sum-down, because the same slab receives the
// parent target's children block in the same launch.
struct NodeRef {
  int32_t fn, node, fchild, sub;
};

void launch_zero(double* p, size_t n, hipStream_t s);
// Clears tab[i][0 .. len[i]) for i < count (device pointer table and lengths).
void launch_zero_batch(double* const* tab, const int64_t* len, int count, size_t maxlen,
                       hipStream_t s);
// mirror != nullptr: also writes the BF16 copy of each children block, layout
// [a][b][c] with c padded to low_up(k), one block per ref.
void launch_filter_up(int k, double* const* coeff_tab, const NodeRef* refs, int count,
                      const double* h0, const double* h1, double* bnorm2, uint16_t* mirror,
                      hipStream_t s);
// True when the low-precision transform kernel is built for this k.
bool low_kernel_available(int k);
// counter: one int of device scratch (the persistent kernel's work counter, set here).
// The BF16 records of every operator must lie within 2^31 - 16 bytes of its array's start.
void launch_apply_low(int k, const uint16_t* mirror, double* const* out_tab,
                      const LowItem* items, const TargetRange* targets, int ntargets,
                      const uint16_t* const* l_tab, const double* const* c_tab, int* counter,
                      hipStream_t s);
// True when the non-standard kernel for this k also applies the level-n subtraction.
bool ns_kernel_fuses_subtraction(int k);
// True when the non-standard kernel for this k shares the y- and z-contractions between
// triples: it needs the FP64 triples of a target ordered by (term, dz, dy, dx).
bool ns_kernel_factored(int k);
// slabs (k = 14): the children blocks in slab order (launch_slab_mirror), by item slot
void launch_apply_ns(int k, const double* const* in_tab, double* const* out_tab,
                     const NSItem* items, const TargetRange* targets, int ntargets,
                     const double* const* r_tab, const double* const* t_tab,
                     const double* const* c_tab, double* partials, double* subbuf,
                     int* counter, hipStream_t s, const double* slabs = nullptr);
// True when the non-standard kernel for this k streams its source blocks from the copies
// that launch_slab_mirror writes.
bool ns_uses_slab_mirror(int k);
// For each listed box, its children block (8 k^3 coefficients from first_child on) rewritten
// into slot i of slabs (8 k^3 doubles per slot) in the streaming kernel's slab order: z-quad
// zq at zq (2k)^2 4, element (x, y, z = 4 zq + zz) at (x 2k + y) 4 + zz.  k = 14 only.
void launch_slab_mirror(int k, double* const* coeff_tab, const NodeRef* refs, int count,
                        double* slabs, hipStream_t s);
void launch_reduce_partials(int k, const double* partials, double* const* out_tab,
                            double* subbuf, const SplitTarget* splits, int nsplits,
                            hipStream_t s);
// t_lds > 0: every target belongs to function 0, whose t table holds t_lds doubles (the
// k = 8 kernel then stages it in LDS when it fits); 0 for batches of several functions
void launch_apply_std(int k, const double* const* in_tab, double* const* out_tab,
                      const NSItem* items, const TargetRange* targets, int ntargets,
                      const double* const* t_tab, const double* const* c_tab, double scale,
                      hipStream_t s, int t_lds = 0);
// children of each listed box += sign * unfilter(box's slab [+ its subbuf block]);
// sign = -1 turns a children block into the box's wavelet part D_P (Sec. 2.2).
void launch_sum_down(int k, double* const* coeff_tab, const NodeRef* refs, int count,
                     const double* subbuf, const double* h0, const double* h1, hipStream_t s,
                     double sign = 1.0);
// out[i] = squared norm of the 8 slabs starting at fchild[i] (a box's children block).
void launch_child_norm2(int k, const double* coeff, const int32_t* fchild, int count,
                        double* out, hipStream_t s);
// dst slab to[i] (slab i when to is null) = src slab from[i], i < count.
void launch_copy_slabs(int k, double* dst, const int32_t* to, const double* src,
                       const int32_t* from, int count, hipStream_t s);
// Adaptive projection of a Gaussian sum, one level (kernels.hip describes the row layout):
// 1D integral rows for the level's distinct box indices, then per box its own coefficients
// into S and (test != 0) the squared norm of its children block's wavelet part into d2.
void launch_gauss1d(int k, const double* gpar, int ng, const int64_t* lvals, int nl, int off1,
                    int off2, int n, double lo, double W, const double* glx, const double* glw,
                    int nq, const double* h0, const double* h1, double* T, uint8_t* nz,
                    hipStream_t s);
void launch_project_level(int k, const double* T, const uint8_t* nz, const int32_t* boxu,
                          int nbox, int ng, const double* gpar, int test, double* d2,
                          double* S, hipStream_t s);
void launch_leaf_reduce(int k, const double* a, const double* b, const int32_t* leaves_a,
                        const int32_t* leaves_b, const double* weight, int count, int mode,
                        double* partial, int nblocks, hipStream_t s);

// Allocation-free norm2: address of this device's static scratch array (looked up once per
// device with hipGetSymbolAddress) and the reduction into it; returns sum ||s_leaf||^2.
double* static_scratch_init(int device);
double norm2_noalloc(int device, int k, const double* coeff, const int32_t* leaves_dev,
                     int64_t count, hipStream_t s);

// Host drivers
void apply_nonstandard_batch(Ctx* ctx, const std::vector<Op*>& ops,
                             const std::vector<Func*>& funcs, double tau, double tau_tier,
                             const std::vector<Func*>& outs);
void filter_up_function(Ctx* ctx, Func& f);

}  // namespace mra
