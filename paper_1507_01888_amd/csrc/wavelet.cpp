// Wavelet form of a function (Sec. 2.2, two-scale relation and fast wavelet transform):
// compression, reconstruction and truncation on the device.
//
// Layout of the wavelet form: the same flat octree and slab array as the scaling form; the
// root's slab holds the root's scaling coefficients s_0, and the slab of every other node C
// holds the part of its parent P's wavelet block D_P = B_P - unfilter(s_P) that sits at C's
// position in the (2k)^3 children block.  The 8 children of a box are contiguous, so D_P is
// the 8 k^3 doubles starting at P's first child.
//
// compress:     bottom-up over refined levels, s_P = filter(B_P) into P's slab, then the
//               children block minus unfilter(s_P) (sum-down kernel with sign -1).
// reconstruct:  top-down, children block += unfilter(s_P) (sum-down kernel, sign +1).
// truncate:     compress, ||D_P|| of every refined box (child-norm kernel), bottom-up pruning
//               on the host (a refined box whose children are all leaves loses them when
//               ||D_P|| <= tol), gather of the kept slabs into the new tree, reconstruct.
#include <cmath>

#include "mra_internal.hpp"

namespace mra {
namespace {

void copy_structure(const Func& src, Func& dst) {
  dst.ctx = src.ctx;
  dst.k = src.k;
  dst.nlev = src.nlev;
  dst.level_off = src.level_off;
  dst.code = src.code;
  dst.first_child = src.first_child;
  dst.leaves = src.leaves;
  dst.interior = src.interior;
  dst.inter_level_off = src.inter_level_off;
}

void copy_coefficients(Ctx* ctx, const Func& src, Func& dst) {
  dst.coeff.alloc(ctx, src.coeff.n);
  if (src.coeff.n)
    hip_check(hipMemcpyAsync(dst.coeff.p, src.coeff.p, src.coeff.n * sizeof(double),
                             hipMemcpyDeviceToDevice, ctx->stream),
              "hipMemcpyAsync D2D");
}

struct Filters {
  DevArray<double> h0, h1;
  Filters(Ctx* ctx, int k) {
    std::vector<double> a, b;
    two_scale_filters(k, a, b);
    h0.upload(ctx, a);
    h1.upload(ctx, b);
  }
};

// NodeRefs of the refined boxes of level n of f (slab table entry 0).
std::vector<NodeRef> level_refs(const Func& f, int n) {
  std::vector<NodeRef> r;
  for (int64_t q = f.inter_level_off[n]; q < f.inter_level_off[n + 1]; ++q)
    r.push_back({0, f.interior[q], f.first_child[f.interior[q]], -1});
  return r;
}

// Top-down sum-down of g's own slabs: every children block += unfilter(parent's slab).
void reconstruct_inplace(Ctx* ctx, Func& g) {
  if (g.nlev > 1) {
    Filters h(ctx, g.k);
    std::vector<double*> tab{g.coeff.p};
    DevArray<double*> d_tab;
    d_tab.upload(ctx, tab);
    std::vector<NodeRef> refs;
    std::vector<int64_t> off{0};
    for (int n = 0; n + 1 < g.nlev; ++n) {
      const auto r = level_refs(g, n);
      refs.insert(refs.end(), r.begin(), r.end());
      off.push_back((int64_t)refs.size());
    }
    DevArray<NodeRef> d_refs;
    d_refs.upload(ctx, refs);
    for (size_t j = 0; j + 1 < off.size(); ++j)
      launch_sum_down(g.k, d_tab.p, d_refs.p + off[j], (int)(off[j + 1] - off[j]), nullptr,
                      h.h0.p, h.h1.p, ctx->stream, 1.0);
    ctx->sync();
  }
  g.wavelet_form = false;
  g.interior_valid = true;
}

}  // namespace

void compress_function(Ctx* ctx, const Func& f, Func& out) {
  copy_structure(f, out);
  copy_coefficients(ctx, f, out);
  if (f.nlev > 1) {
    Filters h(ctx, f.k);
    std::vector<double*> tab{out.coeff.p};
    DevArray<double*> d_tab;
    d_tab.upload(ctx, tab);
    std::vector<NodeRef> refs;
    std::vector<int64_t> off{0};
    for (int n = f.nlev - 2; n >= 0; --n) {   // finest refined level first
      const auto r = level_refs(f, n);
      refs.insert(refs.end(), r.begin(), r.end());
      off.push_back((int64_t)refs.size());
    }
    DevArray<NodeRef> d_refs;
    d_refs.upload(ctx, refs);
    DevArray<double> d_bn2;
    d_bn2.alloc(ctx, std::max<size_t>(1, refs.size()));
    // Level n's filter reads the slabs of level n + 1, which still hold scaling coefficients
    // (level n + 1's own subtraction changed level n + 2); then level n's subtraction turns
    // level n + 1's slabs into wavelet parts.
    for (size_t j = 0; j + 1 < off.size(); ++j) {
      const int cnt = (int)(off[j + 1] - off[j]);
      launch_filter_up(f.k, d_tab.p, d_refs.p + off[j], cnt, h.h0.p, h.h1.p, d_bn2.p + off[j],
                       nullptr, ctx->stream);
      launch_sum_down(f.k, d_tab.p, d_refs.p + off[j], cnt, nullptr, h.h0.p, h.h1.p,
                      ctx->stream, -1.0);
    }
    ctx->sync();
  }
  out.wavelet_form = true;
  out.interior_valid = false;
}

void reconstruct_function(Ctx* ctx, const Func& c, Func& out) {
  copy_structure(c, out);
  copy_coefficients(ctx, c, out);
  reconstruct_inplace(ctx, out);
}

void truncate_function(Ctx* ctx, const Func& f, double tol, Func& out, double& removed2) {
  const int k = f.k;
  Func C;
  compress_function(ctx, f, C);
  const int64_t ni = (int64_t)f.interior.size();
  std::vector<double> n2(ni);
  if (ni > 0) {
    std::vector<int32_t> fch(ni);
    for (int64_t q = 0; q < ni; ++q) fch[q] = f.first_child[f.interior[q]];
    DevArray<int32_t> d_fch;
    d_fch.upload(ctx, fch);
    DevArray<double> d_n2;
    d_n2.alloc(ctx, ni);
    launch_child_norm2(k, C.coeff.p, d_fch.p, (int)ni, d_n2.p, ctx->stream);
    hip_check(hipMemcpyAsync(n2.data(), d_n2.p, ni * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream),
              "hipMemcpyAsync D2H");
    ctx->sync();
  }
  // bottom-up pruning; refined[node] says whether the box keeps its children
  std::vector<char> refined(f.nodes(), 0);
  for (int32_t p : f.interior) refined[p] = 1;
  removed2 = 0.0;
  for (int n = f.nlev - 2; n >= 0; --n) {
    for (int64_t q = f.inter_level_off[n]; q < f.inter_level_off[n + 1]; ++q) {
      const int32_t p = f.interior[q], fc = f.first_child[p];
      bool kid_refined = false;
      for (int c = 0; c < 8; ++c) kid_refined = kid_refined || refined[fc + c];
      if (!kid_refined && std::sqrt(n2[q]) <= tol) {
        refined[p] = 0;
        removed2 += n2[q];
      }
    }
  }
  // kept tree, level by level in code order (children of consecutive parents are
  // consecutive), with the source node of every kept node
  std::vector<std::vector<uint64_t>> levels;
  std::vector<int32_t> from;
  std::vector<int32_t> cur{0};
  while (!cur.empty()) {
    std::vector<uint64_t> codes;
    std::vector<int32_t> next;
    for (int32_t i : cur) {
      codes.push_back(f.code[i]);
      from.push_back(i);
      if (refined[i])
        for (int c = 0; c < 8; ++c) next.push_back(f.first_child[i] + c);
    }
    levels.push_back(std::move(codes));
    cur.swap(next);
  }
  out.ctx = ctx;
  out.k = k;
  build_tree(out, levels);
  out.coeff.alloc(ctx, (size_t)out.nodes() * k * k * k);
  DevArray<int32_t> d_from;
  d_from.upload(ctx, from);
  launch_copy_slabs(k, out.coeff.p, nullptr, C.coeff.p, d_from.p, (int)from.size(), ctx->stream);
  out.wavelet_form = true;
  reconstruct_inplace(ctx, out);
  out.device_leaves();
  ctx->sync();
}

}  // namespace mra
