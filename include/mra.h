/*
 * mra.h -- C ABI of libmra: separated-operator apply on Legendre multiwavelet octrees
 * for AMD Instinct MI355X (gfx950).
 *
 * The calls follow the statement of the problem in the example of Sec. 3.1 of
 * Harrison et al., "MADNESS: a multiresolution, adaptive numerical environment for
 * scientific simulation" (arXiv:1507.01888): a cubic cell, an operator built from
 * (lo, eps), the adaptive projection of a function with (k, thresh), op(g), and the
 * trace / 2-norm / inner product of the result.
 *
 * Conventions
 *  - Every call returns an mra_status: MRA_OK (0) or a negative error code.  Output
 *    pointers are written only on success.  No C++ exception crosses the ABI.  The
 *    message of the last failure on a context is returned by mra_last_error().
 *  - Host pointers are plain host memory, read during the call and not retained.
 *  - Device memory is obtained through the context's allocator callbacks (or
 *    hipMalloc/hipFree when none are given) and released by the *_free calls.
 *  - All device work is issued on the context's HIP stream.  Calls that return host
 *    values (norms, exports, stats) synchronise that stream.
 *  - A context is not thread-safe; handles belong to the context that made them.
 *
 * Error codes
 *  MRA_E_INVALID      bad argument: k outside [2, 14], thresh <= 0, cell_hi <= cell_lo,
 *                     ng < 1, M < 1, expnt <= 0, tau_drop < 0, tau_tier < 0, ...
 *  MRA_E_NOMEM        the allocator returned NULL
 *  MRA_E_DEVICE       a HIP runtime error (its text is in the message)
 *  MRA_E_UNSUPPORTED  a combination this build does not implement (non-standard apply with
 *                     k = 11 or 13; the low-precision tier with k other than 10, 12, 14)
 *  MRA_E_MISMATCH     operator and function disagree on k or context
 */
#ifndef MRA_H
#define MRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int mra_status;
#define MRA_OK 0
#define MRA_E_INVALID (-1)
#define MRA_E_NOMEM (-2)
#define MRA_E_DEVICE (-3)
#define MRA_E_UNSUPPORTED (-4)
#define MRA_E_MISMATCH (-5)

typedef struct mra_ctx mra_ctx;
typedef struct mra_func mra_func;
typedef struct mra_op mra_op;

/* Device allocator callbacks: alloc returns a device pointer of at least nbytes (NULL on
 * failure); free releases it.  user is passed through unchanged. */
typedef void* (*mra_alloc_fn)(size_t nbytes, void* user);
typedef void (*mra_free_fn)(void* ptr, void* user);

/* One term coeff * exp(-expnt |x - center|^2) of a Gaussian-sum function. */
typedef struct {
  double coeff;
  double expnt;
  double center[3];
} mra_gaussian;

/* Adaptive projection parameters (Sec. 2.1): wavelet order k (number of Legendre
 * polynomials per dimension), refinement threshold thresh on the Frobenius norm of a box's
 * wavelet coefficients, uniform starting level and deepest level (<= 20). */
typedef struct {
  int k;
  double thresh;
  int initial_level;
  int max_level;
} mra_project_params;

#define MRA_FORM_NONSTANDARD 0
#define MRA_FORM_STANDARD 1

#define MRA_LOW_NONE 0
#define MRA_LOW_BF16 1

/* Apply parameters.
 *  form         MRA_FORM_NONSTANDARD: telescoped non-standard form of Sec. 2.2 on an
 *               adaptive tree; MRA_FORM_STANDARD: level-n operator P^n T P^n on a uniform
 *               tree with displacements |delta|_inf <= disp_radius, no screening.
 *  tau_drop     non-standard form: a (box, displacement, term) triple is applied iff its
 *               norm bound eta = |c_mu| N(delta) ||B_P||_F is >= tau_drop.
 *  disp_radius  standard form only.
 *  tau_tier     non-standard form, levels n > 0: a kept triple with eta < tau_tier runs in
 *               the low-precision tier (0: every triple runs in FP64).  The low tier
 *               evaluates the triple's whole contribution c_mu [(R x R x R) - (P x P x P)] B_P,
 *               P = H^T t H, in the cancellation-free form
 *               E x R x R + P x E x R + P x P x E (E = R - P, Sec. 2.2 two-scale relation),
 *               so its rounding error is a small multiple of u_low * eta.
 *  low_precision MRA_LOW_BF16: BF16 inputs and operator blocks, FP32 accumulation per
 *               target, FP64 addition into the result (built for k = 10, 12, 14).
 *               Ignored when tau_tier == 0. */
typedef struct {
  int form;
  int disp_radius;
  double tau_drop;
  double tau_tier;
  int low_precision;
} mra_apply_params;

/* Counters of the last mra_apply on a context. */
typedef struct {
  int64_t triples;        /* kept (box, displacement, term) triples                  */
  int64_t targets;        /* distinct target boxes                                   */
  int64_t in_leaves;      /* leaves of the input tree                                */
  int64_t out_nodes;      /* nodes of the output tree                                */
  int64_t out_leaves;     /* leaves of the output tree                               */
  double useful_flops;    /* sum over triples of 6(2k)^4 + 6k^4 [n>0] (6k^4 standard) */
  double ms_filter;       /* device time of filter-up                                */
  double ms_plan;         /* host time of screening and planning (incl. copies)      */
  double ms_apply;        /* device time of the transform-and-accumulate kernels     */
  double ms_sumdown;      /* device time of sum-down                                 */
  double ms_main_kernel;  /* device time of the non-standard (or standard) main kernel */
  int64_t triples_low;    /* triples run in the low-precision tier (part of triples)   */
  double flops_low;       /* useful flops of those triples (part of useful_flops)      */
  double eta_low;         /* sum of eta over those triples                             */
  double ms_low_kernel;   /* device time of the low-precision transform kernel         */
  double flops_kernel;    /* FP64 flops the main kernel executes, unpadded: 2(2k)^4 per
                             mode product of a children block and 2k^4 per mode product
                             of a scaling block.  Equals useful_flops - flops_low unless
                             the kernel shares contractions between triples (k = 10: one
                             y-product per (term, dz, dy) group and one z-product per
                             (term, dz) group of a target's list instead of per triple)  */
  int64_t launches_main;  /* launches of the main kernel behind ms_main_kernel (a batched
                             apply plans and launches in chunks)                         */
  int64_t launches_low;   /* launches of the low-precision kernel behind ms_low_kernel    */
} mra_apply_stats;

/* Create a context on HIP device `device` using HIP stream `stream` (NULL: the null
 * stream) and the cubic cell [cell_lo, cell_hi]^3 (Sec. 3.1, set_cubic_cell). alloc/free
 * may both be NULL (hipMalloc/hipFree are used). */
mra_status mra_ctx_create(int device, void* stream, mra_alloc_fn alloc, mra_free_fn free_fn,
                          void* user, double cell_lo, double cell_hi, mra_ctx** out);
mra_status mra_ctx_free(mra_ctx* ctx);
/* Message of the last failure on ctx ("" if none).  Valid until the next call on ctx.
 * With ctx == NULL: the message of the last failed mra_ctx_create on this thread. */
const char* mra_last_error(const mra_ctx* ctx);

/* Adaptive projection of sum_g coeff_g exp(-expnt_g |x - center_g|^2) (Sec. 2.1, eq.
 * projection): exact separable 1D integrals, refinement of a box iff the norm of its
 * wavelet coefficients exceeds thresh. The result lives in device memory.  Level by level,
 * the device computes the 1D integrals, every box's coefficients and the wavelet norms of
 * its children block; the host keeps the frontier and the refinement decisions (one small
 * copy of the norms per level).  ng <= 4096, and per level the table of 1D integrals
 * (ng x the distinct box indices of the three axes x 5k doubles) at most 8 GiB; MRA_E_UNSUPPORTED
 * beyond. */
mra_status mra_project(mra_ctx* ctx, const mra_gaussian* g, int ng,
                       const mra_project_params* params, mra_func** out);

/* Tree size of a function. */
mra_status mra_func_info(const mra_func* f, int* k, int64_t* nodes, int64_t* leaves,
                         int* max_level);
/* Copy the leaves out: keys[i] is the level-prefixed Morton code
 * (1 << 3n) | interleave(lx, ly, lz) (x in the highest bit of each triple), coeffs holds
 * nleaves * k^3 doubles, each leaf row-major [i][j][m].  Leaves are ordered by level,
 * then by key.  cap is the capacity of keys in leaves; *nleaves receives the count. */
mra_status mra_func_export(mra_ctx* ctx, const mra_func* f, int64_t cap, uint64_t* keys,
                           double* coeffs, int64_t* nleaves);
mra_status mra_func_free(mra_func* f);

/* Wavelet form (Sec. 2.2: two-scale relation, fast wavelet transform).  Every refined box
 * P has the children block B_P (its 8 children's coefficients as one (2k)^3 block), its
 * scaling coefficients s_P = (H x H x H) B_P (H = [h0 | h1], the two-scale filters) and its
 * wavelet part D_P = B_P - (H^T x H^T x H^T) s_P, orthogonal to the parent's polynomial.
 * A function in wavelet form keeps its tree and slab layout: the root's slab holds s_0 and
 * the slab of every other node holds the part of its parent's D_P at that node's position.
 * ||f||^2 = ||s_0||^2 + sum_P ||D_P||^2 (orthonormal bases).
 *
 * Only mra_reconstruct, mra_norm2 (over every slab), mra_func_info, mra_func_repr,
 * mra_func_export_nodes and mra_func_free accept a function in wavelet form; every other
 * call returns MRA_E_INVALID for one.  Each call below creates a new function (the input
 * is unchanged; out is untouched on error) and synchronises the context's stream. */
enum { MRA_REPR_SCALING = 0, MRA_REPR_WAVELET = 1 };
mra_status mra_func_repr(const mra_func* f, int* repr);
/* f (scaling form) -> its wavelet form on the same tree. */
mra_status mra_compress(mra_ctx* ctx, const mra_func* f, mra_func** out);
/* c (wavelet form) -> the scaling form: top-down, every children block is
 * unfilter(s_P) + D_P; interior slabs hold s_P as well. */
mra_status mra_reconstruct(mra_ctx* ctx, const mra_func* c, mra_func** out);
/* Truncation (Sec. 2.2 discards wavelet coefficients below the threshold): bottom-up, a
 * refined box whose 8 children are all leaves (after the pruning of finer levels) loses
 * its children, becoming a leaf holding s_P, iff ||D_P||_F <= tol (the norm and
 * non-strict comparison of the projection's refinement test).  *out is the truncated
 * function in scaling form; *removed2 (may be NULL) receives sum ||D_P||^2 over the
 * removed boxes, which equals ||f - out||^2.  tol >= 0. */
mra_status mra_truncate(mra_ctx* ctx, const mra_func* f, double tol, mra_func** out,
                        double* removed2);
/* Every node's slab: keys as in mra_func_export (every node, ordered by level, then key),
 * coeffs nnodes * k^3 doubles.  In scaling form interior nodes hold their filtered
 * coefficients s_P; in wavelet form the slabs described above. */
mra_status mra_func_export_nodes(mra_ctx* ctx, const mra_func* f, int64_t cap,
                                 uint64_t* keys, double* coeffs, int64_t* nnodes);

/* Operators: sum_mu c_mu exp(-t_mu r^2), with the 1D operator blocks for wavelet order k
 * cached per (level, displacement, term) on first use (Sec. 2.2 Toeplitz blocks).
 *  mra_op_coulomb   1/r to relative eps on [lo, sqrt(3) W] (Sec. 2.3 quadrature).
 *  mra_op_bsh       exp(-mu r)/r (kernel of eq. bshkernel without 1/(4 pi)), error eps/r.
 *  mra_op_gaussians explicit terms (M >= 1, t > 0). */
mra_status mra_op_coulomb(mra_ctx* ctx, int k, double lo, double eps, mra_op** out);
mra_status mra_op_bsh(mra_ctx* ctx, int k, double mu, double lo, double eps, mra_op** out);
mra_status mra_op_gaussians(mra_ctx* ctx, int k, int M, const double* c, const double* t,
                            mra_op** out);
/* Number of terms and the terms themselves (c, t may be NULL to query M only). */
mra_status mra_op_terms(const mra_op* op, int* M, double* c, double* t);
mra_status mra_op_free(mra_op* op);

/* op(f) (Sec. 3.1 example; Sec. 2.2-2.3 method).  The result is a new function on the
 * output tree (input tree, all targets with their children, their ancestors). */
mra_status mra_apply(mra_ctx* ctx, const mra_op* op, const mra_func* f,
                     const mra_apply_params* params, mra_func** out);

/* (The non-standard form needs at least one refined box: an input whose root is a leaf is
 * rejected with MRA_E_INVALID.  A result without any kept triple is the zero function on
 * the root box.) */

/* op_i(f_i) for i < n in one pass: filter-up, screening, transform-and-accumulate and
 * sum-down each run as one launch sequence over all functions (non-standard form only).
 * The paper applies an operator to one function at a time (Sec. 3.1); this batched form
 * is this library's extension for many functions with uneven trees and operators with
 * different terms (e.g. one bound-state Helmholtz kernel per orbital, Sec. 3.2), so that
 * one transform launch covers the kept triples of all of them, longest target lists
 * first.  Each result equals that of mra_apply on the same pair up to the summation order
 * of split target lists.
 * Functions may have different trees and operators different terms, but all share k.
 * outs receives n new functions (written only on success).  A function may appear only
 * once (its refined-box slabs are workspace); operators may repeat. */
mra_status mra_apply_batch(mra_ctx* ctx, int n, const mra_op* const* ops,
                           const mra_func* const* fs, const mra_apply_params* params,
                           mra_func** outs);

/* The three reductions of the example program of Sec. 3.1 (norm2, trace, inner), which
 * prints the 2-norm, the integral and the Coulomb self-energy <g, op(g)> of its function.
 * All are FP64 with a fixed-order reduction (2048 workgroup partials summed in index order
 * on the host), so repeated calls give bitwise identical results.  Each synchronises the
 * context's stream.
 *
 * mra_norm2: 2-norm sqrt(sum over leaves ||s||^2) (the basis is orthonormal, Sec. 2.1);
 * for a function in wavelet form sqrt(||s_0||^2 + sum_P ||D_P||^2), the sum over every
 * slab (Sec. 2.2). */
mra_status mra_norm2(mra_ctx* ctx, const mra_func* f, double* out);
/* mra_norm2_noalloc: mra_norm2 for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  It calls no
 * allocator (neither hipMalloc/hipFree nor the context's callbacks nor any allocating
 * library routine): the 2048 workgroup partials and their ordered sum live in a fixed
 * static device array of 2080 doubles (16.3 KiB) per GPU, held until the process ends.
 * The reduction grid is fixed, so every function fits; the result is bitwise equal to
 * mra_norm2's (same partials, summed in the same order).  The function's leaf list is
 * resident on the device from its creation (MRA_E_INVALID otherwise).  Calls on one GPU
 * share the array: calls that overlap on that GPU (from two streams at once) race.
 * Synchronises the context's stream. */
mra_status mra_norm2_noalloc(mra_ctx* ctx, const mra_func* f, double* out);
/* mra_trace: integral of f over the cell, sum over leaves s_000 h_n^{3/2} (phi_0 is the
 * constant h_n^{-1/2} on its box). */
mra_status mra_trace(mra_ctx* ctx, const mra_func* f, double* out);
/* mra_inner: <f, g> over the cell (both with the same k; the trees may differ: every box
 * that is a leaf of one function and present in the other pairs the leaf's coefficients
 * with the other's filtered coefficients of that box). */
mra_status mra_inner(mra_ctx* ctx, const mra_func* f, const mra_func* g, double* out);
/* mra_distance: ||f - g||_2 for two functions on the same tree (same nodes, as the results
 * of two applies that differ only in arithmetic, e.g. with and without the low-precision
 * tier); MRA_E_MISMATCH when the trees or k differ.  Used to state the error of one
 * evaluation against another without copying either to the host. */
mra_status mra_distance(mra_ctx* ctx, const mra_func* f, const mra_func* g, double* out);

/* Counters of the last mra_apply on ctx. */
mra_status mra_last_stats(const mra_ctx* ctx, mra_apply_stats* out);

/* Work schedule of mra_apply / mra_apply_batch on a context (this library's own tuning
 * knobs; the paper's method is unaffected, results differ only in the summation order of
 * split target lists):
 *  sub_batches  functions are planned and launched in this many pipelined sub-batches
 *               (0: automatic, 4 for >= 8 functions, 2 for >= 2, else 1);
 *  split_div    a target list longer than max(24, items / split_div) is split over several
 *               workgroups whose partial blocks are summed in a fixed order (>= 1). */
typedef struct {
  int sub_batches;
  int split_div;
} mra_schedule;
mra_status mra_set_schedule(mra_ctx* ctx, const mra_schedule* s);
mra_status mra_get_schedule(const mra_ctx* ctx, mra_schedule* s);

/* Autotuner of the batched apply (the batching extension's "autotuned schedules"): times one
 * mra_apply_batch of (ops, fs, params) under each candidate schedule (sub_batches 1, 2, 4 x
 * split_div 256, 512, 1024; one untimed apply first, which also builds the operator block
 * caches), keeps on ctx the first candidate in that order whose time is within 1% of the
 * fastest (smaller differences are timing noise; the pick stays stable from run to run) and
 * returns it in *best.  With cache_path != NULL the
 * JSON file is read first: if it holds the key "<gfx arch>/k<k>/<fp64|tiered>", that schedule
 * is set without timing; otherwise the result is added to the file.  times_ms (optional,
 * capacity 9) receives the measured milliseconds in candidate order (-1 when read from the
 * cache).  The functions are only read; every result is freed. */
mra_status mra_autotune_batch(mra_ctx* ctx, int n, const mra_op* const* ops,
                              const mra_func* const* fs, const mra_apply_params* params,
                              const char* cache_path, mra_schedule* best, double* times_ms);

/* ---------------------------------------------------------------- host-only helpers
 * These run on the host only (no device, no context) and expose the library's FP64 host
 * numerics for testing.  Arrays are caller-owned host memory.
 *
 * mra_host_fit: kind 0 = Coulomb 1/r, 1 = exp(-mu r)/r; range [lo, r_hi], accuracy eps.
 *   With c == t == NULL only *M is written; otherwise cap must be >= M.
 * mra_host_block: the k x k block t^{n,delta} (row-major, rows = target index) of
 *   exp(-texp r^2) between boxes of width h at displacement delta (Sec. 2.2 Toeplitz).
 * mra_host_filters: two-scale filters h0, h1 (row-major k x k).
 * mra_host_spectral_norm: largest singular value of a row-major m x m matrix.
 * mra_host_project: adaptive projection on the host; leaves as in mra_func_export. */
mra_status mra_host_fit(int kind, double mu, double lo, double eps, double r_hi, int cap,
                        double* c, double* t, int* M);
mra_status mra_host_block(int k, double h, int delta, double texp, double* out);
mra_status mra_host_filters(int k, double* h0, double* h1);
mra_status mra_host_spectral_norm(int m, const double* a, double* out);
mra_status mra_host_project(double cell_lo, double cell_hi, const mra_gaussian* g, int ng,
                            const mra_project_params* params, int64_t cap, uint64_t* keys,
                            double* coeffs, int64_t* nleaves);

#ifdef __cplusplus
}
#endif

#endif /* MRA_H */
