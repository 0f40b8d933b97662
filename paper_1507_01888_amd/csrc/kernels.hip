// Device kernels of libmra for gfx950 (MI355X), FP64.
//
//  filter_up      children block B_P (8 consecutive child slabs) -> s_P = (H x H x H) B_P
//                 and ||B_P||_F^2 (two-scale relation, Sec. 2.2)
//  apply_ns       acc_T += c_mu (R_x x R_y x R_z) B_P over the target's kept triples
//                 (non-standard form, Sec. 2.2-2.3): three mode products per triple
//  apply_std      out_T += scale c_mu (t_x x t_y x t_z) s_S (standard form / the level-n
//                 subtraction of the non-standard form)
//  sum_down       children += (H^T x H^T x H^T) s_T (reconstruction, Sec. 2.2)
//  leaf_reduce    fixed-order partial sums for norm2 / trace / inner
//
// Mode products: a workgroup owns one target; thread t owns one "column" of the (N x N x N)
// tensor in each phase: phase x contracts the first index (thread = (Y, Z)), phase y the
// second (thread = (a, Z), in place), phase z the third (thread = (a, b)) and accumulates
// into registers that stay resident across all triples of the target.  Tensors live in LDS
// with the innermost index padded to N+1 doubles so that the strided phase-z reads are
// bank-conflict free.  Operator blocks are stored transposed (R^T[i][a] = R[a][i]) so that
// the N coefficients a thread needs for one input element are contiguous and uniform
// across the workgroup.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mra_internal.hpp"

namespace mra {

namespace {

constexpr int round64(int x) { return (x + 63) / 64 * 64; }

// Pointers read from the per-function tables are generic to the compiler, which then emits
// flat loads; those count against the LDS counter too, so every LDS wait would also wait for
// in-flight global prefetches.  The tables only hold device memory: cast to the global
// address space.
#define MRA_GLOBAL __attribute__((address_space(1)))
#define MRA_LDS __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ MRA_GLOBAL T* as_global(T* p) {
  return (MRA_GLOBAL T*)p;
}

__global__ void zero_kernel(double* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

// Sets the work counters c[0 .. n) of persistent kernels to v (vector stores, n <= 64).
__global__ void set_counter_kernel(int* __restrict__ c, int n, int v) {
  if ((int)threadIdx.x < n) as_global(c)[threadIdx.x] = v;
}

// Clears arrays tab[y][0 .. len[y]) for every y = blockIdx.y.
__global__ void zero_batch_kernel(double* const* __restrict__ tab, const int64_t* __restrict__ len) {
  MRA_GLOBAL double* __restrict__ p = as_global(tab[blockIdx.y]);
  const size_t n = (size_t)len[blockIdx.y];
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// FP64 -> FP32 -> BF16, both steps rounding to nearest even (bits of the BF16 value).
__device__ inline uint32_t bf16_bits_dev(float v) {
  return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)v);
}
__device__ inline uint32_t bf16_pair(float lo, float hi) {
  return bf16_bits_dev(lo) | (bf16_bits_dev(hi) << 16);
}

// --------------------------------------------------------------------------- filter-up
// The children block is read straight from the 8 child slabs; the z-contraction happens
// on the fly (each thread owns (X, Y) rows), so LDS only holds the two partially filtered
// tensors ((2k)^2 k and (2k) k^2 doubles).  With mirror != nullptr each row is also written
// as BF16 (layout [X][Y][Z], Z padded with zeros to UP = 8 ceil(2k/8)) for the
// low-precision tier.
template <int K>
__global__ __launch_bounds__(256) void filter_up_kernel(
    double* const* __restrict__ tab, const NodeRef* __restrict__ refs,
    const double* __restrict__ h0, const double* __restrict__ h1, double* __restrict__ bnorm2,
    uint16_t* __restrict__ mirror) {
  constexpr int N = 2 * K, K3 = K * K * K, KP1 = K + 1;
  constexpr int UP = (N + 7) / 8 * 8;
  __shared__ double T1[N * N * KP1];   // [X][Y][m]
  __shared__ double T2[N * K * KP1];   // [X][j][m]
  __shared__ __attribute__((aligned(16))) double H[K * N];    // [i][X]
  __shared__ __attribute__((aligned(16))) double HT[N * K];   // [X][i]
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const NodeRef ref = refs[blockIdx.x];
  const int node = ref.node, fc = ref.fchild;
  MRA_GLOBAL double* __restrict__ coeff = as_global(tab[ref.fn]);
  for (int e = tid; e < K * N; e += 256) {
    int i = e / N, X = e % N;
    const double h = X < K ? h0[i * K + X] : h1[i * K + X - K];
    H[e] = h;
    HT[X * K + i] = h;
  }
  __syncthreads();
  double sq = 0.0;
  // phase z: T1[X][Y][m] = sum_Z H[m][Z] B[X][Y][Z]; row (X, Y) = two contiguous child rows
  for (int e = tid; e < N * N; e += 256) {
    const int X = e / N, Y = e % N;
    const int bx = X / K, i = X % K, by = Y / K, j = Y % K;
    const MRA_GLOBAL double* r0 = coeff + (size_t)(fc + ((bx << 2) | (by << 1))) * K3 + (i * K + j) * K;
    const MRA_GLOBAL double* r1 = r0 + K3;
    double row[UP];
#pragma unroll
    for (int z = 0; z < K; ++z) {
      row[z] = r0[z];
      row[K + z] = r1[z];
    }
#pragma unroll
    for (int z = N; z < UP; ++z) row[z] = 0.0;
#pragma unroll
    for (int z = 0; z < K; ++z) sq += row[z] * row[z] + row[K + z] * row[K + z];
    // the row stays in registers, H is read from LDS (broadcast); two of the K sums at a
    // time, so that their LDS reads and products overlap
#pragma unroll 2
    for (int m = 0; m < K; ++m) {
      double t = 0.0;
#pragma unroll
      for (int z = 0; z < N; ++z) t += H[m * N + z] * row[z];
      T1[(X * N + Y) * KP1 + m] = t;
    }
    if (mirror) {
      u32x4* dst = reinterpret_cast<u32x4*>(mirror + (size_t)blockIdx.x * N * N * UP +
                                            (size_t)(X * N + Y) * UP);
#pragma unroll
      for (int c = 0; c < UP / 8; ++c) {
        u32x4 w;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          w[q] = bf16_pair((float)row[8 * c + 2 * q], (float)row[8 * c + 2 * q + 1]);
        dst[c] = w;
      }
    }
  }
  red[tid] = sq;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {   // fixed-order tree
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) bnorm2[blockIdx.x] = red[0];
  // phase y: T2[X][j][m] = sum_Y H[j][Y] T1[X][Y][m], thread (X, m)
  for (int e = tid; e < N * K; e += 256) {
    const int X = e / K, m = e % K;
    double t[K];
#pragma unroll
    for (int j = 0; j < K; ++j) t[j] = 0.0;
#pragma unroll 4
    for (int Y = 0; Y < N; ++Y) {
      const double v = T1[(X * N + Y) * KP1 + m];
#pragma unroll
      for (int j = 0; j < K; ++j) t[j] += HT[Y * K + j] * v;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) T2[(X * K + j) * KP1 + m] = t[j];
  }
  __syncthreads();
  // phase x: s[i][j][m] = sum_X H[i][X] T2[X][j][m], thread (j, m)
  for (int e = tid; e < K * K; e += 256) {
    const int j = e / K, m = e % K;
    double t[K];
#pragma unroll
    for (int i = 0; i < K; ++i) t[i] = 0.0;
#pragma unroll 4
    for (int X = 0; X < N; ++X) {
      const double v = T2[(X * K + j) * KP1 + m];
#pragma unroll
      for (int i = 0; i < K; ++i) t[i] += HT[X * K + i] * v;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) coeff[(size_t)node * K3 + (i * K + j) * K + m] = t[i];
  }
}

// --------------------------------------------------------------------------- apply (NS)
template <int K>
__global__ __launch_bounds__(round64(4 * K * K)) void apply_ns_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const double* const* __restrict__ r_tab, const double* const* __restrict__ c_tab,
    double* __restrict__ partials) {
  constexpr int N = 2 * K, N2 = N * N, K3 = K * K * K, ZP = N + 1;
  __shared__ double S[N * N * ZP];
  __shared__ double W[N * N * ZP];
  const int tid = threadIdx.x;
  const TargetRange tr = targets[blockIdx.x];
  const MRA_GLOBAL double* __restrict__ in = as_global(in_tab[tr.fn]);
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dR = as_global(r_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dc = as_global(c_tab[tr.fn]);
  double acc[N];
#pragma unroll
  for (int c = 0; c < N; ++c) acc[c] = 0.0;
  int loaded = -1;
  for (int it = tr.beg; it < tr.end; ++it) {
    const NSItem item = items[it];
    if (item.src_fc != loaded) {
      __syncthreads();
      for (int e = tid; e < 8 * K3; e += blockDim.x) {
        int c = e / K3, r = e - c * K3;
        int i = r / (K * K), j = (r / K) % K, m = r % K;
        S[((((c >> 2) & 1) * K + i) * N + ((c >> 1) & 1) * K + j) * ZP + (c & 1) * K + m] =
            in[(size_t)(item.src_fc + c) * K3 + r];
      }
      loaded = item.src_fc;
    }
    __syncthreads();
    const MRA_GLOBAL double* RX = dR + (size_t)item.rx * N2;
    const MRA_GLOBAL double* RY = dR + (size_t)item.ry * N2;
    const MRA_GLOBAL double* RZ = dR + (size_t)item.rz * N2;
    const double cmu = dc[item.mu];
    if (tid < N2) {  // phase x: thread (Y, Z)
      int Y = tid / N, Z = tid % N;
      double t[N];
#pragma unroll
      for (int a = 0; a < N; ++a) t[a] = 0.0;
      for (int i = 0; i < N; ++i) {
        double v = S[(i * N + Y) * ZP + Z];
#pragma unroll
        for (int a = 0; a < N; ++a) t[a] += RX[i * N + a] * v;
      }
#pragma unroll
      for (int a = 0; a < N; ++a) W[(a * N + Y) * ZP + Z] = t[a];
    }
    __syncthreads();
    if (tid < N2) {  // phase y: thread (a, Z), in place
      int a = tid / N, Z = tid % N;
      double t[N];
#pragma unroll
      for (int b = 0; b < N; ++b) t[b] = 0.0;
      for (int j = 0; j < N; ++j) {
        double v = W[(a * N + j) * ZP + Z];
#pragma unroll
        for (int b = 0; b < N; ++b) t[b] += RY[j * N + b] * v;
      }
#pragma unroll
      for (int b = 0; b < N; ++b) W[(a * N + b) * ZP + Z] = t[b];
    }
    __syncthreads();
    if (tid < N2) {  // phase z: thread (a, b) accumulates
      int a = tid / N, b = tid % N;
      double t[N];
#pragma unroll
      for (int c = 0; c < N; ++c) t[c] = 0.0;
      for (int m = 0; m < N; ++m) {
        double v = W[(a * N + b) * ZP + m];
#pragma unroll
        for (int c = 0; c < N; ++c) t[c] += RZ[m * N + c] * v;
      }
#pragma unroll
      for (int c = 0; c < N; ++c) acc[c] += cmu * t[c];
    }
    __syncthreads();
  }
  if (tid < N2) {
    int a = tid / N, b = tid % N;
    int ca = a / K, i = a % K, cb = b / K, j = b % K;
    if (tr.partial >= 0) {
      double* dst = partials + (size_t)tr.partial * (N * N2 + K3);
#pragma unroll
      for (int c = 0; c < N; ++c) dst[(a * N + b) * N + c] = acc[c];
    } else {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        int child = (ca << 2) | (cb << 1) | (c / K);
        size_t idx = (size_t)(tr.fc + child) * K3 + (i * K + j) * K + (c % K);
        out[idx] += acc[c];
      }
    }
  }
}

// Sum the partial children blocks of split targets in slot order and add them to the output.
// blockIdx.y selects a chunk of the target's elements; each thread sums its element over the
// slots in ascending order (loads of four slots in flight), so the result is fixed.
template <int K>
__global__ __launch_bounds__(256) void reduce_partials_kernel(
    const double* __restrict__ partials, double* const* __restrict__ out_tab,
    double* __restrict__ subbuf, const SplitTarget* __restrict__ splits) {
  constexpr int N = 2 * K, N3 = N * N * N, K3 = K * K * K, SLOT = N3 + K3;
  const SplitTarget sp = splits[blockIdx.x];
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[sp.fn]);
  const int e0 = blockIdx.y * blockDim.x + threadIdx.x, stride = gridDim.y * blockDim.x;
  auto slot_sum = [&](int e) {
    const double* p = partials + (size_t)sp.first * SLOT + e;
    double s = 0.0;
    int q = 0;
    for (; q + 4 <= sp.count; q += 4) {
      const double v0 = p[(size_t)q * SLOT], v1 = p[(size_t)(q + 1) * SLOT],
                   v2 = p[(size_t)(q + 2) * SLOT], v3 = p[(size_t)(q + 3) * SLOT];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; q < sp.count; ++q) s += p[(size_t)q * SLOT];
    return s;
  };
  for (int e = e0; e < N3; e += stride) {
    const double s = slot_sum(e);
    const int a = e / (N * N), b = (e / N) % N, c = e % N;
    const int child = ((a / K) << 2) | ((b / K) << 1) | (c / K);
    out[(size_t)(sp.fc + child) * K3 + ((a % K) * K + (b % K)) * K + (c % K)] += s;
  }
  if (sp.sub >= 0)
    for (int e = e0; e < K3; e += stride) subbuf[(size_t)sp.sub * K3 + e] = slot_sum(N3 + e);
}

// ------------------------------------------------------- LDS layouts of the 4x4x4 operands
// The 64-bit LDS reads of gfx950 are served a quarter wave (16 lanes, fixed kk = lane >> 4)
// at a time; they are conflict free when those 16 lanes address 16 distinct 8-byte slots
// modulo 16.  A tensor read as a 4x4x4 A operand (lane 16 kk + 4 bb + ii reads
// T[4xs + kk][4yt + ii][4zq + bb]) is therefore stored quad-blocked,
// [x][y/4][z/4][y%4][z%4]; the exchange tensor, written with (b, z) and read with (a, b)
// varying inside a quarter wave, is stored in 4x4x4 cubes with the z slot rotated by a%4.
template <int Q>
__device__ __forceinline__ int qb_off(int x, int y, int z) {
  return x * (16 * Q * Q) + ((y >> 2) * Q + (z >> 2)) * 16 + (y & 3) * 4 + (z & 3);
}
template <int Q>
__device__ __forceinline__ int sk_off(int a, int b, int z) {
  return (((a >> 2) * Q + (b >> 2)) * Q + (z >> 2)) * 64 + (a & 3) * 16 + (b & 3) * 4 +
         (((z & 3) + (a & 3)) & 3);
}
// True when T[x][y][z] with strides (sx, sy, 1) is read conflict free as such an operand.
constexpr bool quarter_distinct(int sx, int sy) {
  for (int kk = 0; kk < 4; ++kk) {
    bool seen[16] = {};
    for (int ii = 0; ii < 4; ++ii)
      for (int bb = 0; bb < 4; ++bb) {
        const int slot = (kk * sx + ii * sy + bb) % 16;
        if (seen[slot]) return false;
        seen[slot] = true;
      }
  }
  return true;
}

// Global -> LDS staging: a thread issues its loads in chunks of CH before the matching LDS
// stores, so that a chunk costs one memory latency instead of one per element.  load(e) is
// called with a clamped index (no branch between the loads of a chunk); store(e, v) only
// for e = tid + 256 q < TOT.
template <int TOT, int CH, typename Ld, typename St>
__device__ __forceinline__ void stage_chunks(int tid, Ld load, St store) {
  constexpr int PER = (TOT + 255) / 256;
#pragma unroll
  for (int q0 = 0; q0 < PER; q0 += CH) {
    double v[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = load(min(tid + 256 * (q0 + q), TOT - 1));
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int e = tid + 256 * (q0 + q);
      if (q0 + q < PER && e < TOT) store(e, v[q]);
    }
  }
}
// The children block B_P (8 consecutive child slabs of k^3, i.e. one contiguous run of
// 8 k^3 doubles) into LDS, quad-blocked over the (2k)^3 index space.
template <int K, int Q, int CH, typename P>
__device__ __forceinline__ void stage_children_qb(double* __restrict__ Xs, P src, int tid) {
  constexpr int K2 = K * K, K3 = K * K * K;
  stage_chunks<8 * K3, CH>(
      tid, [&](int e) { return src[e]; },
      [&](int e, double v) {
        const int c = e / K3, r = e - c * K3;
        const int i = r / K2, j = (r / K) % K, m = r % K;
        Xs[qb_off<Q>(((c >> 2) & 1) * K + i, ((c >> 1) & 1) * K + j, (c & 1) * K + m)] = v;
      });
}
// s_P (k^3) into LDS zero-padded to KP^3 = (4 Q2)^3, quad-blocked.
template <int K, int Q2, int CH, typename P>
__device__ __forceinline__ void stage_scaling_qb(double* __restrict__ Ss, P sp, int tid) {
  constexpr int KP = 4 * Q2;
  stage_chunks<KP * KP * KP, CH>(
      tid,
      [&](int e) {
        const int x = e / (KP * KP), y = (e / KP) % KP, z = e % KP;
        const bool ok = x < K && y < K && z < K;
        return sp[ok ? (x * K + y) * K + z : 0];
      },
      [&](int e, double v) {
        const int x = e / (KP * KP), y = (e / KP) % KP, z = e % KP;
        Ss[qb_off<Q2>(x, y, z)] = (x < K && y < K && z < K) ? v : 0.0;
      });
}

// ------------------------------------------------------------------- apply (NS, MFMA)
// FP64 matrix-core version for even k (2k = 4Q).  Uses v_mfma_f64_4x4x4f64, which performs
// four independent 4x4x4 products ("blocks") per instruction at the full FP64 matrix rate
// of gfx950.  Lane l = 16 kk + 4 bb + ii holds A_bb[ii][kk] and B_bb[kk][ii]; the result
// D_bb[ii'][jj] sits in lane 16 ii' + 4 bb + jj.  With the block index carrying the z index
// inside a quad of z, the output of the x-contraction (rows y, columns a) is exactly the A
// operand of the y-contraction (rows a, contraction y), so steps 1 and 2 chain in registers.
// The z-contraction needs the full z range, so the y-contracted tensor is exchanged through
// LDS.  Work split for 4 waves: step 1+2 units are (a-quad, z-quad) pairs grouped by
// z-quad, step 3 units are (a-quad, b-quad) pairs; results stay in registers across all
// triples of the target.  The operator blocks of a triple (three (2k)^2 and three k^2
// blocks) sit in LDS; those of the next triple are loaded into registers while the current
// one finishes and written to LDS after it.  The quad-structured LDS accesses are
// bank-conflict free without padding.
template <int K>
__global__ __launch_bounds__(256) void apply_ns_mfma_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const double* const* __restrict__ r_tab, const double* const* __restrict__ t_tab,
    const double* const* __restrict__ c_tab, double* __restrict__ partials,
    double* __restrict__ subbuf) {
  constexpr int N = 2 * K, Q = N / 4, N2 = N * N, N3 = N * N * N, K2 = K * K, K3 = K * K * K;
  static_assert(N % 4 == 0, "k must be even");
  static_assert(Q >= 4 && Q <= 5, "register budget sized for 2k = 16 or 20");
  constexpr int EXTRA = (Q - 4) * Q;                 // (z-quad >= 4) pairs, round robin
  constexpr int EXTRA_PER_WAVE = (EXTRA + 3) / 4;
  constexpr int P3 = Q * Q;                          // step-3 (a-quad, b-quad) pairs
  constexpr int P3_PER_WAVE = (P3 + 3) / 4;
  // level-n subtraction -c (t x t x t) s_P on k^3 padded to KP = 4 Q2
  constexpr int Q2 = (K + 3) / 4, KP = 4 * Q2;
  constexpr int S3 = Q2 * Q2;
  // subtraction step-3 pairs go to the waves with fewer main step-3 pairs
  constexpr int SW = (P3 % 4 == 0) ? 4 : 3;
  constexpr int S3_PER_WAVE = (S3 + SW - 1) / SW;
  constexpr int OPS = 3 * N2 + 3 * K2;               // operator doubles per triple
  constexpr int OPS_PER_LANE = (OPS + 255) / 256;
  constexpr int CHUNK = 16;                          // children-block loads in flight
  __shared__ double Xs[N3];
  __shared__ double Zs[N3];
  __shared__ double Z2[KP * KP * KP];
  __shared__ double Os[OPS];                          // Rx^T, Ry^T, Rz^T, tx^T, ty^T, tz^T
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  const TargetRange tr = targets[blockIdx.x];
  const MRA_GLOBAL double* __restrict__ in = as_global(in_tab[tr.fn]);
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dR = as_global(r_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dT = as_global(t_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dc = as_global(c_tab[tr.fn]);
  const double* RXs = Os;
  const double* RYs = Os + N2;
  const double* RZs = Os + 2 * N2;
  const double* TXs = Os + 3 * N2;
  const double* TYs = Os + 3 * N2 + K2;
  const double* TZs = Os + 3 * N2 + 2 * K2;

  // operator blocks of item `it` into registers (this thread's share)
  auto fetch_ops = [&](const NSItem nx, double* reg) {
#pragma unroll
    for (int q = 0; q < OPS_PER_LANE; ++q) {
      const int e = tid + 256 * q;
      double v = 0.0;
      if (e < 3 * N2) {
        const int w = e / N2, r = e - w * N2;
        const int blk = w == 0 ? nx.rx : (w == 1 ? nx.ry : nx.rz);
        v = dR[(size_t)blk * N2 + r];
      } else if (e < OPS) {
        const int e2 = e - 3 * N2, w = e2 / K2, r = e2 - w * K2;
        const int blk = w == 0 ? nx.tx : (w == 1 ? nx.ty : nx.tz);
        v = dT[(size_t)blk * K2 + r];
      }
      reg[q] = v;
    }
  };
  auto store_ops = [&](const double* reg) {
#pragma unroll
    for (int q = 0; q < OPS_PER_LANE; ++q) {
      const int e = tid + 256 * q;
      if (e < OPS) Os[e] = reg[q];
    }
  };

  double acc[P3_PER_WAVE][Q];
#pragma unroll
  for (int p = 0; p < P3_PER_WAVE; ++p)
#pragma unroll
    for (int c = 0; c < Q; ++c) acc[p][c] = 0.0;
  double sacc[S3_PER_WAVE][Q2];
#pragma unroll
  for (int p = 0; p < S3_PER_WAVE; ++p)
#pragma unroll
    for (int c = 0; c < Q2; ++c) sacc[p][c] = 0.0;
  const bool with_sub = tr.sub >= 0;

  double spv[Q2][Q2];   // s_P fragment of the current source (waves < Q2)
#pragma unroll
  for (int xs = 0; xs < Q2; ++xs)
#pragma unroll
    for (int yt = 0; yt < Q2; ++yt) spv[xs][yt] = 0.0;

  // the item record of triple it + 1 is loaded at the start of triple it, long before the
  // operator prefetch needs it
  NSItem nxt{};
  double pre[OPS_PER_LANE], c_cur = 0.0, c_pre = 0.0;   // c_mu travels with the operators
  if (tr.beg < tr.end) {
    nxt = items[tr.beg];
    fetch_ops(nxt, pre);
    c_cur = dc[nxt.mu];
    store_ops(pre);
  }
  int loaded = -1;
  for (int it = tr.beg; it < tr.end; ++it) {
    const NSItem item = nxt;
    const bool more = it + 1 < tr.end;
    if (more) nxt = items[it + 1];
    if (item.src_fc != loaded) {
      __syncthreads();
      stage_children_qb<K, Q, CHUNK>(Xs, in + (size_t)item.src_fc * K3, tid);
      if (with_sub && wave < Q2) {
        // this wave's z-quad of s_P as step-1 A operands, zero outside k^3
        const MRA_GLOBAL double* __restrict__ sp = in + (size_t)item.src * K3;
        const int z = 4 * wave + lb;
#pragma unroll
        for (int xs = 0; xs < Q2; ++xs)
#pragma unroll
          for (int yt = 0; yt < Q2; ++yt) {
            const int x = 4 * xs + lk, y = 4 * yt + li;
            const bool ok = x < K && y < K && z < K;
            const double v = sp[ok ? (x * K + y) * K + z : 0];
            spv[xs][yt] = ok ? v : 0.0;
          }
      }
      loaded = item.src_fc;
    }
    __syncthreads();   // Xs and Os of this triple are in place
    const double cmu = c_cur;
    // B fragments: frag(ks, t) = R[4t + li][4ks + lk] = R^T[4ks + lk][4t + li]
    double rx[Q][Q], ry[Q][Q];
#pragma unroll
    for (int ks = 0; ks < Q; ++ks)
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        rx[ks][t] = RXs[(4 * ks + lk) * N + 4 * t + li];
        ry[ks][t] = RYs[(4 * ks + lk) * N + 4 * t + li];
      }
    // ---- steps 1 and 2 for the main z-quad of this wave (all a-quads)
    if (wave < Q) {
      const int zq = wave;
      double d1[Q][Q];   // [at][yt]
#pragma unroll
      for (int at = 0; at < Q; ++at)
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) d1[at][yt] = 0.0;
#pragma unroll
      for (int xs = 0; xs < Q; ++xs)
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) {
          double a = Xs[qb_off<Q>(4 * xs + lk, 4 * yt + li, 4 * zq + lb)];
#pragma unroll
          for (int at = 0; at < Q; ++at)
            d1[at][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, rx[xs][at], d1[at][yt], 0, 0, 0);
        }
#pragma unroll
      for (int at = 0; at < Q; ++at) {
        double d2[Q];
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) d2[bt] = 0.0;
#pragma unroll
        for (int ys = 0; ys < Q; ++ys)
#pragma unroll
          for (int bt = 0; bt < Q; ++bt)
            d2[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[at][ys], ry[ys][bt], d2[bt], 0, 0, 0);
#pragma unroll
        for (int bt = 0; bt < Q; ++bt)
          Zs[sk_off<Q>(4 * at + lk, 4 * bt + li, 4 * zq + lb)] = d2[bt];
      }
    }
    // ---- leftover (z-quad >= 4) pairs, round robin from the last wave (the first Q2 waves
    // also run the subtraction's steps 1 and 2)
#pragma unroll
    for (int e = 0; e < EXTRA_PER_WAVE; ++e) {
      const int p = (3 - wave) + 4 * e;
      if (p < EXTRA) {
        const int zq = 4 + p / Q, at = p % Q;
        double d1[Q];
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) d1[yt] = 0.0;
#pragma unroll
        for (int xs = 0; xs < Q; ++xs) {
          const double b = RXs[(4 * xs + lk) * N + 4 * at + li];
#pragma unroll
          for (int yt = 0; yt < Q; ++yt) {
            double a = Xs[qb_off<Q>(4 * xs + lk, 4 * yt + li, 4 * zq + lb)];
            d1[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, d1[yt], 0, 0, 0);
          }
        }
        double d2[Q];
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) d2[bt] = 0.0;
#pragma unroll
        for (int ys = 0; ys < Q; ++ys)
#pragma unroll
          for (int bt = 0; bt < Q; ++bt)
            d2[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[ys], ry[ys][bt], d2[bt], 0, 0, 0);
#pragma unroll
        for (int bt = 0; bt < Q; ++bt)
          Zs[sk_off<Q>(4 * at + lk, 4 * bt + li, 4 * zq + lb)] = d2[bt];
      }
    }
    // ---- subtraction, steps 1 and 2: (t_x, t_y) on s_P, one z-quad per wave
    if (with_sub && wave < Q2) {
      const int zq = wave;
      double tx[Q2][Q2], ty[Q2][Q2];
#pragma unroll
      for (int ks = 0; ks < Q2; ++ks)
#pragma unroll
        for (int t = 0; t < Q2; ++t) {
          const int r = 4 * ks + lk, cc = 4 * t + li;
          const bool ok = r < K && cc < K;
          tx[ks][t] = ok ? TXs[r * K + cc] : 0.0;
          ty[ks][t] = ok ? TYs[r * K + cc] : 0.0;
        }
      double d1[Q2][Q2];
#pragma unroll
      for (int at = 0; at < Q2; ++at)
#pragma unroll
        for (int yt = 0; yt < Q2; ++yt) d1[at][yt] = 0.0;
#pragma unroll
      for (int xs = 0; xs < Q2; ++xs)
#pragma unroll
        for (int yt = 0; yt < Q2; ++yt) {
#pragma unroll
          for (int at = 0; at < Q2; ++at)
            d1[at][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(spv[xs][yt], tx[xs][at], d1[at][yt], 0, 0, 0);
        }
#pragma unroll
      for (int at = 0; at < Q2; ++at) {
        double d2[Q2];
#pragma unroll
        for (int bt = 0; bt < Q2; ++bt) d2[bt] = 0.0;
#pragma unroll
        for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
          for (int bt = 0; bt < Q2; ++bt)
            d2[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[at][ys], ty[ys][bt], d2[bt], 0, 0, 0);
#pragma unroll
        for (int bt = 0; bt < Q2; ++bt)
          Z2[sk_off<Q2>(4 * at + lk, 4 * bt + li, 4 * zq + lb)] = d2[bt];
      }
    }
    // the next triple's operator blocks travel while step 3 runs
    if (more) {
      fetch_ops(nxt, pre);
      c_pre = dc[nxt.mu];
    }
    __syncthreads();
    // ---- subtraction, step 3: z-contraction with -c t_z
    if (with_sub) {
      double tz[Q2][Q2];
#pragma unroll
      for (int ks = 0; ks < Q2; ++ks)
#pragma unroll
        for (int t = 0; t < Q2; ++t) {
          const int r = 4 * ks + lk, cc = 4 * t + li;
          tz[ks][t] = (r < K && cc < K) ? -cmu * TZs[r * K + cc] : 0.0;
        }
#pragma unroll
      for (int e = 0; e < S3_PER_WAVE; ++e) {
        const int p = wave + SW * e;
        if (wave < SW && p < S3) {
          const int at3 = p / Q2, bt3 = p % Q2;
#pragma unroll
          for (int zs = 0; zs < Q2; ++zs) {
            double a = Z2[sk_off<Q2>(4 * at3 + lb, 4 * bt3 + li, 4 * zs + lk)];
#pragma unroll
            for (int ct = 0; ct < Q2; ++ct)
              sacc[e][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, tz[zs][ct], sacc[e][ct], 0, 0, 0);
          }
        }
      }
    }
    // ---- step 3: z-contraction into the register accumulators
    {
      double rz[Q][Q];
#pragma unroll
      for (int ks = 0; ks < Q; ++ks)
#pragma unroll
        for (int t = 0; t < Q; ++t) rz[ks][t] = cmu * RZs[(4 * ks + lk) * N + 4 * t + li];
#pragma unroll
      for (int e = 0; e < P3_PER_WAVE; ++e) {
        const int p = (3 - wave) + 4 * e;
        if (p < P3) {
          const int at3 = p / Q, bt3 = p % Q;
#pragma unroll
          for (int zs = 0; zs < Q; ++zs) {
            double a = Zs[sk_off<Q>(4 * at3 + lb, 4 * bt3 + li, 4 * zs + lk)];
#pragma unroll
            for (int ct = 0; ct < Q; ++ct)
              acc[e][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, rz[zs][ct], acc[e][ct], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();   // Zs, Z2 and Os are free
    if (more) {
      store_ops(pre);
      c_cur = c_pre;
    }
  }
  // ---- write the children block of the target
#pragma unroll
  for (int e = 0; e < P3_PER_WAVE; ++e) {
    const int p = (3 - wave) + 4 * e;
    if (p < P3) {
      const int at3 = p / Q, bt3 = p % Q;
      const int a = 4 * at3 + lb, b = 4 * bt3 + lk;
      if (tr.partial >= 0) {
        double* dst = partials + (size_t)tr.partial * (N3 + K3);
#pragma unroll
        for (int ct = 0; ct < Q; ++ct) dst[(a * N + b) * N + 4 * ct + li] = acc[e][ct];
      } else {
#pragma unroll
        for (int ct = 0; ct < Q; ++ct) {
          const int c = 4 * ct + li;
          const int child = ((a / K) << 2) | ((b / K) << 1) | (c / K);
          out[(size_t)(tr.fc + child) * K3 + ((a % K) * K + (b % K)) * K + (c % K)] += acc[e][ct];
        }
      }
    }
  }
  if (with_sub) {
#pragma unroll
    for (int e = 0; e < S3_PER_WAVE; ++e) {
      const int p = wave + SW * e;
      if (wave < SW && p < S3) {
        const int a = 4 * (p / Q2) + lb, b = 4 * (p % Q2) + lk;
#pragma unroll
        for (int ct = 0; ct < Q2; ++ct) {
          const int c = 4 * ct + li;
          if (a < K && b < K && c < K) {
            if (tr.partial >= 0)
              partials[(size_t)tr.partial * (N3 + K3) + N3 + (a * K + b) * K + c] = sacc[e][ct];
            else
              subbuf[(size_t)tr.sub * K3 + (a * K + b) * K + c] = sacc[e][ct];
          }
        }
      }
    }
  }
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS accesses and meets the
// other waves, but, unlike __syncthreads, not for global loads still in flight (those
// stage the next triple's blocks and are waited for where they are stored to LDS).  The
// memory clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Scheduling pattern for a group of matrix products and the memory instructions issued
// beside them (LDS reads of the next group's operands, global loads and LDS stores of the
// next triple's blocks): rounds of PM products followed by at most one instruction of each
// kind (NR LDS reads, NV global loads, NW LDS stores in all), then the remaining products.
// The memory instructions trickle out behind the products instead of holding up the
// in-order wave in one burst.
template <int NR, int NV, int NW, int PM>
__device__ __forceinline__ void interleave_mem() {
  constexpr int NI = NR > NV ? (NR > NW ? NR : NW) : (NV > NW ? NV : NW);
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, PM, 0);              // matrix products
    if (i < NR) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
    if (i < NV) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // global load
    if (i < NW) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // LDS store
  }
  __builtin_amdgcn_sched_group_barrier(0x008, 64, 0);
}

// Copies 16 bytes per lane from base + voff (bytes) into LDS at dst + 16 * lane with a buffer
// load that writes LDS directly; the descriptor bounds the read to nbytes from base (lanes
// past the end read zeros).  The copy completes on the vector-memory counter only.
__device__ __forceinline__ void lds_copy16(const double* base, int nbytes, MRA_LDS void* dst,
                                           int voff) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nbytes, 0x00020000);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 16, voff, 0, 0, 0);
}

// The value of v, opaque to the optimiser (it cannot hoist computations on the result out
// of the enclosing loop).
__device__ __forceinline__ int opaque_int(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Workgroup barrier for LDS written and read by this wave's own instructions, with the
// wait given by the caller: waitcnt (an s_waitcnt immediate) should include lgkmcnt(0), so
// that this wave's LDS reads and writes are done.  Unlike __syncthreads() it does not
// imply a wait for every LDS copy in flight (a workgroup fence must cover those); the
// empty asm statements keep the compiler from moving memory accesses across it.
template <int WAITCNT>
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(WAITCNT);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int B>
struct BufTag {
  static constexpr int value = B;
};
template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};
// ------------------------------------------------------------ apply (NS, MFMA, factored)
// FP64 matrix-core kernel for k = 10 that shares contractions between the triples of a
// target.  Mode products along different axes commute and a target's result is a sum over
// its triples, so with the triples ordered by (term mu, dz, dy, dx)
//   acc_T = sum_{mu, dz} c_mu R_z x_z [ sum_{dy} R_y x_y [ sum_{dx} R_x x_x B_{T - d} ] ]
// (R_x = R^{n, dx}_mu etc.): step 1 (contract x) runs once per triple and accumulates in
// registers, step 2 (contract y) once per (mu, dz, dy) group, step 3 (contract z, through
// the LDS exchange tensor) once per (mu, dz) group.  The level-n subtraction -c (t x t x t)
// s_P is factored the same way by apply_ns_fac_sub_kernel.  The lane mapping of each step
// is that of apply_ns_mfma_kernel (block index = z inside a z-quad for steps 1 and 2).
// The children block of the next triple and its operator blocks are copied into the other
// half of two LDS buffers (16-byte buffer loads that write LDS directly) while the current
// triple runs; the source block is stored row-major [x][y][z], whose row stride 2k = 20 (= 4 mod
// 16) keeps the step-1 reads bank-conflict free.  The buffer a triple has finished with
// holds the exchange tensors of step 3.  One wave per SIMD hides no latency by switching
// waves, so each step is software-pipelined by hand (operands of the next group read into
// a register double buffer) and its memory instructions are interleaved with the matrix
// products by scheduling-group hints.
template <int K>
__global__ __launch_bounds__(256) void apply_ns_fac_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const double* const* __restrict__ r_tab, const double* const* __restrict__ t_tab,
    const double* const* __restrict__ c_tab, double* __restrict__ partials,
    double* __restrict__ subbuf, const int ntargets, int* __restrict__ next_target) {
  constexpr int N = 2 * K, Q = N / 4, N2 = N * N, N3 = N * N * N, K2 = K * K, K3 = K * K * K;
  static_assert(Q == 5, "row stride 2k = 20 and the wave split below are for k = 10");
  constexpr int EXTRA = (Q - 4) * Q, EPW = (EXTRA + 3) / 4;   // (z-quad 4, a-quad) units
  static_assert(EXTRA == Q && EPW == 2, "the z-quad-4 units are a-quads 3 - wave and 7 - wave");
  constexpr int P3 = Q * Q, P3PW = (P3 + 3) / 4;              // step-3 (a-quad, b-quad) pairs
  // copy geometry, in rows of 64 granules of 16 bytes (two doubles): every wave copies XQ
  // source rows and one row of each operator block per triple; the buffers are padded so
  // that rows past the end of a block land in padding instead of being branched around.
  // An operator block (N^2 doubles) takes OB = 4 rows, so that each copy instruction reads
  // one block: R_x^T, R_y^T, R_z^T start at 0, OBD and 2 OBD doubles.
  constexpr int XG = N3 / 2, XI = (XG + 63) / 64, XQ = (XI + 3) / 4, XPAD = 128 * 4 * XQ;
  constexpr int OB = (N2 / 2 + 63) / 64, OBD = 128 * OB, OPAD = 3 * OBD;
  static_assert(XQ == 16 && OB == 4, "the copy schedule below moves 4 x 4 + 3 rows per wave");
  static_assert(N2 % 2 == 0 && K2 % 2 == 0 && K % 2 == 0, "granules never straddle rows");
  static_assert(64 * Q * Q * Q <= XPAD, "the exchange tensor fits in a source buffer");
  // the two halves of each double buffer are separate objects, so that the compiler can
  // tell reads of one from the stores into the other
  __shared__ __attribute__((aligned(16))) double Xs0[XPAD];
  __shared__ __attribute__((aligned(16))) double Xs1[XPAD];
  __shared__ __attribute__((aligned(16))) double Os0[OPAD];
  __shared__ __attribute__((aligned(16))) double Os1[OPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  // granule g of the row-major source block is (x, y, z = 2 zp), g = (x N + y) N/2 + zp;
  // this lane's offsets (doubles, from the first child's slab) for its wave's instructions
  int xoff[XQ];
#pragma unroll
  for (int q = 0; q < XQ; ++q) {
    const int g = min(64 * (wave + 4 * q) + lane, XG - 1);
    const int x = g / (N2 / 2), r = g - x * (N2 / 2), y = r / (N / 2), z = 2 * (r - y * (N / 2));
    const int child = ((x / K) << 2) | ((y / K) << 1) | (z / K);
    xoff[q] = child * K3 + ((x % K) * K + y % K) * K + z % K;
  }
  // Persistent workgroups: each takes the next target range from a counter until none is
  // left, so a CU that finishes early starts the next range at once (the ranges come
  // longest first) instead of waiting for the hardware's round-robin over the dies.
  __shared__ int s_next;
  for (;;) {
  if (tid == 0) s_next = atomicAdd(next_target, 1);
  __syncthreads();
  const int ti = s_next;
  __syncthreads();   // every wave has read s_next
  if (ti >= ntargets) break;
  const TargetRange tr = targets[ti];
  const MRA_GLOBAL double* __restrict__ in = as_global(in_tab[tr.fn]);
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dc = as_global(c_tab[tr.fn]);
  // The next triple's blocks are copied into the free buffer halves by buffer loads that
  // write LDS directly (no registers; they complete on the vector-memory counter only, so
  // the LDS reads of the running triple never wait for them), in five parts (four of the
  // source block, one of the operators) spread over the x-quad groups of step 1: a burst
  // of memory instructions would stall the in-order wave until the memory pipeline takes
  // them.  The buffer descriptors bound each copy to its block: lanes past the end of an
  // operator block read zeros.
  const double* const in_g = in_tab[tr.fn];
  const double* const dR_g = r_tab[tr.fn];
  auto fetch_part = [&](const NSItem nx, const int part, double* dst, double* dop) {
    if (part < 4) {
#pragma unroll
      for (int q = 4 * part; q < 4 * part + 4; ++q)
        lds_copy16(in_g + (size_t)nx.src_fc * K3, 8 * K3 * 8, (MRA_LDS void*)(dst + 128 * (wave + 4 * q)),
                   8 * xoff[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int blk = q == 0 ? nx.rx : q == 1 ? nx.ry : nx.rz;
        lds_copy16(dR_g + (size_t)blk * N2, N2 * 8, (MRA_LDS void*)(dop + q * OBD + 128 * wave),
                   16 * (64 * wave + lane));
      }
    }
  };
  double d1[Q][Q], d2[Q][Q], d1e[EPW][Q], d2e[EPW][Q], acc[P3PW][Q];
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int j = 0; j < Q; ++j) d1[i][j] = d2[i][j] = 0.0;
#pragma unroll
  for (int e = 0; e < EPW; ++e)
#pragma unroll
    for (int j = 0; j < Q; ++j) d1e[e][j] = d2e[e][j] = 0.0;
#pragma unroll
  for (int e = 0; e < P3PW; ++e)
#pragma unroll
    for (int j = 0; j < Q; ++j) acc[e][j] = 0.0;

  // item records two triples ahead: the next one is in registers when its loads are issued
  NSItem cur{}, nxt{};
  double c_cur = 0.0, c_pre = 0.0;
  if (tr.beg < tr.end) {
    cur = items[tr.beg];
    c_cur = dc[cur.mu];
#pragma unroll
    for (int part = 0; part < 5; ++part) fetch_part(cur, part, Xs0, Os0);
    nxt = items[min(tr.beg + 1, tr.end - 1)];
  }
  // one triple; BUF is a compile-time constant so that the compiler can tell the reads of
  // this triple's buffer halves from the stores into the other halves
  auto triple = [&](const int it, auto buf_tag) {
    constexpr int buf = decltype(buf_tag)::value;
    double* const Xc = buf == 0 ? Xs0 : Xs1;   // this triple's halves
    double* const Oc = buf == 0 ? Os0 : Os1;
    double* const Xn = buf == 0 ? Xs1 : Xs0;   // the next triple's halves
    double* const On = buf == 0 ? Os1 : Os0;
    const NSItem item = cur;
    const bool more = it + 1 < tr.end;
    // this wave's copies of triple it are complete; after the barrier all of them are, and
    // every wave is done with triple it - 1 (the other buffer halves are free)
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    const NSItem nn = items[min(it + 2, tr.end - 1)];   // uniform address: scalar loads
    if (more) {
      c_pre = dc[nxt.mu];
    }
    const bool dy_end = !more || nxt.rz != item.rz || nxt.ry != item.ry;
    const bool dz_end = !more || nxt.rz != item.rz;
    const double* X = Xc;
    const double cmu = c_cur;
    const double* RXs = Oc;
    const double* RYs = Oc + OBD;
    const double* RZs = Oc + 2 * OBD;
    // One wave per SIMD hides no latency by switching waves, so every step is software-
    // pipelined by hand: the LDS operands of group g + 1 are read into the other half of a
    // register double buffer before the matrix products of group g, and scheduling
    // barriers keep the compiler from sinking those reads next to their uses.
    // step 2's operands of its first y-quad are read during the last x-quad group of step 1
    // (whether or not the triple ends a y group)
    double ry[2][Q];
    auto load2 = [&](const int ys, const int b) {
#pragma unroll
      for (int bt = 0; bt < Q; ++bt) ry[b][bt] = RYs[(4 * ys + lk) * N + 4 * bt + li];
    };
    // ---- step 1, per x-quad xs: the main z-quad of this wave (all a-quads) and the
    // z-quad-4 units.  Every wave runs EPW = 2 of those units, so that the block has no
    // wave-dependent branch; a wave with one real unit repeats it into an accumulator that
    // is never stored (it would otherwise wait for the busiest wave anyway).
    {
      const int zq = wave;
      const int ate[EPW] = {min(3 - wave, EXTRA - 1), min(7 - wave, EXTRA - 1)};
      double opA[2][Q], opE[2][Q], opR[2][Q], opB[2][EPW];
      auto load1 = [&](const int xs, const int b) {
        const double* Rr = RXs + (4 * xs + lk) * N + li;
        const double* Xr = X + ((4 * xs + lk) * N + li) * N + lb;
#pragma unroll
        for (int at = 0; at < Q; ++at) opR[b][at] = Rr[4 * at];
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) opA[b][yt] = Xr[4 * yt * N + 4 * zq];
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) opE[b][yt] = Xr[4 * yt * N + 16];
#pragma unroll
        for (int e = 0; e < EPW; ++e) opB[b][e] = Rr[4 * ate[e]];
      };
      load1(0, 0);
#pragma unroll
      for (int xs = 0; xs < Q; ++xs) {
        const int b = xs & 1;
        if (xs + 1 < Q) load1(xs + 1, b ^ 1);
        // the next triple's blocks (for the last triple of the list, nxt repeats the
        // current item: harmless loads into the free halves): the operator blocks with the
        // first source quarter, the other quarters in the next groups, so that the last
        // copy has a whole x-quad group and the later steps to land
        if (xs == 0) fetch_part(nxt, 4, Xn, On);
        if (xs < 4) fetch_part(nxt, xs, Xn, On);
        if (xs == 4) load2(0, 0);
#pragma unroll
        for (int yt = 0; yt < Q; ++yt)
#pragma unroll
          for (int at = 0; at < Q; ++at)
            d1[at][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(opA[b][yt], opR[b][at], d1[at][yt], 0, 0, 0);
#pragma unroll
        for (int e = 0; e < EPW; ++e)
#pragma unroll
          for (int yt = 0; yt < Q; ++yt)
            d1e[e][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(opE[b][yt], opB[b][e], d1e[e][yt], 0, 0, 0);
        if (xs == 0) interleave_mem<11, 7, 0, 2>();
        else if (xs + 1 < Q) interleave_mem<11, 4, 0, 2>();
        else interleave_mem<3, 0, 0, 3>();
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // ---- step 2 at the end of a (mu, dz, dy) group
    if (dy_end) {
#pragma unroll
      for (int ys = 0; ys < Q; ++ys) {
        const int b = ys & 1;
        if (ys + 1 < Q) load2(ys + 1, b ^ 1);
#pragma unroll
        for (int at = 0; at < Q; ++at)
#pragma unroll
          for (int bt = 0; bt < Q; ++bt)
            d2[at][bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[at][ys], ry[b][bt], d2[at][bt], 0, 0, 0);
#pragma unroll
        for (int e = 0; e < EPW; ++e)
#pragma unroll
          for (int bt = 0; bt < Q; ++bt)
            d2e[e][bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1e[e][ys], ry[b][bt], d2e[e][bt], 0, 0, 0);
        if (ys + 1 < Q) interleave_mem<5, 0, 0, 4>();
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int j = 0; j < Q; ++j) d1[i][j] = 0.0;
#pragma unroll
      for (int e = 0; e < EPW; ++e)
#pragma unroll
        for (int j = 0; j < Q; ++j) d1e[e][j] = 0.0;
    }
    // ---- step 3 at the end of a (mu, dz) group, through this triple's source buffer
    if (dz_end) {
      double* Zs = Xc;
      double rz[Q][Q];   // c_mu R_z^T fragments, read while the waves meet
#pragma unroll
      for (int zs = 0; zs < Q; ++zs)
#pragma unroll
        for (int ct = 0; ct < Q; ++ct) rz[zs][ct] = cmu * RZs[(4 * zs + lk) * N + 4 * ct + li];
      lds_barrier();   // every wave is done reading the source block
      {
        const int zq = wave;
#pragma unroll
        for (int at = 0; at < Q; ++at)
#pragma unroll
          for (int bt = 0; bt < Q; ++bt) {
            Zs[sk_off<Q>(4 * at + lk, 4 * bt + li, 4 * zq + lb)] = d2[at][bt];
            d2[at][bt] = 0.0;
          }
      }
#pragma unroll
      for (int e = 0; e < EPW; ++e) {
        const int p = (3 - wave) + 4 * e;
        if (p < EXTRA) {
          const int zq = 4 + p / Q, at = p % Q;
#pragma unroll
          for (int bt = 0; bt < Q; ++bt) {
            Zs[sk_off<Q>(4 * at + lk, 4 * bt + li, 4 * zq + lb)] = d2e[e][bt];
            d2e[e][bt] = 0.0;
          }
        }
      }
      lds_barrier();
      // as in step 1, a wave with fewer real pairs repeats its last one (never stored)
      double za[2][Q];
      auto load3 = [&](const int e, const int b) {
        const int p = min((3 - wave) + 4 * e, P3 - 1);
        const int at3 = p / Q, bt3 = p % Q;
#pragma unroll
        for (int zs = 0; zs < Q; ++zs) za[b][zs] = Zs[sk_off<Q>(4 * at3 + lb, 4 * bt3 + li, 4 * zs + lk)];
      };
      load3(0, 0);
#pragma unroll
      for (int e = 0; e < P3PW; ++e) {
        const int b = e & 1;
        if (e + 1 < P3PW) load3(e + 1, b ^ 1);
#pragma unroll
        for (int zs = 0; zs < Q; ++zs)
#pragma unroll
          for (int ct = 0; ct < Q; ++ct)
            acc[e][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(za[b][zs], rz[zs][ct], acc[e][ct], 0, 0, 0);
        if (e + 1 < P3PW) interleave_mem<5, 0, 0, 3>();
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    c_cur = c_pre;
    cur = nxt;
    nxt = nn;
  };
  for (int it = tr.beg; it < tr.end; it += 2) {
    triple(it, BufTag<0>{});
    if (it + 1 < tr.end) triple(it + 1, BufTag<1>{});
  }
  // ---- write the children block of the target (each element owned by one lane)
#pragma unroll
  for (int e = 0; e < P3PW; ++e) {
    const int p = (3 - wave) + 4 * e;
    if (p < P3) {
      const int at3 = p / Q, bt3 = p % Q;
      const int a = 4 * at3 + lb, b = 4 * bt3 + lk;
      if (tr.partial >= 0) {
        double* dst = partials + (size_t)tr.partial * (N3 + K3);
#pragma unroll
        for (int ct = 0; ct < Q; ++ct) dst[(a * N + b) * N + 4 * ct + li] = acc[e][ct];
      } else {
#pragma unroll
        for (int ct = 0; ct < Q; ++ct) {
          const int c = 4 * ct + li;
          const int child = ((a / K) << 2) | ((b / K) << 1) | (c / K);
          out[(size_t)(tr.fc + child) * K3 + ((a % K) * K + (b % K)) * K + (c % K)] += acc[e][ct];
        }
      }
    }
  }
  // the last triple's copies into the free halves have landed before the buffers are reused
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  }
}

// Level-n subtraction of the factored kernel: sub_T = -sum c_mu (t_x x t_y x t_z) s_P over
// the triples of a target, with the same grouping (step 1 per triple, step 2 per (mu, dz, dy)
// group, step 3 per (mu, dz) group) on the k^3 scaling blocks, zero-padded to KP = 4 Q2.
// The work per triple is small, so the four waves of a workgroup split a target range (a
// counter hands the ranges out) into four runs of consecutive triples, each closing its own
// groups, and meet only to add their four results in a fixed order.  A wave computes all Q2
// z-quads of its triples, turns the step-2 result around through an exchange region of its
// own for step 3, and copies the s_P block and the t blocks of the next triple into the
// other slot of a private LDS double buffer (LDS-writing buffer loads).
template <int K>
__global__ __launch_bounds__(256) void apply_ns_fac_sub_kernel(
    const double* const* __restrict__ in_tab, const NSItem* __restrict__ items,
    const TargetRange* __restrict__ targets, const double* const* __restrict__ t_tab,
    const double* const* __restrict__ c_tab, double* __restrict__ partials,
    double* __restrict__ subbuf, const int ntargets, int* __restrict__ next_target) {
  constexpr int N = 2 * K, N3 = N * N * N, K2 = K * K, K3 = K * K * K;
  constexpr int Q2 = (K + 3) / 4, S3 = Q2 * Q2;
  static_assert(Q2 == 3, "three z-quads of KP = 12");
  static_assert(K2 % 2 == 0 && K2 / 2 <= 64, "a t block fits one row of granules");
  constexpr int SPG = K3 / 2, SPR = (SPG + 63) / 64;   // s_P granules, rows of 64
  constexpr int SPD = 128 * SPR;                        // s_P slot (doubles)
  constexpr int TD = 3 * 128;                           // t slot: t_x^T, t_y^T, t_z^T rows
  // exchange region [a][b][z] over the padded 4 Q2 cube with strides (ZA, ZB, 1): the
  // step-3 writes and reads then need no masks, and ZB = 4 Q2, ZA = 1 mod 32 spread both
  // access patterns over distinct banks
  constexpr int ZB = 4 * Q2, ZA = ((ZB * (ZB - 1) + ZB - 1) / 32 + 1) * 32 + 1;
  constexpr int ZW = (ZB - 1) * ZA + (ZB - 1) * ZB + ZB;   // doubles per wave (>= K3)
  static_assert(ZW >= K3 && ZA >= ZB * ZB, "exchange layout");
  constexpr int WS = 2 * SPD + 2 * TD + ZW;             // one wave's LDS: two slots + exchange
  constexpr int NCP = SPR + 3;                          // copy instructions per triple
  static_assert(NCP < 16, "vmcnt field");
  // the two slots are separate objects, so that the compiler can tell the reads of one
  // from the copies into the other
  __shared__ __attribute__((aligned(16))) double Sp0[4 * SPD];
  __shared__ __attribute__((aligned(16))) double Sp1[4 * SPD];
  __shared__ __attribute__((aligned(16))) double Tt0[4 * TD];
  __shared__ __attribute__((aligned(16))) double Tt1[4 * TD];
  __shared__ double Zx[4 * ZW];                         // exchange regions
  __shared__ int s_next;
  static_assert(4 * WS * 8 <= 160 * 1024, "LDS");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  double* const Z2s = Zx + wave * ZW;
  // LDS layout of an s_P slot: granule zp (two doubles along z) of row (x, y) goes to
  // granule (zp + y) mod K/2 of that row, so that the four y rows of a fragment read fall
  // on distinct banks; this lane's copy offsets (bytes into the block; past the end for
  // the padding granules, which read zeros)
  static_assert(K % 2 == 0, "rows of whole granules");
  constexpr int RG = K / 2;   // granules per (x, y) row
  int spoff[SPR];
#pragma unroll
  for (int r = 0; r < SPR; ++r) {
    const int j = 64 * r + lane, row = j / RG, y = row % K;
    spoff[r] = j < SPG ? 16 * (row * RG + (j % RG + 2 * RG - y) % RG) : 8 * K3;
  }
  for (;;) {
    // the workgroup's next target range; this wave's run of it
    if (tid == 0) s_next = atomicAdd(next_target, 1);
    __syncthreads();
    const int ti = s_next;
    __syncthreads();
    if (ti >= ntargets) break;
    const TargetRange tr = targets[ti];
    if (tr.sub < 0) continue;   // level 0: no subtraction (uniform over the workgroup)
    const int len = tr.end - tr.beg;
    // (wave-uniform bounds, so that the item records are read through the scalar cache)
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    const int wb = tr.beg + wu * len / 4, we = tr.beg + (wu + 1) * len / 4;
    const double* const in_g = in_tab[tr.fn];
    const double* const dT_g = t_tab[tr.fn];
    const __attribute__((address_space(4))) double* __restrict__ dc =
        (const __attribute__((address_space(4))) double*)c_tab[tr.fn];
    // copies of item nx into this wave's part of slot (Sp, Tt)
    auto copy = [&](const NSItem nx, double* Sp, double* Tt) {
      double* sd = Sp + wave * SPD;
      const double* sb = in_g + (size_t)nx.src * K3;
#pragma unroll
      for (int r = 0; r < SPR; ++r)
        lds_copy16(sb, K3 * 8, (MRA_LDS void*)(sd + 128 * r), spoff[r]);
      double* td = Tt + wave * TD;
      lds_copy16(dT_g + (size_t)nx.tx * K2, K2 * 8, (MRA_LDS void*)td, 16 * lane);
      lds_copy16(dT_g + (size_t)nx.ty * K2, K2 * 8, (MRA_LDS void*)(td + 128), 16 * lane);
      lds_copy16(dT_g + (size_t)nx.tz * K2, K2 * 8, (MRA_LDS void*)(td + 256), 16 * lane);
    };
    // s_P[x][y][z] as an A operand, without zeroing: the lanes outside k read an element
    // of the block (finite), which the zero rows and columns of the t fragments cancel or
    // which lands in padding that is never stored
    auto spraw = [&](const double* S, int xs, int yt, int zq) {
      const int x = 4 * xs + lk, y = 4 * yt + li, z = 4 * zq + lb;
      const bool ok = x < K && y < K && z < K;
      const int row = x * K + y;
      return S[ok ? 2 * (row * RG + ((z >> 1) + y) % RG) + (z & 1) : 0];
    };
    // t^T[r][c] as a B operand, zero outside k (clamped index, selected at use)
    auto tfrag = [&](const double* T, int rq, int cq) {
      const int r = 4 * rq + lk, c = 4 * cq + li;
      const bool ok = r < K && c < K;
      const double v = T[ok ? r * K + c : 0];
      return ok ? v : 0.0;
    };
    double d1[Q2][Q2][Q2], d2[Q2][Q2][Q2], acc[S3][Q2];   // [zq][a][b]; [pair][c]
#pragma unroll
    for (int z = 0; z < Q2; ++z)
#pragma unroll
      for (int i = 0; i < Q2; ++i)
#pragma unroll
        for (int j = 0; j < Q2; ++j) d1[z][i][j] = d2[z][i][j] = 0.0;
#pragma unroll
    for (int e = 0; e < S3; ++e)
#pragma unroll
      for (int j = 0; j < Q2; ++j) acc[e][j] = 0.0;
    NSItem cur{}, nxt{};
    if (wb < we) {
      cur = items[wb];
      nxt = items[min(wb + 1, we - 1)];
      copy(cur, Sp0, Tt0);
    }
    auto triple = [&](const int it, auto buf_tag) {
      constexpr int buf = decltype(buf_tag)::value;
      const double* const S = (buf == 0 ? Sp0 : Sp1) + wave * SPD;
      const double* const T = (buf == 0 ? Tt0 : Tt1) + wave * TD;
      const NSItem item = cur;
      const bool more = it + 1 < we;
      const NSItem nn = items[min(it + 2, we - 1)];   // uniform address: scalar loads
      const double cmu = dc[item.mu];
      // copy of the next triple (for the last one, a harmless repeat into the free slot),
      // then wait for this triple's copies: all but the NCP just issued have landed
      copy(nxt, buf == 0 ? Sp1 : Sp0, buf == 0 ? Tt1 : Tt0);
      __builtin_amdgcn_s_waitcnt(0x0F70 | NCP);   // vmcnt(NCP)
      const bool dy_end = !more || nxt.rz != item.rz || nxt.ry != item.ry;
      const bool dz_end = !more || nxt.rz != item.rz;
      // step 1 (contract x) for the three z-quads, the fragments of x-quad xs + 1 read
      // while those of xs are used (and the t_y fragments of step 2 during the last)
      double fa[2][Q2][Q2], fb[2][Q2], ty[Q2][Q2];
      auto load1 = [&](int xs, double (&fs)[Q2][Q2], double (&ft)[Q2]) {
#pragma unroll
        for (int at = 0; at < Q2; ++at) ft[at] = tfrag(T, xs, at);
#pragma unroll
        for (int zq = 0; zq < Q2; ++zq)
#pragma unroll
          for (int yt = 0; yt < Q2; ++yt) fs[zq][yt] = spraw(S, xs, yt, zq);
      };
      load1(0, fa[0], fb[0]);
#pragma unroll
      for (int xs = 0; xs < Q2; ++xs) {
        const int bb = xs & 1;
        if (xs + 1 < Q2) {
          load1(xs + 1, fa[bb ^ 1], fb[bb ^ 1]);
        } else {
#pragma unroll
          for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
            for (int bt = 0; bt < Q2; ++bt) ty[ys][bt] = tfrag(T + 128, ys, bt);
        }
#pragma unroll
        for (int zq = 0; zq < Q2; ++zq)
#pragma unroll
          for (int yt = 0; yt < Q2; ++yt)
#pragma unroll
            for (int at = 0; at < Q2; ++at)
              d1[zq][at][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[bb][zq][yt], fb[bb][at],
                                                                  d1[zq][at][yt], 0, 0, 0);
        interleave_mem<12, 0, 0, 2>();
        __builtin_amdgcn_sched_barrier(0);
      }
      // step 2 (contract y) at the end of a (mu, dz, dy) group
      if (dy_end) {
#pragma unroll
        for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
          for (int zq = 0; zq < Q2; ++zq)
#pragma unroll
            for (int at = 0; at < Q2; ++at)
#pragma unroll
              for (int bt = 0; bt < Q2; ++bt)
                d2[zq][at][bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[zq][at][ys], ty[ys][bt],
                                                                    d2[zq][at][bt], 0, 0, 0);
#pragma unroll
        for (int z = 0; z < Q2; ++z)
#pragma unroll
          for (int i = 0; i < Q2; ++i)
#pragma unroll
            for (int j = 0; j < Q2; ++j) d1[z][i][j] = 0.0;
      }
      // step 3 (contract z) at the end of a (mu, dz) group, through this wave's exchange
      // (the whole padded cube is written, so that the padding lanes read finite values
      // that the zero rows of t_z cancel or that land in padding); the exchange reads of
      // pair p + 1 are issued while pair p is used
      if (dz_end) {
        double tz[Q2][Q2];
#pragma unroll
        for (int zs = 0; zs < Q2; ++zs)
#pragma unroll
          for (int ct = 0; ct < Q2; ++ct) tz[zs][ct] = tfrag(T + 256, zs, ct);
#pragma unroll
        for (int zq = 0; zq < Q2; ++zq)
#pragma unroll
          for (int at = 0; at < Q2; ++at)
#pragma unroll
            for (int bt = 0; bt < Q2; ++bt) {
              const int a = 4 * at + lk, b = 4 * bt + li, z = 4 * zq + lb;
              Z2s[a * ZA + b * ZB + z] = d2[zq][at][bt];
              d2[zq][at][bt] = 0.0;
            }
#pragma unroll
        for (int zs = 0; zs < Q2; ++zs)
#pragma unroll
          for (int ct = 0; ct < Q2; ++ct) tz[zs][ct] *= -cmu;
        double zr[2][Q2];
        auto load3 = [&](int p, double (&v)[Q2]) {
          const int a = 4 * (p / Q2) + lb, b = 4 * (p % Q2) + li;
#pragma unroll
          for (int zs = 0; zs < Q2; ++zs)
            v[zs] = Z2s[a * ZA + b * ZB + 4 * zs + lk];
        };
        load3(0, zr[0]);
#pragma unroll
        for (int p = 0; p < S3; ++p) {
          const int bb = p & 1;
          if (p + 1 < S3) load3(p + 1, zr[bb ^ 1]);
#pragma unroll
          for (int zs = 0; zs < Q2; ++zs)
#pragma unroll
            for (int ct = 0; ct < Q2; ++ct)
              acc[p][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(zr[bb][zs], tz[zs][ct], acc[p][ct], 0, 0, 0);
          interleave_mem<3, 0, 0, 3>();
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      cur = nxt;
      nxt = nn;
    };
    for (int it = wb; it < we; it += 2) {
      triple(it, BufTag<0>{});
      if (it + 1 < we) triple(it + 1, BufTag<1>{});
    }
    // the last triple's copy into the free slot has landed before the slots are reused
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    // this wave's result into its exchange region (after its own last step-3 reads, in
    // order), then the four results added in wave order
#pragma unroll
    for (int p = 0; p < S3; ++p) {
      const int a = 4 * (p / Q2) + lb, b = 4 * (p % Q2) + lk;
#pragma unroll
      for (int ct = 0; ct < Q2; ++ct) {
        const int c = 4 * ct + li;
        if (a < K && b < K && c < K) Z2s[(a * K + b) * K + c] = acc[p][ct];
      }
    }
    lds_barrier();
    double* const dst = tr.partial >= 0 ? partials + (size_t)tr.partial * (N3 + K3) + N3
                                        : subbuf + (size_t)tr.sub * K3;
    for (int e = tid; e < K3; e += 256)
      dst[e] = ((Zx[e] + Zx[ZW + e]) + Zx[2 * ZW + e]) + Zx[3 * ZW + e];
    // (the next range's first barrier keeps the exchange regions until every wave has read)
  }
}

// --------------------------------------------------------------------------- apply (std)
template <int K>
__global__ __launch_bounds__(round64(K * K)) void apply_std_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const double* const* __restrict__ t_tab, const double* const* __restrict__ c_tab,
    double scale) {
  constexpr int K2 = K * K, K3 = K * K * K, ZP = K + 1;
  __shared__ double S[K * K * ZP];
  __shared__ double W[K * K * ZP];
  const int tid = threadIdx.x;
  const TargetRange tr = targets[blockIdx.x];
  const MRA_GLOBAL double* __restrict__ in = as_global(in_tab[tr.fn]);
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dT = as_global(t_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dc = as_global(c_tab[tr.fn]);
  double acc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) acc[c] = 0.0;
  int loaded = -1;
  for (int it = tr.beg; it < tr.end; ++it) {
    const NSItem item = items[it];
    if (item.src != loaded) {
      __syncthreads();
      for (int e = tid; e < K3; e += blockDim.x) {
        int i = e / K2, j = (e / K) % K, m = e % K;
        S[(i * K + j) * ZP + m] = in[(size_t)item.src * K3 + e];
      }
      loaded = item.src;
    }
    __syncthreads();
    const MRA_GLOBAL double* TX = dT + (size_t)item.tx * K2;
    const MRA_GLOBAL double* TY = dT + (size_t)item.ty * K2;
    const MRA_GLOBAL double* TZ = dT + (size_t)item.tz * K2;
    const double cmu = dc[item.mu] * scale;
    if (tid < K2) {
      int Y = tid / K, Z = tid % K;
      double t[K];
#pragma unroll
      for (int a = 0; a < K; ++a) t[a] = 0.0;
      for (int i = 0; i < K; ++i) {
        double v = S[(i * K + Y) * ZP + Z];
#pragma unroll
        for (int a = 0; a < K; ++a) t[a] += TX[i * K + a] * v;
      }
#pragma unroll
      for (int a = 0; a < K; ++a) W[(a * K + Y) * ZP + Z] = t[a];
    }
    __syncthreads();
    if (tid < K2) {
      int a = tid / K, Z = tid % K;
      double t[K];
#pragma unroll
      for (int b = 0; b < K; ++b) t[b] = 0.0;
      for (int j = 0; j < K; ++j) {
        double v = W[(a * K + j) * ZP + Z];
#pragma unroll
        for (int b = 0; b < K; ++b) t[b] += TY[j * K + b] * v;
      }
#pragma unroll
      for (int b = 0; b < K; ++b) W[(a * K + b) * ZP + Z] = t[b];
    }
    __syncthreads();
    if (tid < K2) {
      int a = tid / K, b = tid % K;
      double t[K];
#pragma unroll
      for (int c = 0; c < K; ++c) t[c] = 0.0;
      for (int m = 0; m < K; ++m) {
        double v = W[(a * K + b) * ZP + m];
#pragma unroll
        for (int c = 0; c < K; ++c) t[c] += TZ[m * K + c] * v;
      }
#pragma unroll
      for (int c = 0; c < K; ++c) acc[c] += cmu * t[c];
    }
    __syncthreads();
  }
  if (tid < K2) {
    int a = tid / K, b = tid % K;
#pragma unroll
    for (int c = 0; c < K; ++c) out[(size_t)tr.node * K3 + (a * K + b) * K + c] += acc[c];
  }
}

// ------------------------------------------------------------------ apply (std, MFMA)
// Standard form for k = 8 (two quads per index) on the FP64 matrix cores: one wave per
// target, four targets per workgroup.  The three mode products of a triple are the chain of
// apply_ns_stream_kernel on a k^3 block: step 1 contracts x (block index = z inside a z-quad,
// source fragments read straight from the input slab), step 2 contracts y in registers, and
// step 3 contracts z after an in-wave permutation (ds_bpermute) into the target's block,
// which stays in registers (8 doubles per lane) over all triples of the target.  The next
// triple's source and operator fragments are loaded while the current one computes, and
// several waves per SIMD hide what remains of the load latency.  With TL the launch's t
// blocks (one function's table of t_lds doubles, every target of that function) are first
// staged in LDS, and the operator fragments are read from there: a triple then issues only
// its eight source loads to the vector memory pipeline.
template <int K, bool TL>
__global__ __launch_bounds__(256, 4) void apply_std_mfma_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets, const int ntargets,
    const double* const* __restrict__ t_tab, const double* const* __restrict__ c_tab,
    double scale, const int t_lds) {
  constexpr int K2 = K * K, K3 = K * K * K, Q = K / 4;
  static_assert(K % 4 == 0 && Q == 2, "k = 8: two quads per index");
  extern __shared__ double Ts[];      // TL: the t table (t_lds doubles)
  if constexpr (TL) {
    const MRA_GLOBAL double* __restrict__ t0 = as_global(t_tab[0]);
    for (int e = threadIdx.x; e < t_lds; e += 256) Ts[e] = t0[e];
    __syncthreads();                  // before any wave can leave
  }
  const int lane = threadIdx.x & 63;
  // Workgroups go to the eight dies (XCDs) in turn; renumber them so that each die takes a
  // contiguous eighth of the targets, which come in Morton order: its L2 then serves one
  // spatial octant of source blocks and their neighbours instead of the whole level.
  const int nwg = gridDim.x, wg = blockIdx.x, per = nwg >> 3, rem = nwg & 7, xcd = wg & 7;
  const int lwg = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + (wg >> 3);
  // uniform per wave: the range and the items are read with scalar loads
  const int ti = __builtin_amdgcn_readfirstlane(lwg * 4 + (threadIdx.x >> 6));
  if (ti >= ntargets) return;                 // a whole wave leaves; no barriers below
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  const int swap = (16 * lb + 4 * lk + li) * 4;
  const TargetRange tr = targets[ti];
  const MRA_GLOBAL double* __restrict__ in = as_global(in_tab[tr.fn]);
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dT = as_global(t_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dc = as_global(c_tab[tr.fn]);
  auto lane_swap = [&](double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(swap, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(swap, w.y);
    return __builtin_bit_cast(double, r);
  };
  // fragments of one triple: source s[x][y][z] as A operands of step 1 ([xs][yt][zq]),
  // transposed t blocks as B operands ([quad of the contracted index][quad of the output])
  struct Frag {
    double s[Q][Q][Q], tx[Q][Q], ty[Q][Q], tz[Q][Q];
    double c;
  };
  auto load = [&](const NSItem& it, Frag& f) {
    const MRA_GLOBAL double* sp = in + (size_t)it.src * K3;
#pragma unroll
    for (int xs = 0; xs < Q; ++xs)
#pragma unroll
      for (int yt = 0; yt < Q; ++yt)
#pragma unroll
        for (int zq = 0; zq < Q; ++zq)
          f.s[xs][yt][zq] = sp[((4 * xs + lk) * K + 4 * yt + li) * K + 4 * zq + lb];
    if constexpr (TL) {
      const int ox = it.tx * K2 + lk * K + li, oy = it.ty * K2 + lk * K + li, oz = it.tz * K2 + lk * K + li;
#pragma unroll
      for (int u = 0; u < Q; ++u)
#pragma unroll
        for (int v = 0; v < Q; ++v) {
          f.tx[u][v] = Ts[ox + 4 * u * K + 4 * v];
          f.ty[u][v] = Ts[oy + 4 * u * K + 4 * v];
          f.tz[u][v] = Ts[oz + 4 * u * K + 4 * v];
        }
    } else {
      const MRA_GLOBAL double* TX = dT + (size_t)it.tx * K2;
      const MRA_GLOBAL double* TY = dT + (size_t)it.ty * K2;
      const MRA_GLOBAL double* TZ = dT + (size_t)it.tz * K2;
#pragma unroll
      for (int u = 0; u < Q; ++u)
#pragma unroll
        for (int v = 0; v < Q; ++v) {
          f.tx[u][v] = TX[(4 * u + lk) * K + 4 * v + li];
          f.ty[u][v] = TY[(4 * u + lk) * K + 4 * v + li];
          f.tz[u][v] = TZ[(4 * u + lk) * K + 4 * v + li];
        }
    }
    f.c = dc[it.mu] * scale;
  };
  double acc[Q][Q][Q];
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
      for (int c = 0; c < Q; ++c) acc[a][b][c] = 0.0;
  Frag cur, nxt;
  if (tr.beg < tr.end) load(items[tr.beg], cur);
  for (int it = tr.beg; it < tr.end; ++it) {
    if (it + 1 < tr.end) load(items[it + 1], nxt);
    // step 1: d1[zq][at][yt] (rows y, columns a, block index z)
    double d1[Q][Q][Q];
#pragma unroll
    for (int zq = 0; zq < Q; ++zq)
#pragma unroll
      for (int at = 0; at < Q; ++at)
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) {
          double d = 0.0;
#pragma unroll
          for (int xs = 0; xs < Q; ++xs)
            d = __builtin_amdgcn_mfma_f64_4x4x4f64(cur.s[xs][yt][zq], cur.tx[xs][at], d, 0, 0, 0);
          d1[zq][at][yt] = d;
        }
    // step 2: zr[zq][at][bt]
    double zr[Q][Q][Q];
#pragma unroll
    for (int zq = 0; zq < Q; ++zq)
#pragma unroll
      for (int at = 0; at < Q; ++at)
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) {
          double d = 0.0;
#pragma unroll
          for (int ys = 0; ys < Q; ++ys)
            d = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[zq][at][ys], cur.ty[ys][bt], d, 0, 0, 0);
          zr[zq][at][bt] = d;
        }
    // step 3: acc[at][bt][ct] += sum over z-quads of c (permuted zr) t_z
#pragma unroll
    for (int at = 0; at < Q; ++at)
#pragma unroll
      for (int bt = 0; bt < Q; ++bt)
#pragma unroll
        for (int zq = 0; zq < Q; ++zq) {
          const double zt = lane_swap(zr[zq][at][bt]);
#pragma unroll
          for (int ct = 0; ct < Q; ++ct)
            acc[at][bt][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(zt, cur.c * cur.tz[zq][ct],
                                                                 acc[at][bt][ct], 0, 0, 0);
        }
    cur = nxt;
  }
#pragma unroll
  for (int at = 0; at < Q; ++at)
#pragma unroll
    for (int bt = 0; bt < Q; ++bt)
#pragma unroll
      for (int ct = 0; ct < Q; ++ct) {
        const int a = 4 * at + lb, b = 4 * bt + lk, c = 4 * ct + li;
        out[(size_t)tr.node * K3 + (a * K + b) * K + c] += acc[at][bt][ct];
      }
}

// --------------------------------------------------------------------------- sum-down
// One workgroup of 512 threads per interior output box: three mode products with the
// unfilter matrix [h0 | h1]^T.  The first (over z) goes through LDS, one thread per (i, j)
// row; the last two are fused per output column (Y, Z): the thread forms the column's k
// values of the middle product from the first product's rows and contracts them at once,
// half of the x range at a time, with the unfilter rows (the same for every lane) read by
// scalar loads.  Only the first product's result is held in LDS (at k = 14 about 70 KB, so
// that two boxes share a CU and one's loads overlap the other's products).  The
// contraction over the first product's rows stays rolled.
template <int K>
__global__ __launch_bounds__(512, 4) void sum_down_kernel(
    double* const* __restrict__ tab, const NodeRef* __restrict__ refs,
    const double* __restrict__ subbuf, const double* __restrict__ h0,
    const double* __restrict__ h1, const double sign) {
  constexpr int N = 2 * K, K3 = K * K * K, ZP = N + 1;
  __shared__ double T1[K * K * ZP];   // [i][j][Z] = sum_m H[m][Z] V[i][j][m]
  __shared__ double Vs[K3];           // the box's coefficients plus its level-n part
  __shared__ double H[K * N];         // H[m][X] = [h0 | h1][m][X]
  const int tid = threadIdx.x;
  const NodeRef ref = refs[blockIdx.x];
  const int node = ref.node, fc = ref.fchild;
  MRA_GLOBAL double* __restrict__ coeff = as_global(tab[ref.fn]);
  for (int e = tid; e < K * N; e += 512) {
    int i = e / N, X = e % N;
    H[e] = X < K ? h0[i * K + X] : h1[i * K + X - K];
  }
  const MRA_GLOBAL double* __restrict__ V = coeff + (size_t)node * K3;
  const double* __restrict__ VS = ref.sub >= 0 ? subbuf + (size_t)ref.sub * K3 : nullptr;
  for (int e = tid; e < K3; e += 512) Vs[e] = VS ? V[e] + VS[e] : V[e];
  __syncthreads();
  typedef const __attribute__((address_space(4))) double* CPtr;
  const CPtr hc0 = (CPtr)h0, hc1 = (CPtr)h1;
  for (int col = tid; col < K * K; col += 512) {
    const int i = col / K, j = col % K;
    double t[N];
#pragma unroll
    for (int Z = 0; Z < N; ++Z) t[Z] = 0.0;
#pragma unroll 1
    for (int m = 0; m < K; ++m) {
      const double v = Vs[(i * K + j) * K + m];
#pragma unroll
      for (int Z = 0; Z < N; ++Z) t[Z] += (Z < K ? hc0[m * K + Z] : hc1[m * K + Z - K]) * v;
    }
#pragma unroll
    for (int Z = 0; Z < N; ++Z) T1[(i * K + j) * ZP + Z] = t[Z];
  }
  __syncthreads();
  for (int col = tid; col < N * N; col += 512) {  // child[X][Y][Z] += sum_i H[i][X] T2[i][Y][Z]
    const int Y = col / N, Z = col % N;
    const int cy = Y / K, jy = Y % K, cz = Z / K, m = Z % K;
    double t2[K];   // T2[i][Y][Z] = sum_j H[j][Y] T1[i][j][Z]
#pragma unroll
    for (int i = 0; i < K; ++i) t2[i] = 0.0;
#pragma unroll 1
    for (int j = 0; j < K; ++j) {
      const double hy = H[j * N + Y];
#pragma unroll
      for (int i = 0; i < K; ++i) t2[i] += hy * T1[(i * K + j) * ZP + Z];
    }
#pragma unroll
    for (int cx = 0; cx < 2; ++cx) {
      const CPtr hx = cx ? hc1 : hc0;   // H[i][cx k + x] = hx[i k + x]
      double t[K];
#pragma unroll
      for (int x = 0; x < K; ++x) t[x] = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int x = 0; x < K; ++x) t[x] += hx[i * K + x] * t2[i];
      MRA_GLOBAL double* __restrict__ dst =
          coeff + (size_t)(fc + (cx << 2 | cy << 1 | cz)) * K3 + jy * K + m;
      double old[K];
#pragma unroll
      for (int x = 0; x < K; ++x) old[x] = dst[x * K * K];
#pragma unroll
      for (int x = 0; x < K; ++x) dst[x * K * K] = old[x] + sign * t[x];
    }
  }
}

// ----------------------------------------------------------------- wavelet-form helpers
// Squared Frobenius norm of the 8 contiguous child slabs (the (2k)^3 children block) of
// each listed box; one workgroup per box, fixed-order tree, so the result is reproducible.
__global__ __launch_bounds__(256) void child_norm2_kernel(
    int k3, const double* __restrict__ coeff, const int32_t* __restrict__ fchild,
    double* __restrict__ out) {
  __shared__ double red[256];
  const double* __restrict__ p = coeff + (size_t)fchild[blockIdx.x] * k3;
  double s = 0.0;
  for (int e = threadIdx.x; e < 8 * k3; e += 256) s += p[e] * p[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// dst slab to[i] (i if to is null) = src slab from[i]; one workgroup per slab.
__global__ __launch_bounds__(256) void copy_slabs_kernel(
    int k3, double* __restrict__ dst, const int32_t* __restrict__ to,
    const double* __restrict__ src, const int32_t* __restrict__ from) {
  const double* __restrict__ a = src + (size_t)from[blockIdx.x] * k3;
  double* __restrict__ b = dst + (size_t)(to ? to[blockIdx.x] : (int32_t)blockIdx.x) * k3;
  for (int e = threadIdx.x; e < k3; e += 256) b[e] = a[e];
}

// --------------------------------------------------------------- adaptive projection
// Projection of f = sum_g c_g exp(-a_g |x - X_g|^2) (Sec. 2.1), one level of the adaptive
// refinement per pair of launches.
//
// gauss1d_kernel: one thread per (1D box, Gaussian) row.  The level's distinct 1D box
// indices l of the three axes are concatenated (x, then y, then z); row (u, g) holds
//   [0, K)     int exp(-a (x - X)^2) phi^n_{l,i}(x) dx          (the box itself, level n)
//   [K, 3K)    the same on the two children 2l, 2l+1 (level n + 1), concatenated
//   [3K, 5K)   H^T H applied to those 2K values (their part in the parent's space)
// where H = [h0 | h1] is the two-scale filter.  The integrals are composite Gauss-Legendre
// rules (nq nodes per panel, panels no wider than min(1, beta^{-1/2}) in the box's unit
// coordinate, beta = a h^2) over the intersection of the box with the Gaussian's numerical
// support |u - u0| <= sqrt((50 + log(1 + beta)/2) / beta).  nz[row] is 1 iff any of the
// 3K integrals is nonzero.
template <int K>
__device__ __forceinline__ void scaled_legendre(double u, double* ph) {
  if (u < 0.0 || u > 1.0) {
#pragma unroll
    for (int i = 0; i < K; ++i) ph[i] = 0.0;
    return;
  }
  const double t = 2.0 * u - 1.0;
  double pm = 1.0, p = t;
  ph[0] = 1.0;
  if (K > 1) ph[1] = sqrt(3.0) * t;
#pragma unroll
  for (int i = 1; i + 1 < K; ++i) {
    const double pn = ((2.0 * i + 1.0) * t * p - i * pm) / (i + 1.0);
    pm = p;
    p = pn;
    ph[i + 1] = sqrt(2.0 * (i + 1) + 1.0) * pn;
  }
}

template <int K>
__device__ void gaussian_box_integrals(double a, double X, double lo, double h, int64_t l,
                                       const double* __restrict__ glx,
                                       const double* __restrict__ glw, int nq, double* out) {
#pragma unroll
  for (int i = 0; i < K; ++i) out[i] = 0.0;
  const double beta = a * h * h;
  const double u0 = (X - lo) / h - (double)l;
  const double half = beta > 0.0 ? sqrt((50.0 + 0.5 * log1p(beta)) / beta) : INFINITY;
  const double ua = fmax(0.0, u0 - half), ub = fmin(1.0, u0 + half);
  if (ub <= ua) return;
  const double width = beta > 0.0 ? fmin(1.0, 1.0 / sqrt(beta)) : 1.0;
  const int npan = max(1, (int)ceil((ub - ua) / width));
  const double step = (ub - ua) / npan;
  double ph[K];
  for (int pn = 0; pn < npan; ++pn) {
    const double ea = ua + pn * step, eb = (pn + 1 == npan) ? ub : ua + (pn + 1) * step;
    for (int q = 0; q < nq; ++q) {
      const double u = ea + (eb - ea) * glx[q];
      const double wt = (eb - ea) * glw[q] * exp(-beta * (u - u0) * (u - u0));
      scaled_legendre<K>(u, ph);
#pragma unroll
      for (int i = 0; i < K; ++i) out[i] += wt * ph[i];
    }
  }
  const double sh = sqrt(h);
#pragma unroll
  for (int i = 0; i < K; ++i) out[i] *= sh;
}

template <int K>
__global__ __launch_bounds__(64) void gauss1d_kernel(
    const double* __restrict__ gpar, int ng, const int64_t* __restrict__ lvals, int nl,
    int off1, int off2, int n, double lo, double W, const double* __restrict__ glx,
    const double* __restrict__ glw, int nq, const double* __restrict__ h0,
    const double* __restrict__ h1, double* __restrict__ T, uint8_t* __restrict__ nz) {
  constexpr int RW = 5 * K;
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (r >= (int64_t)nl * ng) return;
  const int u = (int)(r / ng), g = (int)(r % ng);
  const int ax = (u >= off1) + (u >= off2);
  const double a = gpar[5 * g], X = gpar[5 * g + 1 + ax];
  const int64_t l = lvals[u];
  const double h = W / ldexp(1.0, n), hc = W / ldexp(1.0, n + 1);
  double own[K], c0[K], c1[K];
  gaussian_box_integrals<K>(a, X, lo, h, l, glx, glw, nq, own);
  gaussian_box_integrals<K>(a, X, lo, hc, 2 * l, glx, glw, nq, c0);
  gaussian_box_integrals<K>(a, X, lo, hc, 2 * l + 1, glx, glw, nq, c1);
  double sp[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int x = 0; x < K; ++x) acc += h0[i * K + x] * c0[x];
#pragma unroll
    for (int x = 0; x < K; ++x) acc += h1[i * K + x] * c1[x];
    sp[i] = acc;
  }
  double* __restrict__ row = T + r * RW;
  bool any = false;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    row[i] = own[i];
    row[K + i] = c0[i];
    row[2 * K + i] = c1[i];
    any = any || own[i] != 0.0 || c0[i] != 0.0 || c1[i] != 0.0;
  }
#pragma unroll
  for (int x = 0; x < K; ++x) {
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      p0 += h0[i * K + x] * sp[i];
      p1 += h1[i * K + x] * sp[i];
    }
    row[3 * K + x] = p0;
    row[4 * K + x] = p1;
  }
  nz[r] = any ? 1 : 0;
}

// project_level_kernel: one workgroup per box of the level's frontier, boxu[3 b + ax] = the
// box's row index u on axis ax.  The Gaussians whose three rows are nonzero are listed (in
// ascending order) and staged in LDS GC at a time.  Thread (i, j) < K^2 accumulates the
// box's own coefficients s[i][j][m] = sum_g c_g x_i y_j z_m (into S, slab b); with test set,
// thread (X, Y) < (2K)^2 accumulates the wavelet part of the children block column
//   d[X][Y][Z] = sum_g c_g (xc_X yc_Y zc_Z - xp_X yp_Y zp_Z)
// (B minus its part in the parent's space; rank one per Gaussian, so the filter acts on
// the 1D rows), and d2[b] = ||d||_F^2 by a fixed-order tree.
template <int K>
__global__ __launch_bounds__(1024) void project_level_kernel(
    const double* __restrict__ T, const uint8_t* __restrict__ nz,
    const int32_t* __restrict__ boxu, int ng, const double* __restrict__ gpar, int test,
    double* __restrict__ d2, double* __restrict__ S) {
  constexpr int N = 2 * K, RW = 5 * K, GC = 16, K3 = K * K * K;
  __shared__ double rows[GC][3][RW];
  __shared__ double cg[GC];
  __shared__ double red[1024];
  __shared__ int nact_s;
  extern __shared__ int act[];   // ng entries
  const int tid = threadIdx.x, nt = blockDim.x;
  const int bu0 = boxu[3 * blockIdx.x], bu1 = boxu[3 * blockIdx.x + 1],
            bu2 = boxu[3 * blockIdx.x + 2];
  if (tid < 64) {   // wave 0 lists the active Gaussians in ascending order
    int cnt = 0;
    for (int base = 0; base < ng; base += 64) {
      const int g = base + tid;
      const bool f = g < ng && nz[(size_t)bu0 * ng + g] && nz[(size_t)bu1 * ng + g] &&
                     nz[(size_t)bu2 * ng + g];
      const unsigned long long m = __ballot(f);
      if (f) act[cnt + __popcll(m & ((1ULL << tid) - 1ULL))] = g;
      cnt += __popcll(m);
    }
    if (tid == 0) nact_s = cnt;
  }
  __syncthreads();
  const int nact = nact_s;
  double d[N], s[K];
#pragma unroll
  for (int z = 0; z < N; ++z) d[z] = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) s[m] = 0.0;
  const int X = tid / N, Y = tid % N, i = tid / K, j = tid % K;
  for (int c0 = 0; c0 < nact; c0 += GC) {
    const int cnt = min(GC, nact - c0);
    __syncthreads();
    for (int e = tid; e < cnt * 3 * RW; e += nt) {
      const int gi = e / (3 * RW), rem = e % (3 * RW), ax = rem / RW, w = rem % RW;
      const int bu = ax == 0 ? bu0 : (ax == 1 ? bu1 : bu2);
      rows[gi][ax][w] = T[((size_t)bu * ng + act[c0 + gi]) * RW + w];
    }
    if (tid < cnt) cg[tid] = gpar[5 * act[c0 + tid] + 4];
    __syncthreads();
    if (test && tid < N * N) {
      for (int gi = 0; gi < cnt; ++gi) {
        const double a = cg[gi] * rows[gi][0][K + X] * rows[gi][1][K + Y];
        const double b = cg[gi] * rows[gi][0][3 * K + X] * rows[gi][1][3 * K + Y];
#pragma unroll
        for (int z = 0; z < N; ++z) d[z] += a * rows[gi][2][K + z] - b * rows[gi][2][3 * K + z];
      }
    }
    if (tid < K * K) {
      for (int gi = 0; gi < cnt; ++gi) {
        const double cij = cg[gi] * rows[gi][0][i] * rows[gi][1][j];
#pragma unroll
        for (int m = 0; m < K; ++m) s[m] += cij * rows[gi][2][m];
      }
    }
  }
  if (tid < K * K) {
    double* __restrict__ o = S + (size_t)blockIdx.x * K3 + (size_t)(i * K + j) * K;
#pragma unroll
    for (int m = 0; m < K; ++m) o[m] = s[m];
  }
  if (test) {
    double sq = 0.0;
    if (tid < N * N) {
#pragma unroll
      for (int z = 0; z < N; ++z) sq += d[z] * d[z];
    }
    red[tid] = sq;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
      if (tid < st && tid + st < nt) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) d2[blockIdx.x] = red[0];
  }
}

// --------------------------------------------------------------------------- reductions
// mode 0: sum ||a_leaf||^2; mode 1: sum a_leaf[0] * weight[leaf]; mode 2: sum <a_la, b_lb>;
// mode 3: sum ||a_la - b_lb||^2.
// Workgroup g takes leaves g, g + G, g + 2G, ... (G = gridDim.x) in that order, its threads
// the elements e = t, t + 256, ... of each leaf, and the partials are combined in a fixed
// tree: the result does not depend on scheduling.  The next leaf's index is loaded before
// the current leaf's elements so that consecutive leaves overlap their latencies.
__global__ __launch_bounds__(256) void leaf_reduce_kernel(
    int k3, const double* __restrict__ a, const double* __restrict__ b,
    const int32_t* __restrict__ la, const int32_t* __restrict__ lb,
    const double* __restrict__ weight, int count, int mode, double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  int l = blockIdx.x;
  const bool paired = mode >= 2;
  int ia = l < count ? la[l] : 0, ib = (paired && l < count) ? lb[l] : 0;
  for (; l < count; l += gridDim.x) {
    const int ln = l + gridDim.x;
    const int na = ln < count ? la[ln] : 0, nb = (paired && ln < count) ? lb[ln] : 0;
    const double* pa = a + (size_t)ia * k3;
    if (mode == 0) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q;
        v[q] = e < k3 ? pa[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) s += v[q] * v[q];
      for (int e = threadIdx.x + 1024; e < k3; e += 256) s += pa[e] * pa[e];
    } else if (mode == 1) {
      if (threadIdx.x == 0) s += pa[0] * weight[l];
    } else if (mode == 3) {
      const double* pb = b + (size_t)ib * k3;
      for (int e = threadIdx.x; e < k3; e += 256) {
        const double d = pa[e] - pb[e];
        s += d * d;
      }
    } else {
      const double* pb = b + (size_t)ib * k3;
      double v[4], w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q;
        v[q] = e < k3 ? pa[e] : 0.0;
        w[q] = e < k3 ? pb[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) s += v[q] * w[q];
      for (int e = threadIdx.x + 1024; e < k3; e += 256) s += pa[e] * pb[e];
    }
    ia = na;
    ib = nb;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------- apply (NS, MFMA, a-quad ownership per wave)
// FP64 matrix-core kernel for even k in [8, 12] (2k = 4Q).  Same 4x4x4 (four blocks)
// product chain as apply_ns_mfma_kernel: step 1 contracts x (block index = z inside a
// z-quad), step 2 contracts y in registers.  The work of a triple is split into (a-quad,
// z-quad) units handed to the four waves in contiguous a-major runs, so a wave owns at most
// two a-quads and finishes the z-contraction (step 3) of its units itself: the step-2 result
// (block = z, row = a) is turned into the step-3 A operand (block = a, k = z) by an in-wave
// lane permutation (ds_bpermute, no LDS storage) and accumulated per z-quad.  There is no
// exchange tensor, so a triple needs one workgroup barrier (for the double-buffered operator
// blocks) and the source block stays resident in LDS for all triples of a source.  a-quads
// shared by two neighbouring waves are summed through LDS once at the end, and the children
// block is written out coalesced.
template <int K>
__global__ __launch_bounds__(256) void apply_ns_own_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const double* const* __restrict__ r_tab, const double* const* __restrict__ t_tab,
    const double* const* __restrict__ c_tab, double* __restrict__ partials,
    double* __restrict__ subbuf) {
  constexpr int N = 2 * K, Q = N / 4, N2 = N * N, N3 = N * N * N, K2 = K * K, K3 = K * K * K;
  static_assert(N % 4 == 0 && Q >= 4 && Q <= 6, "even k in [8, 12]");
  constexpr int NU = Q * Q;                              // (a-quad, z-quad) units
  constexpr int Q2 = (K + 3) / 4, KP = 4 * Q2, SU = Q2 * Q2;
  constexpr int OPS = 3 * N2 + 3 * K2, OPS_PER_LANE = (OPS + 255) / 256;
  __shared__ double Xs[N3];          // children block B_P, quad-blocked; at the end: sums
  __shared__ double Ss[KP * KP * KP]; // s_P zero-padded to KP^3, quad-blocked; at the end: sums
  __shared__ double Os[2][OPS];     // R_x^T, R_y^T, R_z^T, t_x^T, t_y^T, t_z^T
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  const int swap = (16 * lb + 4 * lk + li) * 4;          // lane with kk and bb exchanged
  const TargetRange tr = targets[blockIdx.x];
  const MRA_GLOBAL double* __restrict__ in = as_global(in_tab[tr.fn]);
  MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dR = as_global(r_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dT = as_global(t_tab[tr.fn]);
  const MRA_GLOBAL double* __restrict__ dc = as_global(c_tab[tr.fn]);
  const bool with_sub = tr.sub >= 0;
  const int u0 = wave * NU / 4, u1 = (wave + 1) * NU / 4, at0 = u0 / Q;
  const int v0 = wave * SU / 4, v1 = (wave + 1) * SU / 4, sat0 = v0 / Q2;

  auto fetch_ops = [&](const NSItem nx, double* reg) {
#pragma unroll
    for (int q = 0; q < OPS_PER_LANE; ++q) {
      const int e = tid + 256 * q;
      double v = 0.0;
      if (e < 3 * N2) {
        const int w = e / N2, r = e - w * N2;
        const int blk = w == 0 ? nx.rx : (w == 1 ? nx.ry : nx.rz);
        v = dR[(size_t)blk * N2 + r];
      } else if (e < OPS) {
        const int e2 = e - 3 * N2, w = e2 / K2, r = e2 - w * K2;
        const int blk = w == 0 ? nx.tx : (w == 1 ? nx.ty : nx.tz);
        v = dT[(size_t)blk * K2 + r];
      }
      reg[q] = v;
    }
  };
  auto store_ops = [&](const double* reg, double* dst) {
#pragma unroll
    for (int q = 0; q < OPS_PER_LANE; ++q) {
      const int e = tid + 256 * q;
      if (e < OPS) dst[e] = reg[q];
    }
  };
  auto lane_swap = [&](double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(swap, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(swap, w.y);
    return __builtin_bit_cast(double, r);
  };

  double acc[2][Q][Q];    // [a-quad at0 + slot][b-quad][c-quad]
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
      for (int c = 0; c < Q; ++c) acc[s2][b][c] = 0.0;
  double sacc[2][Q2][Q2];
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
    for (int b = 0; b < Q2; ++b)
#pragma unroll
      for (int c = 0; c < Q2; ++c) sacc[s2][b][c] = 0.0;

  NSItem cur{}, nxt{};   // item records of this and the next triple, loaded ahead
  double pre[OPS_PER_LANE], c_cur = 0.0, c_pre = 0.0;   // c_mu travels with the operators
  if (tr.beg < tr.end) {
    cur = items[tr.beg];
    fetch_ops(cur, pre);
    c_cur = dc[cur.mu];
    store_ops(pre, Os[tr.beg & 1]);
    if (tr.beg + 1 < tr.end) nxt = items[tr.beg + 1];
  }
  int loaded = -1;
  for (int it = tr.beg; it < tr.end; ++it) {
    const NSItem item = cur;
    const bool more = it + 1 < tr.end;
    if (item.src_fc != loaded) {
      __syncthreads();   // every wave is done with the previous source block
      stage_children_qb<K, Q, 18>(Xs, in + (size_t)item.src_fc * K3, tid);
      if (with_sub) stage_scaling_qb<K, Q2, 8>(Ss, in + (size_t)item.src * K3, tid);
      loaded = item.src_fc;
    }
    __syncthreads();     // source block and this triple's operators are in place
    if (more) {
      fetch_ops(nxt, pre);
      c_pre = dc[nxt.mu];
    }
    cur = nxt;
    if (it + 2 < tr.end) nxt = items[it + 2];
    const double* Ob = Os[it & 1];
    const double* RXs = Ob;
    const double* RYs = Ob + N2;
    const double* RZs = Ob + 2 * N2;
    const double* TXs = Ob + 3 * N2;
    const double* TYs = Ob + 3 * N2 + K2;
    const double* TZs = Ob + 3 * N2 + 2 * K2;
    const double cmu = c_cur;
    {
      double ry[Q][Q];
#pragma unroll
      for (int ys = 0; ys < Q; ++ys)
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) ry[ys][bt] = RYs[(4 * ys + lk) * N + 4 * bt + li];
      // both a-quads of the wave share the step-1 reads of the source block where their
      // z-quad ranges overlap
      const int zl0 = max(0, u0 - at0 * Q), zh0 = min(Q, u1 - at0 * Q);
      const int zl1 = max(0, u0 - (at0 + 1) * Q), zh1 = min(Q, u1 - (at0 + 1) * Q);
      double rx[2][Q];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int xs = 0; xs < Q; ++xs)
          rx[s2][xs] = (at0 + s2 < Q) ? RXs[(4 * xs + lk) * N + 4 * (at0 + s2) + li] : 0.0;
      // steps 2 and 3 of one a-quad slot from its step-1 result
      auto finish = [&](double (&d1)[Q], double (&ac)[Q][Q], int zq) {
        double zr[Q];
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) zr[bt] = 0.0;
#pragma unroll
        for (int ys = 0; ys < Q; ++ys)
#pragma unroll
          for (int bt = 0; bt < Q; ++bt)
            zr[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[ys], ry[ys][bt], zr[bt], 0, 0, 0);
        double rz[Q];
#pragma unroll
        for (int ct = 0; ct < Q; ++ct) rz[ct] = cmu * RZs[(4 * zq + lk) * N + 4 * ct + li];
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) {
          const double zt = lane_swap(zr[bt]);
#pragma unroll
          for (int ct = 0; ct < Q; ++ct)
            ac[bt][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(zt, rz[ct], ac[bt][ct], 0, 0, 0);
        }
      };
      const int zfirst = min(zl0 < zh0 ? zl0 : Q, zl1 < zh1 ? zl1 : Q);
      const int zlast = max(zh0, zh1);
#pragma unroll 1
      for (int zq = zfirst; zq < zlast; ++zq) {
        const bool on0 = zq >= zl0 && zq < zh0, on1 = zq >= zl1 && zq < zh1;
        if (!on0 && !on1) continue;
        if (on0 && on1) {
          double d1a[Q], d1b[Q];
#pragma unroll
          for (int yt = 0; yt < Q; ++yt) d1a[yt] = d1b[yt] = 0.0;
#pragma unroll
          for (int xs = 0; xs < Q; ++xs)
#pragma unroll
            for (int yt = 0; yt < Q; ++yt) {
              const double xv = Xs[qb_off<Q>(4 * xs + lk, 4 * yt + li, 4 * zq + lb)];
              d1a[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(xv, rx[0][xs], d1a[yt], 0, 0, 0);
              d1b[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(xv, rx[1][xs], d1b[yt], 0, 0, 0);
            }
          finish(d1a, acc[0], zq);
          finish(d1b, acc[1], zq);
        } else {
          // one slot: select its operator column without dynamic register indexing
          double rxs[Q];
#pragma unroll
          for (int xs = 0; xs < Q; ++xs) rxs[xs] = on0 ? rx[0][xs] : rx[1][xs];
          double d1[Q];
#pragma unroll
          for (int yt = 0; yt < Q; ++yt) d1[yt] = 0.0;
#pragma unroll
          for (int xs = 0; xs < Q; ++xs)
#pragma unroll
            for (int yt = 0; yt < Q; ++yt)
              d1[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                  Xs[qb_off<Q>(4 * xs + lk, 4 * yt + li, 4 * zq + lb)], rxs[xs], d1[yt],
                  0, 0, 0);
          if (on0)
            finish(d1, acc[0], zq);
          else
            finish(d1, acc[1], zq);
        }
      }
    }
    // ---- level-n subtraction -c (t_x x t_y x t_z) s_P, same scheme on the KP^3 grid
    if (with_sub) {
      double ty[Q2][Q2];
#pragma unroll
      for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
        for (int bt = 0; bt < Q2; ++bt) {
          const int r = 4 * ys + lk, cc = 4 * bt + li;
          ty[ys][bt] = (r < K && cc < K) ? TYs[r * K + cc] : 0.0;
        }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int at = sat0 + s2;
        const int z_lo = max(0, v0 - at * Q2), z_hi = min(Q2, v1 - at * Q2);
        if (z_lo < z_hi) {
          double tx[Q2];
#pragma unroll
          for (int xs = 0; xs < Q2; ++xs) {
            const int r = 4 * xs + lk, cc = 4 * at + li;
            tx[xs] = (r < K && cc < K) ? TXs[r * K + cc] : 0.0;
          }
#pragma unroll 1
          for (int zq = z_lo; zq < z_hi; ++zq) {
            double d1[Q2];
#pragma unroll
            for (int yt = 0; yt < Q2; ++yt) d1[yt] = 0.0;
#pragma unroll
            for (int xs = 0; xs < Q2; ++xs)
#pragma unroll
              for (int yt = 0; yt < Q2; ++yt)
                d1[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                    Ss[qb_off<Q2>(4 * xs + lk, 4 * yt + li, 4 * zq + lb)], tx[xs], d1[yt],
                    0, 0, 0);
            double zr[Q2];
#pragma unroll
            for (int bt = 0; bt < Q2; ++bt) zr[bt] = 0.0;
#pragma unroll
            for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
              for (int bt = 0; bt < Q2; ++bt)
                zr[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[ys], ty[ys][bt], zr[bt], 0, 0, 0);
            double tz[Q2];
#pragma unroll
            for (int ct = 0; ct < Q2; ++ct) {
              const int r = 4 * zq + lk, cc = 4 * ct + li;
              tz[ct] = (r < K && cc < K) ? -cmu * TZs[r * K + cc] : 0.0;
            }
#pragma unroll
            for (int bt = 0; bt < Q2; ++bt) {
              const double zt = lane_swap(zr[bt]);
#pragma unroll
              for (int ct = 0; ct < Q2; ++ct)
                sacc[s2][bt][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(zt, tz[ct], sacc[s2][bt][ct], 0, 0, 0);
            }
          }
        }
      }
    }
    if (more) {
      store_ops(pre, Os[(it + 1) & 1]);
      c_cur = c_pre;
    }
  }
  // ---- sum the waves' partial blocks in LDS (even waves, then odd waves: the a-quads of
  // waves two apart are disjoint), then write the target's blocks coalesced
  __syncthreads();
  double* Bsum = Xs;    // [a][b][c], N^3
  double* Ssum = Ss;    // [a][b][c], K^3
  for (int e = tid; e < N3; e += 256) Bsum[e] = 0.0;
  if (with_sub)
    for (int e = tid; e < K3; e += 256) Ssum[e] = 0.0;
  __syncthreads();
  for (int par = 0; par < 2; ++par) {
    if ((wave & 1) == par) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int at = at0 + s2;
        if (max(0, u0 - at * Q) < min(Q, u1 - at * Q)) {
          const int a = 4 * at + lb;
#pragma unroll
          for (int bt = 0; bt < Q; ++bt)
#pragma unroll
            for (int ct = 0; ct < Q; ++ct)
              Bsum[(a * N + 4 * bt + lk) * N + 4 * ct + li] += acc[s2][bt][ct];
        }
      }
      if (with_sub) {
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const int at = sat0 + s2;
          if (max(0, v0 - at * Q2) < min(Q2, v1 - at * Q2)) {
            const int a = 4 * at + lb;
#pragma unroll
            for (int bt = 0; bt < Q2; ++bt)
#pragma unroll
              for (int ct = 0; ct < Q2; ++ct) {
                const int b = 4 * bt + lk, c = 4 * ct + li;
                if (a < K && b < K && c < K) Ssum[(a * K + b) * K + c] += sacc[s2][bt][ct];
              }
          }
        }
      }
    }
    __syncthreads();
  }
  if (tr.partial >= 0) {
    double* dst = partials + (size_t)tr.partial * (N3 + K3);
    for (int e = tid; e < N3; e += 256) dst[e] = Bsum[e];
    if (with_sub)
      for (int e = tid; e < K3; e += 256) dst[N3 + e] = Ssum[e];
  } else {
    // child slab c gets rows (a, b) of its octant: element e of the slab is (i, j, m);
    // the 8 k^3 output elements are one contiguous run starting at the first child
    MRA_GLOBAL double* __restrict__ dst = out + (size_t)tr.fc * K3;
    stage_chunks<8 * K3, 18>(
        tid, [&](int e) { return dst[e]; },
        [&](int e, double v) {
          const int c = e / K3, r = e - c * K3;
          const int i = r / K2, j = (r / K) % K, m = r % K;
          const int a = ((c >> 2) & 1) * K + i, b = ((c >> 1) & 1) * K + j, cc = (c & 1) * K + m;
          dst[e] = v + Bsum[(a * N + b) * N + cc];
        });
    if (with_sub)
      for (int e = tid; e < K3; e += 256) subbuf[(size_t)tr.sub * K3 + e] = Ssum[e];
  }
}

// ----------------------------------------- apply (NS, MFMA, source streamed in z-slabs)
// FP64 matrix-core kernel for k = 14 (2k = 28 = 4Q, Q = 7), whose (2k)^3 children block
// (172 KB) does not fit in LDS.  A triple is processed in Q stages, one per z-quad: stage
// zq needs only the slab B_P[.][.][4zq .. 4zq+3] (25 KB), which is triple buffered in LDS
// and copied two stages ahead (across triples: the next triple's first slabs during the
// last two stages) by buffer loads that write LDS directly, so that a copy has two stages'
// products to land in.  Eight waves per workgroup, two per SIMD, so that one wave's LDS,
// permutation and barrier latencies overlap the other's products: waves 0-6 own one a-quad
// each and run the three contractions of it (step 1 contracts x, block index = z inside
// the z-quad; step 2 contracts y, chained in registers; the step-2 result is permuted
// in-wave into the step-3 operand, which contracts the z-quad's four z into the target's
// block held in registers).  Wave 7 owns the level-n subtraction -c (t x t x t) s_P (s_P
// resident in LDS per source; k = 14 is padded to 16 by masking the t fragments): its 16
// (a-quad, z-quad) units run in stages 0-5 (3, 3, 3, 3, 2, 2 units), those of a stage
// together (they share their s_P or t_x fragments).  Each wave keeps only its own
// accumulators, in half the register file, and waves 0-6 their a-quad's R_x fragments for
// the whole triple (step 1 then reads only the slab at each stage).  Operator blocks of the next triple are loaded
// into registers at its predecessor's last stage and stored to LDS at its first stage.
// Persistent workgroups take target ranges, longest first, from a counter.
template <int K>
__global__ __launch_bounds__(512) void apply_ns_stream_kernel(
    const double* const* __restrict__ in_tab, double* const* __restrict__ out_tab,
    const NSItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const double* const* __restrict__ r_tab, const double* const* __restrict__ t_tab,
    const double* const* __restrict__ c_tab, double* __restrict__ partials,
    double* __restrict__ subbuf, const int ntargets, int* __restrict__ next_target,
    const double* __restrict__ slabs) {
  constexpr int N = 2 * K, Q = N / 4, N2 = N * N, N3 = N * N * N, K2 = K * K, K3 = K * K * K;
  static_assert(K == 14 && Q == 7, "the wave split below is for k = 14");
  constexpr int Q2 = (K + 3) / 4;                              // subtraction quads (4)
  static_assert(Q2 == 4, "sixteen subtraction units");
  constexpr int SLY = 4, SLX = N * SLY, SLAB = N * SLX;        // slab [x][y][z in quad]
  static_assert(quarter_distinct(SLX, SLY), "slab strides");
  // slab copy: the children block of the source sits in `slabs` in slab order (granule g =
  // 2 (x N + y) + h holds (x, y, 4 zq + 2h .. 4 zq + 2h + 1)), so a stage copies one
  // contiguous range; rows of 64 granules, row r by wave r % 8
  // Every wave copies SRPW rows per stage (rows past SROWS read zeros into padding), so the
  // number of copies a wave has in flight at a stage's start is always SRPW.
  constexpr int SG = SLAB / 2, SROWS = (SG + 63) / 64, SRPW = (SROWS + 7) / 8, SPAD = 128 * 8 * SRPW;
  static_assert(SROWS == 25 && SRPW == 4, "four slab rows per wave");
  // operator buffer: R_x^T, R_y^T, R_z^T (N^2 each), then t_x^T, t_y^T, t_z^T (K^2 each in
  // slots of TSLOT, whose tails stay zero: a padded fragment read stays inside its slot)
  // R blocks in slots of 512 RL doubles, so that every thread loads and stores its RL
  // elements of each without a condition (the tail of a slot is never read; conditional
  // stores made the compiler wait for all copies in flight before each of them)
  constexpr int RL = (N2 + 511) / 512, RSLOT = 512 * RL, TSLOT = 256, OPS = 3 * RSLOT + 3 * TSLOT;
  static_assert(K2 <= 256 && (4 * Q2 - 1) * K + 4 * Q2 - 1 < TSLOT, "t slot");
  // s_P, row-major [x][y][z] as stored (granule copies), zero tail up to SSPAD: padded
  // fragment reads (x, y, z < 16) stay inside
  constexpr int SSG = K3 / 2, SSROWS = (SSG + 63) / 64, SSRPW = (SSROWS + 7) / 8;
  constexpr int SSPAD = ((15 * K2 + 15 * K + 16 + 127) / 128) * 128;
  static_assert(SSPAD >= 128 * SSROWS, "s_P rows fit");
  __shared__ __attribute__((aligned(16))) double Xl0[SPAD];
  __shared__ __attribute__((aligned(16))) double Xl1[SPAD];
  __shared__ __attribute__((aligned(16))) double Xl2[SPAD];
  __shared__ double Os[OPS];          // the current triple's operator blocks
  __shared__ __attribute__((aligned(16))) double Ss[SSPAD];
  __shared__ int s_next;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  const int swap = (16 * lb + 4 * lk + li) * 4;
  // padding that no copy writes is zero once and for all (fragment reads of padded quads
  // multiply it by zero operator entries, so it must be finite)
  for (int e = tid; e < SSPAD; e += 512) Ss[e] = 0.0;
  for (int e = tid; e < OPS; e += 512) Os[e] = 0.0;

  // row q of this wave's part of the slab copy (one instruction: 64 consecutive granules;
  // rows past the slab read zeros, their offsets being past the descriptor's end)
  auto copy_slab_row = [&](const int slot, const int zq, double* dst, const int q) {
    lds_copy16(slabs + (size_t)slot * (8 * K3) + (size_t)zq * SLAB, SLAB * 8,
               (MRA_LDS void*)(dst + 128 * (wave + 8 * q)), 16 * (64 * (wave + 8 * q) + lane));
  };
  static_assert(Q * SLAB == 8 * K3, "the seven slabs are the children block");
  auto copy_slab = [&](const int slot, const int zq, double* dst) {
#pragma unroll
    for (int q = 0; q < SRPW; ++q) copy_slab_row(slot, zq, dst, q);
  };
  // s_P (K3 doubles) into Ss, granule by granule, SSRPW rows per wave (rows past the block
  // read zeros into the zero tail: their offsets are past the descriptor's end)
  static_assert(SSPAD >= 128 * 8 * SSRPW, "every wave's s_P rows fit");
  auto copy_sp = [&](const double* in_g, const int src) {
#pragma unroll
    for (int q = 0; q < SSRPW; ++q)
      lds_copy16(in_g + (size_t)src * K3, K3 * 8, (MRA_LDS void*)(Ss + 128 * (wave + 8 * q)),
                 16 * (64 * (wave + 8 * q) + lane));
  };
  auto lane_swap = [&](double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(swap, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(swap, w.y);
    return __builtin_bit_cast(double, r);
  };
  __syncthreads();

  // The two roles (waves 0-6: an a-quad each; wave 7: the subtraction) run separate
  // instances of the loop, so that each keeps only its own accumulators live; both execute
  // the same sequence of barriers.
  // the range table, items and c_mu through the constant address space: scalar loads,
  // which do not count against the vector memory counter the slab copies are waited on with
  typedef const __attribute__((address_space(4))) NSItem* SItemPtr;
  typedef const __attribute__((address_space(4))) TargetRange* STargetPtr;
  typedef const __attribute__((address_space(4))) double* CPtr;
  const SItemPtr its = (SItemPtr)items;
  const STargetPtr tgs = (STargetPtr)targets;
  auto item_at = [&](const int i) {   // field by field: no struct copy across address spaces
    const SItemPtr p = its + i;
    NSItem r;
    r.src = p->src, r.src_fc = p->src_fc, r.mu = p->mu;
    r.rx = p->rx, r.ry = p->ry, r.rz = p->rz, r.tx = p->tx, r.ty = p->ty, r.tz = p->tz;
    r.slot = p->slot;
    return r;
  };
  auto run = [&](auto role_tag) {
    constexpr bool sub_wave = decltype(role_tag)::value;
    const int at0 = sub_wave ? 0 : wave;
    // per-lane offsets of the fragment reads, opaque so that every read is one offset from
    // its LDS array plus a constant: the compiler tags only short address chains with the
    // array they read, and an untagged read waits for every LDS copy in flight
    const int o_r = opaque_int(lk * N + li);                         // R^T fragment (row, col)
    const int o_ra = opaque_int(lk * N + li + 4 * at0);
    const int o_x = opaque_int(lk * SLX + li * SLY + lb);            // slab fragment
    const int o_t = sub_wave ? opaque_int(lk * K + li) : 0;          // t^T fragment
    const int o_s = sub_wave ? opaque_int(lk * K2 + li * K + lb) : 0;  // s_P fragment
    for (;;) {
      if (tid == 0) s_next = atomicAdd(next_target, 1);
      __syncthreads();
      const int ti = __builtin_amdgcn_readfirstlane(s_next);   // uniform: scalar item loads
      __syncthreads();   // every wave has read s_next (and is done with the previous range)
      if (ti >= ntargets) break;
      TargetRange tr;
      {
        const STargetPtr p = tgs + ti;
        tr.fn = p->fn, tr.node = p->node, tr.fc = p->fc, tr.beg = p->beg, tr.end = p->end;
        tr.partial = p->partial, tr.sub = p->sub;
      }
      const double* const in_g = in_tab[tr.fn];
      MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
      const MRA_GLOBAL double* __restrict__ dR = as_global(r_tab[tr.fn]);
      const MRA_GLOBAL double* __restrict__ dT = as_global(t_tab[tr.fn]);
      const CPtr dc = (CPtr)c_tab[tr.fn];
      const bool with_sub = tr.sub >= 0;

      // operator blocks of a triple: element tid + 512 q of each block (t blocks: tid,
      // clamped to the slot's last element, which those threads write with the same value)
      double opre[3 * RL + 3];
      auto fetch_ops = [&](const NSItem& nx) {
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          const MRA_GLOBAL double* __restrict__ src =
              dR + (size_t)(w == 0 ? nx.rx : w == 1 ? nx.ry : nx.rz) * N2;
#pragma unroll
          for (int q = 0; q < RL; ++q) opre[w * RL + q] = src[min(tid + 512 * q, N2 - 1)];
        }
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          const MRA_GLOBAL double* __restrict__ src =
              dT + (size_t)(w == 0 ? nx.tx : w == 1 ? nx.ty : nx.tz) * K2;
          opre[3 * RL + w] = src[min(tid, K2 - 1)];   // the slot's tail is read masked only
        }
      };
      auto store_ops = [&](double* dst) {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
          for (int q = 0; q < RL; ++q) dst[w * RSLOT + tid + 512 * q] = opre[w * RL + q];
#pragma unroll
        for (int w = 0; w < 3; ++w) dst[3 * RSLOT + w * TSLOT + min(tid, TSLOT - 1)] = opre[3 * RL + w];
      };

      // accumulators: waves 0-6 keep their a-quad's block in acc0, wave 7 the subtraction
      // block (4 a-quads x 4 b-quads x 4 c-quads) in acc1
      constexpr int A1 = sub_wave ? Q2 * Q2 * Q2 : 1;
      double acc0[Q][Q], acc1[A1];
#pragma unroll
      for (int b = 0; b < Q; ++b)
#pragma unroll
        for (int c = 0; c < Q; ++c) acc0[b][c] = 0.0;
#pragma unroll
      for (int e = 0; e < A1; ++e) acc1[e] = 0.0;

      // the current triple needs its source (children block and s_P) and c_mu; the next
      // one its whole record
      int cur_slot = 0, cur_src = -1;
      double c_cur = 0.0;
      NSItem nxt{};
      if (tr.beg < tr.end) {
        const NSItem first = item_at(tr.beg);
        cur_slot = first.slot;
        cur_src = first.src;
        c_cur = dc[first.mu];
        nxt = item_at(min(tr.beg + 1, tr.end - 1));
        copy_slab(cur_slot, 0, Xl0);
        if (with_sub) copy_sp(in_g, cur_src);
        fetch_ops(first);   // stored at the triple's first stage
        copy_slab(cur_slot, 1, Xl1);   // last: the first stage waits for all but these
      }
      int it = tr.beg, zq = 0;
      const int nstages = Q * (tr.end - tr.beg);
      // wave 7: the t_y fragments of the current triple (the same for all its 16 units)
      constexpr int TYC = sub_wave ? Q2 : 1;
      double tyc[TYC][TYC];
      // waves 0-6: the R_x fragments of their a-quad for the current triple
      constexpr int RXA = sub_wave ? 1 : Q;
      double rxa[RXA];

      auto stage = [&](auto buf_tag) {
        constexpr int buf = decltype(buf_tag)::value;
        double* const Xc = buf == 0 ? Xl0 : buf == 1 ? Xl1 : Xl2;   // this stage's slab
        double* const Xn = buf == 0 ? Xl2 : buf == 1 ? Xl0 : Xl1;   // two stages ahead
        // vmcnt(SRPW) lgkmcnt(0): everything this wave issued before its last SRPW copies
        // (those of the next stage) has landed, i.e. this stage's slab and the operator
        // blocks and s_P loaded during the previous stage, and its LDS reads of the previous
        // stage are done; after the barrier the same holds for every wave, so the slab is
        // complete and the previous stage's buffer is free
        static_assert(SRPW < 16, "vmcnt field");
        lds_barrier<0x0070 | SRPW>();
        if (zq == 0) {
          // this triple's operator blocks (loaded into registers during the previous triple's
          // last stage) into LDS: every wave has finished that triple
          store_ops(Os);
          lds_barrier<0xC07F>();   // lgkmcnt(0): the stores are done
        }
        const bool more = it + 1 < tr.end;
        // the slab two stages ahead (this triple's zq + 2 or the next triple's zq + 2 - Q;
        // past the range's last stage a repeat of this triple's first slab into the free
        // buffer, which keeps the number of copies in flight fixed), one copy instruction per
        // x-quad group of step 1, so that the in-order wave never waits for the memory
        // pipeline to take a burst of them
        const bool same = zq + 2 < Q;
        const int copy_slot = same || !more ? cur_slot : nxt.slot;
        const int copy_zq = same ? zq + 2 : more ? zq + 2 - Q : 0;
        auto copy_part = [&](const int q) { copy_slab_row(copy_slot, copy_zq, Xn, q); };
        // the next triple's operator blocks into registers (stored after this stage's
        // products; issued before this stage's copies, so that the wait for them before the
        // stores is not a wait for the copies), then s_P of its source (wave 7 reads s_P in
        // stages 0-5 only)
        if (zq + 1 == Q && more) fetch_ops(nxt);
        if (zq + 1 == Q && more && with_sub && nxt.src != cur_src) copy_sp(in_g, nxt.src);
        const double cmu = c_cur;
        if constexpr (!sub_wave) {
          // ---- waves 0-6: a-quad `wave`
          double rz[Q];
#pragma unroll
          for (int ct = 0; ct < Q; ++ct) rz[ct] = cmu * Os[2 * RSLOT + o_r + 4 * zq * N + 4 * ct];
          double d1[Q];
#pragma unroll
          for (int yt = 0; yt < Q; ++yt) d1[yt] = 0.0;
          double xa[2][Q];
          // the a-quad's R_x fragments are the same at every stage of a triple: read once
          if (zq == 0) {
#pragma unroll
            for (int xs = 0; xs < Q; ++xs) rxa[xs] = Os[o_ra + 4 * xs * N];
          }
          auto load1 = [&](const int xs, const int b) {
#pragma unroll
            for (int yt = 0; yt < Q; ++yt) xa[b][yt] = Xc[o_x + 4 * xs * SLX + 4 * yt * SLY];
          };
          load1(0, 0);
#pragma unroll
          for (int xs = 0; xs < Q; ++xs) {
            const int b = xs & 1;
            if (xs < SRPW) copy_part(xs);
            if (xs + 1 < Q) load1(xs + 1, b ^ 1);
#pragma unroll
            for (int yt = 0; yt < Q; ++yt)
              d1[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(xa[b][yt], rxa[xs], d1[yt], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
          }
          double zr[Q];
#pragma unroll
          for (int bt = 0; bt < Q; ++bt) zr[bt] = 0.0;
          double ry[2][Q];
          auto load2 = [&](const int ys, const int b) {
#pragma unroll
            for (int bt = 0; bt < Q; ++bt) ry[b][bt] = Os[RSLOT + o_r + 4 * ys * N + 4 * bt];
          };
          load2(0, 0);
          double za_n;
#pragma unroll
          for (int ys = 0; ys < Q; ++ys) {
            const int b = ys & 1;
            if (ys + 1 < Q) load2(ys + 1, b ^ 1);
#pragma unroll
            for (int bt = 0; bt < Q; ++bt) {
              zr[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(d1[ys], ry[b][bt], zr[bt], 0, 0, 0);
              if (ys == Q - 1 && bt == 3) za_n = lane_swap(zr[0]);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int bt = 0; bt < Q; ++bt) {
            const double za = za_n;
            if (bt + 1 < Q) za_n = lane_swap(zr[bt + 1]);
#pragma unroll
            for (int ct = 0; ct < Q; ++ct)
              acc0[bt][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(za, rz[ct], acc0[bt][ct], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
          }
        } else {
          // ---- wave 7: its rows of the slab copy, then the level-n subtraction units
#pragma unroll
          for (int q = 0; q < SRPW; ++q) copy_part(q);
          // ---- the level-n subtraction units of this stage: (sa, sz), sa fixed per call; the
          // units of a stage are independent, so their instructions may interleave
          if (with_sub && zq < 6) {
            // The units of a stage share their source fragments (stages 0-3: sa = 0, 1, 2 at
            // sz = zq, one s_P z-quad) or their t_x fragments (stages 4-5: sa = 3 at two sz),
            // so they run together: shared fragments read once, 8-12 independent product
            // chains per step, and all in-wave permutations issued before the last products.
            // t fragment (row quad rq, column quad cq) of a transposed t block at slot
            // offset base, zero outside k x k (row 4 rq + lk, column 4 cq + li)
            auto tf = [&](const int base, const int rq, const int cq) {
              const double v = Os[base + o_t + 4 * rq * K + 4 * cq];
              return ((rq < Q2 - 1 || lk < K - 4 * (Q2 - 1)) && (cq < Q2 - 1 || li < K - 4 * (Q2 - 1))) ? v : 0.0;
            };
            auto units = [&](auto case_tag) {
              constexpr bool by_sa = decltype(case_tag)::value;
              constexpr int NU = by_sa ? 3 : 2;
              const int sz0 = by_sa ? zq : 2 * (zq - 4);   // unit u has sz = sz0 (+ u if !by_sa)
              double e1[NU][Q2];
#pragma unroll
              for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int yt = 0; yt < Q2; ++yt) e1[u][yt] = 0.0;
#pragma unroll
              for (int xs = 0; xs < Q2; ++xs) {
                if constexpr (by_sa) {
                  double sf[Q2], tq[NU];
#pragma unroll
                  for (int yt = 0; yt < Q2; ++yt) sf[yt] = Ss[o_s + 4 * xs * K2 + 4 * yt * K + 4 * sz0];
#pragma unroll
                  for (int u = 0; u < NU; ++u) tq[u] = tf(3 * RSLOT, xs, u);
#pragma unroll
                  for (int u = 0; u < NU; ++u)
#pragma unroll
                    for (int yt = 0; yt < Q2; ++yt)
                      e1[u][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(sf[yt], tq[u], e1[u][yt], 0, 0, 0);
                } else {
                  double sf[NU][Q2];
#pragma unroll
                  for (int u = 0; u < NU; ++u)
#pragma unroll
                    for (int yt = 0; yt < Q2; ++yt)
                      sf[u][yt] = Ss[o_s + 4 * xs * K2 + 4 * yt * K + 4 * (sz0 + u)];
                  const double tq = tf(3 * RSLOT, xs, Q2 - 1);
#pragma unroll
                  for (int u = 0; u < NU; ++u)
#pragma unroll
                    for (int yt = 0; yt < Q2; ++yt)
                      e1[u][yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(sf[u][yt], tq, e1[u][yt], 0, 0, 0);
                }
              }
              // the t_y fragments (the same for every unit of the triple), read here rather
              // than held across stages: the subtraction block fills half the register file
#pragma unroll
              for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
                for (int bt = 0; bt < Q2; ++bt) tyc[ys % TYC][bt % TYC] = tf(3 * RSLOT + TSLOT, ys, bt);
              double e2[NU][Q2];
#pragma unroll
              for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int bt = 0; bt < Q2; ++bt) e2[u][bt] = 0.0;
#pragma unroll
              for (int ys = 0; ys < Q2; ++ys)
#pragma unroll
                for (int u = 0; u < NU; ++u)
#pragma unroll
                  for (int bt = 0; bt < Q2; ++bt)
                    e2[u][bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(e1[u][ys], tyc[ys % TYC][bt % TYC],
                                                                   e2[u][bt], 0, 0, 0);
              constexpr int NZ = by_sa ? 1 : NU;
              double tz[NZ][Q2];
#pragma unroll
              for (int v = 0; v < NZ; ++v)
#pragma unroll
                for (int ct = 0; ct < Q2; ++ct) tz[v][ct] = -cmu * tf(3 * RSLOT + 2 * TSLOT, sz0 + v, ct);
              double z[NU][Q2];
#pragma unroll
              for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int bt = 0; bt < Q2; ++bt) z[u][bt] = lane_swap(e2[u][bt]);
#pragma unroll
              for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int bt = 0; bt < Q2; ++bt)
#pragma unroll
                  for (int ct = 0; ct < Q2; ++ct) {
                    const int sa = by_sa ? u : Q2 - 1;
                    acc1[((sa * Q2 + bt) * Q2 + ct) % A1] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                        z[u][bt], tz[by_sa ? 0 : u][ct], acc1[((sa * Q2 + bt) * Q2 + ct) % A1], 0, 0, 0);
                  }
            };
            __builtin_amdgcn_sched_barrier(0);
            if (zq < 4)
              units(BoolTag<true>{});
            else
              units(BoolTag<false>{});
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        // advance
        if (++zq == Q) {
          zq = 0;
          ++it;
          cur_slot = nxt.slot;
          cur_src = nxt.src;
          c_cur = dc[nxt.mu];
          nxt = item_at(min(it + 1, tr.end - 1));
        }
      };
      // (nested: the compiler must see that the third stage always follows the second, or
      // it cannot tell that the first stage's copies have landed when the third starts)
      for (int s = 0; s < nstages; s += 3) {
        stage(BufTag<0>{});
        if (s + 1 < nstages) {
          stage(BufTag<1>{});
          if (s + 2 < nstages) stage(BufTag<2>{});
        }
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);   // the repeated copies of the last two stages
      // ---- write the target's blocks (each element owned by exactly one lane).  The lane
      // indices pass through an empty asm statement, so that the compiler recomputes the
      // output offsets here instead of keeping ~100 of them live across the whole loop.
      const int wl = opaque_int(lane);
      const int li = wl & 3, lb = (wl >> 2) & 3, lk = wl >> 4;
      constexpr int nq = sub_wave ? 0 : 1;
#pragma unroll
      for (int s2 = 0; s2 < nq; ++s2) {
        const int a = 4 * at0 + lb;
#pragma unroll
        for (int bt = 0; bt < Q; ++bt) {
          const int b = 4 * bt + lk;
          if (tr.partial >= 0) {
#pragma unroll
            for (int ct = 0; ct < Q; ++ct)
              partials[(size_t)tr.partial * (N3 + K3) + (a * N + b) * N + 4 * ct + li] =
                  acc0[bt][ct];
          } else {
            // a row of Q elements: all loads first, then the sums and stores
            size_t off[Q];
            double o[Q];
#pragma unroll
            for (int ct = 0; ct < Q; ++ct) {
              const int c = 4 * ct + li;
              const int child = ((a / K) << 2) | ((b / K) << 1) | (c / K);
              off[ct] = (size_t)(tr.fc + child) * K3 + ((a % K) * K + (b % K)) * K + (c % K);
              o[ct] = out[off[ct]];
            }
#pragma unroll
            for (int ct = 0; ct < Q; ++ct)
              out[off[ct]] = o[ct] + acc0[bt][ct];
          }
        }
      }
      if (sub_wave && with_sub) {
#pragma unroll
        for (int sa = 0; sa < Q2; ++sa) {
          const int a = 4 * sa + lb;
#pragma unroll
          for (int bt = 0; bt < Q2; ++bt)
#pragma unroll
            for (int ct = 0; ct < Q2; ++ct) {
              const int b = 4 * bt + lk, c = 4 * ct + li;
              if (a < K && b < K && c < K) {
                const double v = acc1[((sa * Q2 + bt) * Q2 + ct) % A1];
                if (tr.partial >= 0)
                  partials[(size_t)tr.partial * (N3 + K3) + N3 + (a * K + b) * K + c] = v;
                else
                  subbuf[(size_t)tr.sub * K3 + (a * K + b) * K + c] = v;
              }
            }
        }
      }
    }
  };
  if (wave == 7)
    run(BoolTag<true>{});
  else
    run(BoolTag<false>{});
}

// For each listed box, its children block rewritten in the k = 14 streaming kernel's slab
// order: the seven z-quad slabs one after another, slab zq holding (x, y, 4 zq + zz) at
// (x 2k + y) 4 + zz.  One workgroup per box, writes in order (reads gather runs of four z).
template <int K>
__global__ __launch_bounds__(256) void slab_mirror_kernel(double* const* __restrict__ tab,
                                                          const NodeRef* __restrict__ refs,
                                                          double* __restrict__ slabs) {
  constexpr int N = 2 * K, K3 = K * K * K, SLAB = N * N * 4;
  static_assert(N % 4 == 0 && (N / 4) * SLAB == 8 * K3, "whole z-quads");
  const NodeRef ref = refs[blockIdx.x];
  const MRA_GLOBAL double* __restrict__ src = as_global(tab[ref.fn]) + (size_t)ref.fchild * K3;
  MRA_GLOBAL double* __restrict__ dst = as_global(slabs) + (size_t)blockIdx.x * (8 * K3);
  for (int e = threadIdx.x; e < 8 * K3; e += 256) {
    const int zq = e / SLAB, r = e - zq * SLAB, xy = r >> 2, z = 4 * zq + (r & 3);
    const int x = xy / N, y = xy - x * N;
    const int c = ((x / K) << 2) | ((y / K) << 1) | (z / K);
    dst[e] = src[c * K3 + ((x % K) * K + y % K) * K + z % K];
  }
}

// ------------------------------------------------------------- apply (low tier, BF16)
// The BF16 tier kernel runs eight waves per workgroup (two per SIMD, so that one wave's
// matrix-core and conversion latencies overlap the other's work); wave w owns a-quad w.
constexpr int kLowWaves = 8;
// Step-x tiles per wave, shifted towards the waves without an a-quad for steps z and y (80
// products per quad against 4 per tile), with at most 7 tiles per wave so that the
// accumulators fit beside the source rows in a half of the register file.
__host__ __device__ constexpr int low_tiles(int k, int w) {
  return k == 14 ? (w < 7 ? 6 : 7) : k == 12 ? (w < 6 ? 4 : 6) : (w < 5 ? 2 : 5);
}
__host__ __device__ constexpr int low_tile0(int k, int w) {
  return w == 0 ? 0 : low_tile0(k, w - 1) + low_tiles(k, w - 1);
}
// Triples whose norm bound eta is far below thresh.  Each adds its whole contribution to
// the target's children block,
//   c_mu [(R_x x R_y x R_z) - (P_x x P_y x P_z)] B_P,   P = H^T t H  (level n > 0),
// which equals the FP64 path's children term plus the unfiltered level-n subtraction.
// It is evaluated in the cancellation-free form
//   E_x R_y R_z + P_x E_y R_z + P_x P_y E_z = E_x (R_y (R_z B)) + P_x (E_y (R_z B) + P_y (E_z B)),
// E = R - P, so each rounding error is relative to a term whose norm is bounded by a part
// of N(delta) = prod(a + e) - prod(a) (Sec. 2.2 decay of the difference operators).
// Operands are BF16 (inputs rounded from FP64), products accumulate in FP32 on
// v_mfma_f32_16x16x32_bf16, the target's block is added to the FP64 output once.
//
// Matrix-core layout (16x16x32): lane l = 16 g + r holds A[r][8g + j] and B[8g + j][r]
// (j < 8) and receives D[4g + i][r] (i < 4).  Tensors are [a][b][c] (x, y, z), each index
// < N = 2k <= 32, i.e. two 16-wide tiles.  For a fixed a, step z (contract c) takes the
// source rows X[a][b][.] as A and R_z / E_z rows as B; its two row tiles (b < 16, b >= 16)
// stacked lane-wise are the B operand of step y (contract b) if the contraction slots of
// step y are permuted accordingly (the V layout of the operator records).  Step x (contract
// a) needs all a of a column (b', c'): each wave handles a whole quad of a (wave w: quad w),
// writes the two results of step y (R_y-part and E_y/P_y-part, c_mu applied, BF16) of the
// quad's four a as one 8-byte write to LDS rows q = (b', c') of 32 a slots, and
// after a barrier every wave contracts its share of the q tiles with E_x and P_x,
// accumulating in registers over all triples of the target.  Granule h (a = 8h .. 8h + 7)
// of row q sits at position h ^ ((q >> 1) & 3) of the row: eight consecutive rows then
// cover all 32 banks with their granules, so the 16-byte reads of step x (eight lanes,
// consecutive q) and the 8-byte writes (sixteen lanes, consecutive q, one half of each
// granule) have no bank conflicts beyond two-way on the writes.  Slots a >= 2k are zero
// from the start and never written.
//
// The seven operator matrices a triple reads (U(R_z), U(E_z), V(R_y), V(E_y), V(P_y), U(E_x),
// U(P_x)) are copied into LDS one triple ahead by buffer loads that write LDS directly
// (rows padded to an odd number of 16-byte granules, so that the fragment reads of 16 rows
// are bank-conflict free); the two halves of that double buffer are separate objects, the
// loop is unrolled by two over them.  Persistent workgroups take target ranges, longest
// first, from a counter.
template <int K>
__global__ __launch_bounds__(64 * kLowWaves) void apply_low_kernel(
    const uint16_t* __restrict__ mirror, double* const* __restrict__ out_tab,
    const LowItem* __restrict__ items, const TargetRange* __restrict__ targets,
    const uint16_t* const* __restrict__ l_tab, const double* const* __restrict__ c_tab,
    const int ntargets, int* __restrict__ next_target) {
  constexpr int N = 2 * K, N2 = N * N, K3 = K * K * K;
  constexpr int UP = (N + 7) / 8 * 8;          // padded contraction length (U layout)
  constexpr int XB = N * N * UP;               // BF16 per mirrored children block
  constexpr int LU = N * UP, LV = N * 32, REC = 3 * LU + 3 * LV;
  constexpr int NW = kLowWaves, NT = 64 * NW;
  constexpr int NQUAD = N / 4, QDW = (NQUAD + NW - 1) / NW;   // a-quads; wave w owns quad w
  static_assert(QDW == 1, "one a-quad per wave");
  constexpr int NQ = N2 / 16;                           // 16-row tiles of step x
  constexpr int TMAX = low_tiles(K, 0) > low_tiles(K, NW - 1) ? low_tiles(K, 0) : low_tiles(K, NW - 1);
  constexpr int TMIN = low_tiles(K, 0) < low_tiles(K, NW - 1) ? low_tiles(K, 0) : low_tiles(K, NW - 1);
  static_assert(low_tile0(K, NW) == NQ && TMAX <= 7, "every step-x tile has one wave");
  constexpr int TSZ = (N2 + 1) * 32;                    // T rows [q][a slot], 4 granules each,
                                                        // and a row that takes the padding writes
  static_assert(N > 16 && N <= 32 && N2 % 16 == 0 && N % 4 == 0, "two 16-wide tiles per index, even k");
  // operator staging: matrix m has N rows of GM[m] granules (8 BF16 each) in the record,
  // RSM[m] (odd) granules per row in LDS; the extra granules read zeros
  constexpr int GU = UP / 8, GV = 4;
  constexpr int RU = GU % 2 ? GU : GU + 1, RV = GV % 2 ? GV : GV + 1;
  constexpr int SU = 8 * RU, SV = 8 * RV;      // LDS row strides in BF16
  constexpr int MU = N * RU, MV = N * RV;      // granules per staged matrix
  constexpr int OPG = 4 * MU + 3 * MV, OROWS = (OPG + 63) / 64, ORPW = (OROWS + NW - 1) / NW;
  // BF16 offsets of the staged matrices
  constexpr int O_RZ = 0, O_EZ = 8 * MU, O_RY = 16 * MU, O_EY = O_RY + 8 * MV, O_PY = O_EY + 8 * MV;
  constexpr int O_EX = O_PY + 8 * MV, O_PX = O_EX + 8 * MU;
  // BF16 per half of the staging buffer: the copied rows, and room for the fragment reads of
  // rows up to 31 (rows >= 2k are read without a mask: they only reach outputs >= 2k, which
  // are never stored)
  constexpr int OPB_C = 8 * 64 * OROWS, OPB_R = (O_PX + 31 * SU + 32 + 511) / 512 * 512;
  constexpr int OPB = OPB_C > OPB_R ? OPB_C : OPB_R;
  static_assert(O_PY + 31 * SV + 32 <= OPB && O_EZ + 31 * SU + 32 <= OPB, "fragment reads in bounds");
  __shared__ __attribute__((aligned(16))) uint16_t T1s[TSZ];
  __shared__ __attribute__((aligned(16))) uint16_t T2s[TSZ];
  __shared__ __attribute__((aligned(16))) uint16_t Ob0[OPB];
  __shared__ __attribute__((aligned(16))) uint16_t Ob1[OPB];
  __shared__ int s_next;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar branches
  const int g = lane >> 4, r = lane & 15;
  // this wave's step-x tiles [tw0, tw0 + tw) (an unrolled sum: a recursive constexpr call
  // with the runtime wave index would be compiled as a real call)
  int tw0 = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) tw0 += w < wave ? low_tiles(K, w) : 0;
  const int tw = low_tiles(K, wave);
  const bf16x8 zero8 = __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
  auto ld8 = [&](const uint16_t* p) { return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p)); };
  auto ld8g = [&](const MRA_GLOBAL uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *(const MRA_GLOBAL u32x4*)p);
  };
  // slots a >= 2k of the T rows are never written, and the staging buffers' tails are read
  // unmasked (into outputs that are never stored): clear everything once, so that all of it
  // is finite
  for (int e = tid; e < TSZ / 8; e += NT) {
    reinterpret_cast<u32x4*>(T1s)[e] = u32x4{0u, 0u, 0u, 0u};
    reinterpret_cast<u32x4*>(T2s)[e] = u32x4{0u, 0u, 0u, 0u};
  }
  for (int e = tid; e < OPB / 8; e += NT) {
    reinterpret_cast<u32x4*>(Ob0)[e] = u32x4{0u, 0u, 0u, 0u};
    reinterpret_cast<u32x4*>(Ob1)[e] = u32x4{0u, 0u, 0u, 0u};
  }
  // Operator staging: lane l of staging row w' = wave + NW q copies granule j = 64 w' + l of
  // the seven matrices laid out one after another with RU / RV granules per row; its source
  // is a granule of the record of R_z, R_y or R_x (selected per triple from the item) or,
  // for row padding and past the last matrix, nothing (an offset past the descriptor's
  // range, which reads zeros).  The per-lane offsets are recomputed at every staging from
  // an opaque copy of the lane index instead of being held in registers.
  constexpr unsigned kPast = 0x7FFFFFF0u;
  // items and c_mu through the constant address space: uniform reads become scalar loads,
  // which do not count against the vector-memory counter that the copies are waited on
  typedef const __attribute__((address_space(4))) LowItem* ItemPtr;
  const ItemPtr itc = (ItemPtr)items;
  auto stage_ops = [&](const MRA_GLOBAL uint16_t* L, const ItemPtr nx, uint16_t* dst) {
    const int sl = opaque_int(lane);
    const unsigned rb[3] = {(unsigned)nx->rz * (2u * REC), (unsigned)nx->ry * (2u * REC),
                            (unsigned)nx->rx * (2u * REC)};
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)L, (short)0, (int)kPast, 0x00020000);
#pragma unroll
    for (int q = 0; q < ORPW; ++q) {
      if (wave + NW * q < OROWS) {
        const int j = 64 * (wave + NW * q) + sl;
        const int mstart[8] = {0, MU, 2 * MU, 2 * MU + MV, 2 * MU + 2 * MV, 2 * MU + 3 * MV,
                               3 * MU + 3 * MV, OPG};
        // record parts: U(R), U(E), U(P) at 0, LU, 2 LU; V(R), V(E), V(P) at 3 LU + m LV
        const int part[7] = {0, LU, 3 * LU, 3 * LU + LV, 3 * LU + 2 * LV, LU, 2 * LU};
        const int recsel[7] = {0, 0, 1, 1, 1, 2, 2};
        unsigned off = kPast, base = 0u;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
          const bool u = m < 2 || m >= 5;
          const int rs_ = u ? RU : RV, gm = u ? GU : GV, w = u ? UP : 32;
          const int jj = j - mstart[m];
          const bool in = j >= mstart[m] && j < mstart[m + 1];
          const int row = jj / rs_, col = jj - (jj / rs_) * rs_;
          off = (in && col < gm) ? (unsigned)(2 * (part[m] + row * w + 8 * col)) : off;
          base = in ? rb[recsel[m]] : base;
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (MRA_LDS void*)(dst + 512 * (wave + NW * q)),
                                                 16, (int)(off + base), 0, 0, 0);
      }
    }
  };
  __syncthreads();

  for (;;) {
    if (tid == 0) s_next = atomicAdd(next_target, 1);
    __syncthreads();
    const int ti = __builtin_amdgcn_readfirstlane(s_next);   // uniform: scalar item loads
    __syncthreads();   // every wave has read s_next (and is done with the previous range)
    if (ti >= ntargets) break;
    const TargetRange tr = targets[ti];
    MRA_GLOBAL double* __restrict__ out = as_global(out_tab[tr.fn]);
    const MRA_GLOBAL uint16_t* __restrict__ L = as_global(l_tab[tr.fn]);
    typedef const __attribute__((address_space(4))) double* CPtr;
    const CPtr dc = (CPtr)c_tab[tr.fn];

    f32x4 acc[TMAX][2];
#pragma unroll
    for (int e = 0; e < TMAX; ++e)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) acc[e][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 xr[QDW][4][2];   // [quad of this wave][a in quad][b tile]: A operand of step z
    // this wave's rows of a mirrored source block into xr
    auto load_src = [&](const int slot) {
      const int wl = opaque_int(lane);      // offsets recomputed here, not held
      const int gg = wl >> 4, rr = wl & 15;
      // global (not flat) loads: they count against the vector-memory counter only, so the
      // LDS waits of step x do not wait for them
      const MRA_GLOBAL uint16_t* xb = as_global(mirror) + (size_t)slot * XB;
#pragma unroll
      for (int hq = 0; hq < QDW; ++hq)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            // rows b >= 2k repeat row 2k - 1 (finite; they only reach step-y slots whose
            // operator columns are zero); slots c >= UP must be zero (the step-z operator
            // fragments there are not masked)
            const int quad = wave + NW * hq, a = 4 * quad + j, b = min(16 * mt + rr, N - 1);
            if (quad < NQUAD)
              xr[hq][j][mt] = (UP == 32 || 8 * gg < UP) ? ld8g(xb + (a * N + b) * UP + 8 * gg) : zero8;
          }
    };
    // items are indexed, never copied (a copy of a whole item went through private memory)
    float cmu_next = 0.f;
    if (tr.beg < tr.end) {
      stage_ops(L, itc + tr.beg, Ob0);
      load_src(itc[tr.beg].slot);
      cmu_next = (float)dc[itc[tr.beg].mu];
    }
    auto triple = [&](const int it, auto buf_tag) {
      constexpr int buf = decltype(buf_tag)::value;
      const uint16_t* const Oc = buf == 0 ? Ob0 : Ob1;   // this triple's operators
      uint16_t* const On = buf == 0 ? Ob1 : Ob0;         // the next triple's
      const ItemPtr item = itc + it, nxt = itc + min(it + 1, tr.end - 1);
      const bool more = it + 1 < tr.end;
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies landed
      __syncthreads();                      // all copies landed; step x of it - 1 is done
      const float cmu = cmu_next;          // loaded one triple ahead
      if (more) stage_ops(L, nxt, On);
      cmu_next = (float)dc[nxt->mu];
      bf16x8 oz[2][2], oy[3][2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int row = 16 * t + r;
        oz[0][t] = ld8(Oc + O_RZ + row * SU + 8 * g);       // U(R_z)
        oz[1][t] = ld8(Oc + O_EZ + row * SU + 8 * g);       // U(E_z)
        oy[0][t] = ld8(Oc + O_RY + row * SV + 8 * g);       // V(R_y)
        oy[1][t] = ld8(Oc + O_EY + row * SV + 8 * g);       // V(E_y)
        oy[2][t] = ld8(Oc + O_PY + row * SV + 8 * g);       // V(P_y)
      }
      // ---- steps z and y for this wave's quads of a; the four results of a (mt', i) slot
      // (the quad's four a) go to LDS as one 8-byte write.  The write offsets depend on the
      // lane and the wave only (the compiler keeps them in registers across the loop).
      const int zl = lane;
      const int zg = zl >> 4, zr = zl & 15;
#pragma unroll
      for (int hq = 0; hq < QDW; ++hq) {
        const int quad = wave + NW * hq;
        if (quad < NQUAD) {
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            bf16x8 b1[4], b2[4];   // step-z results of the quad's four a: B operands of step y
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              f32x4 y1[2], y2[2];
#pragma unroll
              for (int mt = 0; mt < 2; ++mt) {
                const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
                y1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xr[hq][j][mt], oz[0][nt], z4, 0, 0, 0);
                y2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xr[hq][j][mt], oz[1][nt], z4, 0, 0, 0);
              }
              // c_mu is applied here, before the rounding to BF16 (to the 8 values of the step-y
              // operand rather than to the 16 results)
              const bf16x4 p0 = __builtin_convertvector(cmu * y1[0], bf16x4);
              const bf16x4 p1 = __builtin_convertvector(cmu * y1[1], bf16x4);
              const bf16x4 p2 = __builtin_convertvector(cmu * y2[0], bf16x4);
              const bf16x4 p3 = __builtin_convertvector(cmu * y2[1], bf16x4);
              b1[j] = __builtin_shufflevector(p0, p1, 0, 1, 2, 3, 4, 5, 6, 7);
              b2[j] = __builtin_shufflevector(p2, p3, 0, 1, 2, 3, 4, 5, 6, 7);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
              f32x4 u[4], v[4];   // [a in quad]
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
                u[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oy[0][mt], b1[j], z4, 0, 0, 0);
                v[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oy[1][mt], b1[j], z4, 0, 0, 0);
                v[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oy[2][mt], b2[j], v[j], 0, 0, 0);
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                // lanes outside the 2k x 2k (b', c') range write into the extra row N2
                const int bp = 16 * mt + 4 * zg + i, cp = 16 * nt + zr;
                const int q = (bp < N && cp < N) ? bp * N + cp : N2;
                const int off = q * 32 + 8 * ((quad >> 1) ^ ((q >> 1) & 3)) + 4 * (quad & 1);
                const f32x4 cu = {u[0][i], u[1][i], u[2][i], u[3][i]};
                const f32x4 cv = {v[0][i], v[1][i], v[2][i], v[3][i]};
                *reinterpret_cast<bf16x4*>(&T1s[off]) = __builtin_convertvector(cu, bf16x4);
                *reinterpret_cast<bf16x4*>(&T2s[off]) = __builtin_convertvector(cv, bf16x4);
              }
            }
          }
        }
      }
      lds_barrier();   // T1/T2 complete (the operator copies in flight are not waited for)
      // xr is free once steps z and y are done: the next triple's source rows load during
      // step x
      if (more && nxt->slot != item->slot) load_src(nxt->slot);
      // ---- step x: acc[a'][q] += E_x T1 + P_x T2 over this wave's q tiles
      bf16x8 ox[2][2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int row = 16 * t + r;
        ox[0][t] = ld8(Oc + O_EX + row * SU + 8 * g);       // U(E_x)
        ox[1][t] = ld8(Oc + O_PX + row * SU + 8 * g);       // U(P_x)
      }
      const int xl = lane;
      const int xg = xl >> 4, xrr = xl & 15;
      // (the first TMIN tiles, which every wave has, are straight-line code: their reads can
      // be issued ahead of the products)
#pragma unroll
      for (int e = 0; e < TMAX; ++e) {
        if (e < TMIN || e < tw) {
          const int q = 16 * (tw0 + e) + xrr, off = q * 32 + 8 * (xg ^ ((q >> 1) & 3));
          const bf16x8 t1 = ld8(T1s + off);   // slots a >= 2k are zero
          const bf16x8 t2 = ld8(T2s + off);
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            acc[e][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ox[0][mt], t1, acc[e][mt], 0, 0, 0);
            acc[e][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ox[1][mt], t2, acc[e][mt], 0, 0, 0);
          }
        }
      }
    };
    for (int it = tr.beg; it < tr.end; it += 2) {
      triple(it, BufTag<0>{});
      if (it + 1 < tr.end) triple(it + 1, BufTag<1>{});
    }
    // ---- add the target's block to the FP64 output (each element owned by one lane)
    const int wl = opaque_int(lane);        // offsets recomputed here, not held
    const int gg = wl >> 4, rr = wl & 15;
#pragma unroll
    for (int e = 0; e < TMAX; ++e) {
      if (e < tw) {
        const int q = 16 * (tw0 + e) + rr, bp = q / N, cp = q % N;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          size_t off[4];
          double o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int ap = min(16 * mt + 4 * gg + i, N - 1);
            const int child = ((ap / K) << 2) | ((bp / K) << 1) | (cp / K);
            off[i] = (size_t)(tr.fc + child) * K3 + ((ap % K) * K + (bp % K)) * K + (cp % K);
            o[i] = out[off[i]];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (16 * mt + 4 * gg + i < N) out[off[i]] = o[i] + (double)acc[e][mt][i];
        }
      }
    }
  }
}

}  // namespace

// ----------------------------------------------------------------------------- launchers
#define MRA_DISPATCH_K(k, ...)                                         \
  switch (k) {                                                          \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;                      \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;                      \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;                      \
    case 5: { constexpr int KK = 5; __VA_ARGS__; } break;                      \
    case 6: { constexpr int KK = 6; __VA_ARGS__; } break;                      \
    case 7: { constexpr int KK = 7; __VA_ARGS__; } break;                      \
    case 8: { constexpr int KK = 8; __VA_ARGS__; } break;                      \
    case 9: { constexpr int KK = 9; __VA_ARGS__; } break;                      \
    case 10: { constexpr int KK = 10; __VA_ARGS__; } break;                    \
    default: fail(MRA_E_UNSUPPORTED, "wavelet order not compiled in this kernel"); \
  }

#define MRA_DISPATCH_K14(k, ...)                                       \
  switch (k) {                                                          \
    case 11: { constexpr int KK = 11; __VA_ARGS__; } break;                    \
    case 12: { constexpr int KK = 12; __VA_ARGS__; } break;                    \
    case 13: { constexpr int KK = 13; __VA_ARGS__; } break;                    \
    case 14: { constexpr int KK = 14; __VA_ARGS__; } break;                    \
    default: MRA_DISPATCH_K(k, __VA_ARGS__);                                   \
  }

void launch_zero_batch(double* const* tab, const int64_t* len, int count, size_t maxlen,
                       hipStream_t s) {
  if (count <= 0 || maxlen == 0) return;
  const int blocks = (int)std::min<size_t>((maxlen + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_batch_kernel, dim3(blocks, count), dim3(256), 0, s, tab, len);
  hip_check(hipGetLastError(), "zero_batch_kernel");
}

void launch_zero(double* p, size_t n, hipStream_t s) {
  if (!n) return;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, p, n);
  hip_check(hipGetLastError(), "zero_kernel");
}

void launch_filter_up(int k, double* const* coeff_tab, const NodeRef* refs, int count,
                      const double* h0, const double* h1, double* bnorm2, uint16_t* mirror,
                      hipStream_t s) {
  if (count <= 0) return;
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(filter_up_kernel<KK>, dim3(count), dim3(256), 0, s,
                                         coeff_tab, refs, h0, h1, bnorm2, mirror));
  hip_check(hipGetLastError(), "filter_up_kernel");
}

bool low_kernel_available(int k) { return k == 10 || k == 12 || k == 14; }

static int device_cus();

void launch_apply_low(int k, const uint16_t* mirror, double* const* out_tab,
                      const LowItem* items, const TargetRange* targets, int ntargets,
                      const uint16_t* const* l_tab, const double* const* c_tab, int* counter,
                      hipStream_t s) {
  if (ntargets <= 0) return;
  // one persistent workgroup per CU (the kernel's LDS allows one), ranges from a counter
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, s, counter, 1, 0);
  const int grid = std::min(ntargets, device_cus());
  if (k == 10) {
    hipLaunchKernelGGL(apply_low_kernel<10>, dim3(grid), dim3(64 * kLowWaves), 0, s, mirror, out_tab,
                       items, targets, l_tab, c_tab, ntargets, counter);
  } else if (k == 12) {
    hipLaunchKernelGGL(apply_low_kernel<12>, dim3(grid), dim3(64 * kLowWaves), 0, s, mirror, out_tab,
                       items, targets, l_tab, c_tab, ntargets, counter);
  } else if (k == 14) {
    hipLaunchKernelGGL(apply_low_kernel<14>, dim3(grid), dim3(64 * kLowWaves), 0, s, mirror, out_tab,
                       items, targets, l_tab, c_tab, ntargets, counter);
  } else {
    fail(MRA_E_UNSUPPORTED, "the low-precision tier is built for k = 10, 12, 14");
  }
  hip_check(hipGetLastError(), "apply_low_kernel");
}

bool ns_kernel_fuses_subtraction(int k) { return k == 8 || k == 10 || k == 12 || k == 14; }

bool ns_kernel_factored(int k) { return k == 10; }

// Compute units of the current device (cached per device).
static int device_cus() {
  static int cus[64] = {};
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) fail(MRA_E_DEVICE, "device index out of range");
  if (cus[dev] <= 0) {
    int n = 0;
    hip_check(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev),
              "hipDeviceGetAttribute");
    cus[dev] = std::max(1, n);
  }
  return cus[dev];
}

bool ns_uses_slab_mirror(int k) { return k == 14; }

void launch_slab_mirror(int k, double* const* coeff_tab, const NodeRef* refs, int count,
                        double* slabs, hipStream_t s) {
  if (count <= 0) return;
  if (k != 14) fail(MRA_E_UNSUPPORTED, "slab-ordered children blocks are built for k = 14");
  hipLaunchKernelGGL(slab_mirror_kernel<14>, dim3(count), dim3(256), 0, s, coeff_tab, refs, slabs);
  hip_check(hipGetLastError(), "slab_mirror_kernel");
}

void launch_apply_ns(int k, const double* const* in_tab, double* const* out_tab,
                     const NSItem* items, const TargetRange* targets, int ntargets,
                     const double* const* r_tab, const double* const* t_tab,
                     const double* const* c_tab, double* partials, double* subbuf,
                     int* counter, hipStream_t s, const double* slabs) {
  if (ntargets <= 0) return;
  if (k == 8) {
    hipLaunchKernelGGL(apply_ns_mfma_kernel<8>, dim3(ntargets), dim3(256), 0, s, in_tab,
                       out_tab, items, targets, r_tab, t_tab, c_tab, partials, subbuf);
  } else if (k == 10) {
    // one persistent workgroup per CU (the kernel's LDS allows one), ranges from a counter
    // (one for each of the two kernels, both cleared here)
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, s, counter, 2, 0);
    hipLaunchKernelGGL(apply_ns_fac_kernel<10>, dim3(std::min(ntargets, device_cus())), dim3(256),
                       0, s, in_tab, out_tab, items, targets, r_tab, t_tab, c_tab, partials,
                       subbuf, ntargets, counter);
    hip_check(hipGetLastError(), "apply_ns_fac_kernel");
    // one persistent workgroup per CU (the kernel's LDS allows one), target ranges from the
    // second counter
    hipLaunchKernelGGL(apply_ns_fac_sub_kernel<10>, dim3(std::min(ntargets, device_cus())),
                       dim3(256), 0, s, in_tab, items, targets, t_tab, c_tab, partials, subbuf,
                       ntargets, counter + 1);
  } else if (k == 12) {
    hipLaunchKernelGGL(apply_ns_own_kernel<12>, dim3(ntargets), dim3(256), 0, s, in_tab,
                       out_tab, items, targets, r_tab, t_tab, c_tab, partials, subbuf);
  } else if (k == 14) {
    // one persistent workgroup per CU (the kernel's LDS allows one), ranges from a counter
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, s, counter, 1, 0);
    if (!slabs) fail(MRA_E_INVALID, "k = 14 apply: the slab-ordered children blocks are missing");
    hipLaunchKernelGGL(apply_ns_stream_kernel<14>, dim3(std::min(ntargets, device_cus())),
                       dim3(512), 0, s, in_tab, out_tab, items, targets, r_tab, t_tab, c_tab,
                       partials, subbuf, ntargets, counter, slabs);
  } else {
    MRA_DISPATCH_K(k, hipLaunchKernelGGL(apply_ns_kernel<KK>, dim3(ntargets),
                                         dim3(round64(4 * KK * KK)), 0, s, in_tab, out_tab,
                                         items, targets, r_tab, c_tab, partials));
  }
  hip_check(hipGetLastError(), "apply_ns_kernel");
}

void launch_reduce_partials(int k, const double* partials, double* const* out_tab,
                            double* subbuf, const SplitTarget* splits, int nsplits,
                            hipStream_t s) {
  if (nsplits <= 0) return;
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(reduce_partials_kernel<KK>, dim3(nsplits, 8), dim3(256),
                                         0, s, partials, out_tab, subbuf, splits));
  hip_check(hipGetLastError(), "reduce_partials_kernel");
}

void launch_apply_std(int k, const double* const* in_tab, double* const* out_tab,
                      const NSItem* items, const TargetRange* targets, int ntargets,
                      const double* const* t_tab, const double* const* c_tab, double scale,
                      hipStream_t s, int t_lds) {
  if (ntargets <= 0) return;
  if (k == 8) {
    // matrix-core kernel: one wave per target, four per workgroup; the t table of a
    // single-function launch in LDS when it fits in 32 KB
    if (t_lds > 0 && t_lds <= 4096) {
      hipLaunchKernelGGL((apply_std_mfma_kernel<8, true>), dim3((ntargets + 3) / 4), dim3(256),
                         (size_t)t_lds * sizeof(double), s, in_tab, out_tab, items, targets,
                         ntargets, t_tab, c_tab, scale, t_lds);
    } else {
      hipLaunchKernelGGL((apply_std_mfma_kernel<8, false>), dim3((ntargets + 3) / 4), dim3(256), 0,
                         s, in_tab, out_tab, items, targets, ntargets, t_tab, c_tab, scale, 0);
    }
    hip_check(hipGetLastError(), "apply_std_mfma_kernel");
    return;
  }
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(apply_std_kernel<KK>, dim3(ntargets),
                                         dim3(round64(KK * KK)), 0, s, in_tab, out_tab, items,
                                         targets, t_tab, c_tab, scale));
  hip_check(hipGetLastError(), "apply_std_kernel");
}

void launch_sum_down(int k, double* const* coeff_tab, const NodeRef* refs, int count,
                     const double* subbuf, const double* h0, const double* h1, hipStream_t s,
                     double sign) {
  if (count <= 0) return;
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(sum_down_kernel<KK>, dim3(count), dim3(512), 0, s,
                                         coeff_tab, refs, subbuf, h0, h1, sign));
  hip_check(hipGetLastError(), "sum_down_kernel");
}

void launch_child_norm2(int k, const double* coeff, const int32_t* fchild, int count,
                        double* out, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(child_norm2_kernel, dim3(count), dim3(256), 0, s, k * k * k, coeff, fchild,
                     out);
  hip_check(hipGetLastError(), "child_norm2_kernel");
}

void launch_copy_slabs(int k, double* dst, const int32_t* to, const double* src,
                       const int32_t* from, int count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(copy_slabs_kernel, dim3(count), dim3(256), 0, s, k * k * k, dst, to, src,
                     from);
  hip_check(hipGetLastError(), "copy_slabs_kernel");
}

void launch_gauss1d(int k, const double* gpar, int ng, const int64_t* lvals, int nl, int off1,
                    int off2, int n, double lo, double W, const double* glx, const double* glw,
                    int nq, const double* h0, const double* h1, double* T, uint8_t* nz,
                    hipStream_t s) {
  const int64_t rows = (int64_t)nl * ng;
  if (rows <= 0) return;
  if ((rows + 63) / 64 > INT32_MAX) fail(MRA_E_UNSUPPORTED, "projection level too large");
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(gauss1d_kernel<KK>, dim3((unsigned)((rows + 63) / 64)),
                                         dim3(64), 0, s, gpar, ng, lvals, nl, off1, off2, n, lo,
                                         W, glx, glw, nq, h0, h1, T, nz));
  hip_check(hipGetLastError(), "gauss1d_kernel");
}

void launch_project_level(int k, const double* T, const uint8_t* nz, const int32_t* boxu,
                          int nbox, int ng, const double* gpar, int test, double* d2,
                          double* S, hipStream_t s) {
  if (nbox <= 0) return;
  const int threads = round64(std::max(4 * k * k, 64));
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(project_level_kernel<KK>, dim3(nbox), dim3(threads),
                                         (size_t)ng * sizeof(int), s, T, nz, boxu, ng, gpar,
                                         test, d2, S));
  hip_check(hipGetLastError(), "project_level_kernel");
}

// ---------------------------------------------------------- norm2 without device allocation
// mra_norm2_noalloc runs the reduction of mra_norm2 (leaf_reduce_kernel, 2048 workgroup
// partials) with its partials and their ordered sum in a file-scope device array instead
// of memory from the context's allocator.  Each GPU holds its own copy of the array, at its
// own address, until the process ends; host code uses only that address (obtained once per
// device with hipGetSymbolAddress), never the array's name.  Every workgroup writes its
// partial, so nothing has to be cleared between calls; calls that overlap on one GPU (two
// streams at once) race on the array.
namespace {
constexpr int kScratchParts = 2048;                    // fixed reduction grid
constexpr int kScratchDoubles = kScratchParts + 32;    // partials, then the ordered sum
static __device__ __align__(256) double scratch[kScratchDoubles];

// Sums p[0 .. n) in index order (the order of the host sum of mra_norm2) into *out.
__global__ void ordered_sum_kernel(const double* __restrict__ p, int n, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += p[i];
  *out = s;
}

std::mutex g_scratch_mutex;
double* g_scratch_addr[64] = {};
}  // namespace

double* static_scratch_init(int device) {
  if (device < 0 || device >= 64) fail(MRA_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[device]) {
    int cur = -1;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (cur != device) hip_check(hipSetDevice(device), "hipSetDevice");
    double* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (cur != device) hip_check(hipSetDevice(cur), "hipSetDevice");
    hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) fail(MRA_E_DEVICE, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_addr[device] = ptr;
  }
  return g_scratch_addr[device];
}

double norm2_noalloc(int device, int k, const double* coeff, const int32_t* leaves_dev,
                     int64_t count, hipStream_t s) {
  static_assert(kScratchParts + 1 <= kScratchDoubles, "partials and their sum fit");
  if (k < 2 || k > kMaxK) fail(MRA_E_INVALID, "mra_norm2_noalloc: k must be in [2, 14]");
  if (count <= 0) return 0.0;
  if (count > INT32_MAX) fail(MRA_E_INVALID, "mra_norm2_noalloc: more than 2^31 - 1 leaves");
  if (!leaves_dev || !coeff) fail(MRA_E_INVALID, "mra_norm2_noalloc: function not resident");
  double* base = static_scratch_init(device);
  hipLaunchKernelGGL(leaf_reduce_kernel, dim3(kScratchParts), dim3(256), 0, s, k * k * k, coeff,
                     nullptr, leaves_dev, nullptr, nullptr, (int)count, 0, base);
  hip_check(hipGetLastError(), "leaf_reduce_kernel");
  hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(64), 0, s, base, kScratchParts,
                     base + kScratchParts);
  hip_check(hipGetLastError(), "ordered_sum_kernel");
  double sum = 0.0;
  hip_check(hipMemcpyAsync(&sum, base + kScratchParts, sizeof(double), hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync D2H");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  return sum;
}

void launch_leaf_reduce(int k, const double* a, const double* b, const int32_t* leaves_a,
                        const int32_t* leaves_b, const double* weight, int count, int mode,
                        double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(leaf_reduce_kernel, dim3(nblocks), dim3(256), 0, s, k * k * k, a, b,
                     leaves_a, leaves_b, weight, count, mode, partial);
  hip_check(hipGetLastError(), "leaf_reduce_kernel");
}

}  // namespace mra
