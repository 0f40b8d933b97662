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

#include "mra_internal.hpp"

namespace mra {

namespace {

constexpr int round64(int x) { return (x + 63) / 64 * 64; }

__global__ void zero_kernel(double* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

// --------------------------------------------------------------------------- filter-up
template <int K>
__global__ __launch_bounds__(round64(4 * K * K)) void filter_up_kernel(
    const double* __restrict__ in, double* __restrict__ out, const int32_t* __restrict__ nodes,
    const int32_t* __restrict__ fchild, const double* __restrict__ h0,
    const double* __restrict__ h1, double* __restrict__ bnorm2) {
  constexpr int N = 2 * K, K3 = K * K * K, ZP = N + 1;
  __shared__ double B[N * N * ZP];
  __shared__ double T[K * N * ZP];
  __shared__ double H[K * N];
  __shared__ double red[round64(4 * K * K)];
  const int tid = threadIdx.x;
  const int node = nodes[blockIdx.x];
  const int fc = fchild[blockIdx.x];
  for (int e = tid; e < K * N; e += blockDim.x) {
    int i = e / N, X = e % N;
    H[e] = X < K ? h0[i * K + X] : h1[i * K + X - K];
  }
  double sq = 0.0;
  for (int e = tid; e < 8 * K3; e += blockDim.x) {
    int c = e / K3, r = e - c * K3;
    int i = r / (K * K), j = (r / K) % K, m = r % K;
    double v = in[(size_t)(fc + c) * K3 + r];
    sq += v * v;
    B[((((c >> 2) & 1) * K + i) * N + ((c >> 1) & 1) * K + j) * ZP + (c & 1) * K + m] = v;
  }
  red[tid] = sq;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {  // fixed-order tree; blockDim need not be a power of 2
    if (tid < s && tid + s < (int)blockDim.x) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) bnorm2[blockIdx.x] = red[0];
  // phase x: thread (Y, Z): T[i][Y][Z] = sum_X H[i][X] B[X][Y][Z]
  if (tid < N * N) {
    int Y = tid / N, Z = tid % N;
    double t[K];
#pragma unroll
    for (int i = 0; i < K; ++i) t[i] = 0.0;
    for (int X = 0; X < N; ++X) {
      double v = B[(X * N + Y) * ZP + Z];
#pragma unroll
      for (int i = 0; i < K; ++i) t[i] += H[i * N + X] * v;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) T[(i * N + Y) * ZP + Z] = t[i];
  }
  __syncthreads();
  // phase y: thread (i, Z): B[i][j][Z] (reuse B as K x K x N) = sum_Y H[j][Y] T[i][Y][Z]
  if (tid < K * N) {
    int i = tid / N, Z = tid % N;
    double t[K];
#pragma unroll
    for (int j = 0; j < K; ++j) t[j] = 0.0;
    for (int Y = 0; Y < N; ++Y) {
      double v = T[(i * N + Y) * ZP + Z];
#pragma unroll
      for (int j = 0; j < K; ++j) t[j] += H[j * N + Y] * v;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) B[(i * K + j) * ZP + Z] = t[j];
  }
  __syncthreads();
  // phase z: thread (i, j): s[i][j][m] = sum_Z H[m][Z] B[i][j][Z]
  if (tid < K * K) {
    int i = tid / K, j = tid % K;
    double t[K];
#pragma unroll
    for (int m = 0; m < K; ++m) t[m] = 0.0;
    for (int Z = 0; Z < N; ++Z) {
      double v = B[(i * K + j) * ZP + Z];
#pragma unroll
      for (int m = 0; m < K; ++m) t[m] += H[m * N + Z] * v;
    }
#pragma unroll
    for (int m = 0; m < K; ++m) out[(size_t)node * K3 + (i * K + j) * K + m] = t[m];
  }
}

// --------------------------------------------------------------------------- apply (NS)
template <int K>
__global__ __launch_bounds__(round64(4 * K * K)) void apply_ns_kernel(
    const double* __restrict__ in, double* __restrict__ out, const NSItem* __restrict__ items,
    const TargetRange* __restrict__ targets, const double* __restrict__ dR,
    const double* __restrict__ dc) {
  constexpr int N = 2 * K, N2 = N * N, K3 = K * K * K, ZP = N + 1;
  __shared__ double S[N * N * ZP];
  __shared__ double W[N * N * ZP];
  const int tid = threadIdx.x;
  const TargetRange tr = targets[blockIdx.x];
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
    const double* RX = dR + (size_t)item.rx * N2;
    const double* RY = dR + (size_t)item.ry * N2;
    const double* RZ = dR + (size_t)item.rz * N2;
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
#pragma unroll
    for (int c = 0; c < N; ++c) {
      int child = (ca << 2) | (cb << 1) | (c / K);
      size_t idx = (size_t)(tr.fc + child) * K3 + (i * K + j) * K + (c % K);
      out[idx] += acc[c];
    }
  }
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
// triples of the target.
template <int K>
__global__ __launch_bounds__(256) void apply_ns_mfma_kernel(
    const double* __restrict__ in, double* __restrict__ out, const NSItem* __restrict__ items,
    const TargetRange* __restrict__ targets, const double* __restrict__ dR,
    const double* __restrict__ dc) {
  constexpr int N = 2 * K, Q = N / 4, N2 = N * N, K3 = K * K * K, ZP = N + 1;
  static_assert(N % 4 == 0, "k must be even");
  static_assert(Q >= 4 && Q <= 5, "register budget sized for 2k = 16 or 20");
  constexpr int EXTRA = (Q - 4) * Q;                 // (z-quad >= 4) pairs, round robin
  constexpr int EXTRA_PER_WAVE = (EXTRA + 3) / 4;
  constexpr int P3 = Q * Q;                          // step-3 (a-quad, b-quad) pairs
  constexpr int P3_PER_WAVE = (P3 + 3) / 4;
  __shared__ double Xs[N * N * ZP];
  __shared__ double Zs[N * N * ZP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 3, lb = (lane >> 2) & 3, lk = lane >> 4;
  const TargetRange tr = targets[blockIdx.x];

  double acc[P3_PER_WAVE][Q];
#pragma unroll
  for (int p = 0; p < P3_PER_WAVE; ++p)
#pragma unroll
    for (int c = 0; c < Q; ++c) acc[p][c] = 0.0;

  int loaded = -1;
  for (int it = tr.beg; it < tr.end; ++it) {
    const NSItem item = items[it];
    if (item.src_fc != loaded) {
      __syncthreads();
      for (int e = tid; e < 8 * K3; e += 256) {
        int c = e / K3, r = e - c * K3;
        int i = r / (K * K), j = (r / K) % K, m = r % K;
        Xs[((((c >> 2) & 1) * K + i) * N + ((c >> 1) & 1) * K + j) * ZP + (c & 1) * K + m] =
            in[(size_t)(item.src_fc + c) * K3 + r];
      }
      loaded = item.src_fc;
      __syncthreads();
    }
    const double* RX = dR + (size_t)item.rx * N2;   // transposed: RX[x*N + a] = R[a][x]
    const double* RY = dR + (size_t)item.ry * N2;
    const double* RZ = dR + (size_t)item.rz * N2;
    const double cmu = dc[item.mu];
    // B fragments: frag(ks, t) = R[4t + li][4ks + lk]
    double rx[Q][Q], ry[Q][Q];
#pragma unroll
    for (int ks = 0; ks < Q; ++ks)
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        rx[ks][t] = RX[(4 * ks + lk) * N + 4 * t + li];
        ry[ks][t] = RY[(4 * ks + lk) * N + 4 * t + li];
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
          double a = Xs[((4 * xs + lk) * N + 4 * yt + li) * ZP + 4 * zq + lb];
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
          Zs[((4 * at + lk) * N + 4 * bt + li) * ZP + 4 * zq + lb] = d2[bt];
      }
    }
    // ---- leftover (z-quad >= 4) pairs, round robin over the waves
#pragma unroll
    for (int e = 0; e < EXTRA_PER_WAVE; ++e) {
      const int p = wave + 4 * e;
      if (p < EXTRA) {
        const int zq = 4 + p / Q, at = p % Q;
        double d1[Q];
#pragma unroll
        for (int yt = 0; yt < Q; ++yt) d1[yt] = 0.0;
#pragma unroll
        for (int xs = 0; xs < Q; ++xs)
#pragma unroll
          for (int yt = 0; yt < Q; ++yt) {
            double a = Xs[((4 * xs + lk) * N + 4 * yt + li) * ZP + 4 * zq + lb];
            double b = 0.0;
#pragma unroll
            for (int t = 0; t < Q; ++t)
              if (t == at) b = rx[xs][t];
            d1[yt] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, d1[yt], 0, 0, 0);
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
          Zs[((4 * at + lk) * N + 4 * bt + li) * ZP + 4 * zq + lb] = d2[bt];
      }
    }
    __syncthreads();
    // ---- step 3: z-contraction into the register accumulators
    double rz[Q][Q];
#pragma unroll
    for (int ks = 0; ks < Q; ++ks)
#pragma unroll
      for (int t = 0; t < Q; ++t) rz[ks][t] = cmu * RZ[(4 * ks + lk) * N + 4 * t + li];
#pragma unroll
    for (int e = 0; e < P3_PER_WAVE; ++e) {
      const int p = (3 - wave) + 4 * e;
      if (p < P3) {
        const int at3 = p / Q, bt3 = p % Q;
#pragma unroll
        for (int zs = 0; zs < Q; ++zs) {
          double a = Zs[((4 * at3 + lb) * N + 4 * bt3 + li) * ZP + 4 * zs + lk];
#pragma unroll
          for (int ct = 0; ct < Q; ++ct)
            acc[e][ct] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, rz[zs][ct], acc[e][ct], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // ---- write the children block of the target
#pragma unroll
  for (int e = 0; e < P3_PER_WAVE; ++e) {
    const int p = (3 - wave) + 4 * e;
    if (p < P3) {
      const int at3 = p / Q, bt3 = p % Q;
      const int a = 4 * at3 + lb, b = 4 * bt3 + lk;
#pragma unroll
      for (int ct = 0; ct < Q; ++ct) {
        const int c = 4 * ct + li;
        const int child = ((a / K) << 2) | ((b / K) << 1) | (c / K);
        out[(size_t)(tr.fc + child) * K3 + ((a % K) * K + (b % K)) * K + (c % K)] += acc[e][ct];
      }
    }
  }
}

// --------------------------------------------------------------------------- apply (std)
template <int K>
__global__ __launch_bounds__(round64(K * K)) void apply_std_kernel(
    const double* __restrict__ in, double* __restrict__ out, const NSItem* __restrict__ items,
    const TargetRange* __restrict__ targets, const double* __restrict__ dT,
    const double* __restrict__ dc, double scale) {
  constexpr int K2 = K * K, K3 = K * K * K, ZP = K + 1;
  __shared__ double S[K * K * ZP];
  __shared__ double W[K * K * ZP];
  const int tid = threadIdx.x;
  const TargetRange tr = targets[blockIdx.x];
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
    const double* TX = dT + (size_t)item.tx * K2;
    const double* TY = dT + (size_t)item.ty * K2;
    const double* TZ = dT + (size_t)item.tz * K2;
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

// --------------------------------------------------------------------------- sum-down
template <int K>
__global__ __launch_bounds__(round64(4 * K * K)) void sum_down_kernel(
    double* __restrict__ coeff, const int32_t* __restrict__ nodes,
    const int32_t* __restrict__ fchild, const double* __restrict__ h0,
    const double* __restrict__ h1) {
  constexpr int N = 2 * K, K3 = K * K * K, ZP = N + 1;
  __shared__ double V[K3];
  __shared__ double T1[K * K * ZP];
  __shared__ double T2[K * N * ZP];
  __shared__ double H[K * N];
  const int tid = threadIdx.x;
  const int node = nodes[blockIdx.x];
  const int fc = fchild[blockIdx.x];
  for (int e = tid; e < K * N; e += blockDim.x) {
    int i = e / N, X = e % N;
    H[e] = X < K ? h0[i * K + X] : h1[i * K + X - K];
  }
  for (int e = tid; e < K3; e += blockDim.x) V[e] = coeff[(size_t)node * K3 + e];
  __syncthreads();
  if (tid < K * K) {  // T1[i][j][Z] = sum_m H[m][Z] V[i][j][m]
    int i = tid / K, j = tid % K;
    double t[N];
#pragma unroll
    for (int Z = 0; Z < N; ++Z) t[Z] = 0.0;
    for (int m = 0; m < K; ++m) {
      double v = V[(i * K + j) * K + m];
#pragma unroll
      for (int Z = 0; Z < N; ++Z) t[Z] += H[m * N + Z] * v;
    }
#pragma unroll
    for (int Z = 0; Z < N; ++Z) T1[(i * K + j) * ZP + Z] = t[Z];
  }
  __syncthreads();
  if (tid < K * N) {  // T2[i][Y][Z] = sum_j H[j][Y] T1[i][j][Z]
    int i = tid / N, Z = tid % N;
    double t[N];
#pragma unroll
    for (int Y = 0; Y < N; ++Y) t[Y] = 0.0;
    for (int j = 0; j < K; ++j) {
      double v = T1[(i * K + j) * ZP + Z];
#pragma unroll
      for (int Y = 0; Y < N; ++Y) t[Y] += H[j * N + Y] * v;
    }
#pragma unroll
    for (int Y = 0; Y < N; ++Y) T2[(i * N + Y) * ZP + Z] = t[Y];
  }
  __syncthreads();
  if (tid < N * N) {  // child[X][Y][Z] += sum_i H[i][X] T2[i][Y][Z]
    int Y = tid / N, Z = tid % N;
    double t[N];
#pragma unroll
    for (int X = 0; X < N; ++X) t[X] = 0.0;
    for (int i = 0; i < K; ++i) {
      double v = T2[(i * N + Y) * ZP + Z];
#pragma unroll
      for (int X = 0; X < N; ++X) t[X] += H[i * N + X] * v;
    }
    int cy = Y / K, j = Y % K, cz = Z / K, m = Z % K;
#pragma unroll
    for (int X = 0; X < N; ++X) {
      int child = ((X / K) << 2) | (cy << 1) | cz;
      coeff[(size_t)(fc + child) * K3 + ((X % K) * K + j) * K + m] += t[X];
    }
  }
}

// --------------------------------------------------------------------------- reductions
// mode 0: sum ||a_leaf||^2; mode 1: sum a_leaf[0] * weight[leaf]; mode 2: sum <a_la, b_lb>
__global__ __launch_bounds__(256) void leaf_reduce_kernel(
    int k3, const double* __restrict__ a, const double* __restrict__ b,
    const int32_t* __restrict__ la, const int32_t* __restrict__ lb,
    const double* __restrict__ weight, int count, int mode, double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int l = blockIdx.x; l < count; l += gridDim.x) {
    const double* pa = a + (size_t)la[l] * k3;
    if (mode == 0) {
      for (int e = threadIdx.x; e < k3; e += blockDim.x) s += pa[e] * pa[e];
    } else if (mode == 1) {
      if (threadIdx.x == 0) s += pa[0] * weight[l];
    } else {
      const double* pb = b + (size_t)lb[l] * k3;
      for (int e = threadIdx.x; e < k3; e += blockDim.x) s += pa[e] * pb[e];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
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

void launch_zero(double* p, size_t n, hipStream_t s) {
  if (!n) return;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, p, n);
  hip_check(hipGetLastError(), "zero_kernel");
}

void launch_filter_up(int k, const double* coeff, double* coeff_out, const int32_t* nodes,
                      const int32_t* fchild, int count, const double* h0, const double* h1,
                      double* bnorm2, hipStream_t s) {
  if (count <= 0) return;
  MRA_DISPATCH_K(k, hipLaunchKernelGGL(filter_up_kernel<KK>, dim3(count),
                                       dim3(round64(4 * KK * KK)), 0, s, coeff, coeff_out, nodes,
                                       fchild, h0, h1, bnorm2));
  hip_check(hipGetLastError(), "filter_up_kernel");
}

void launch_apply_ns(int k, const double* in_coeff, double* out_coeff, const NSItem* items,
                     const TargetRange* targets, int ntargets, const double* dR,
                     const double* dc, hipStream_t s) {
  if (ntargets <= 0) return;
  if (k == 8) {
    hipLaunchKernelGGL(apply_ns_mfma_kernel<8>, dim3(ntargets), dim3(256), 0, s, in_coeff,
                       out_coeff, items, targets, dR, dc);
  } else if (k == 10) {
    hipLaunchKernelGGL(apply_ns_mfma_kernel<10>, dim3(ntargets), dim3(256), 0, s, in_coeff,
                       out_coeff, items, targets, dR, dc);
  } else {
    MRA_DISPATCH_K(k, hipLaunchKernelGGL(apply_ns_kernel<KK>, dim3(ntargets),
                                         dim3(round64(4 * KK * KK)), 0, s, in_coeff, out_coeff,
                                         items, targets, dR, dc));
  }
  hip_check(hipGetLastError(), "apply_ns_kernel");
}

void launch_apply_std(int k, const double* in_coeff, double* out_coeff, const NSItem* items,
                      const TargetRange* targets, int ntargets, const double* dT,
                      const double* dc, double scale, hipStream_t s) {
  if (ntargets <= 0) return;
  MRA_DISPATCH_K14(k, hipLaunchKernelGGL(apply_std_kernel<KK>, dim3(ntargets),
                                         dim3(round64(KK * KK)), 0, s, in_coeff, out_coeff,
                                         items, targets, dT, dc, scale));
  hip_check(hipGetLastError(), "apply_std_kernel");
}

void launch_sum_down(int k, double* coeff, const int32_t* nodes, const int32_t* fchild,
                     int count, const double* h0, const double* h1, hipStream_t s) {
  if (count <= 0) return;
  MRA_DISPATCH_K(k, hipLaunchKernelGGL(sum_down_kernel<KK>, dim3(count),
                                       dim3(round64(4 * KK * KK)), 0, s, coeff, nodes, fchild,
                                       h0, h1));
  hip_check(hipGetLastError(), "sum_down_kernel");
}

void launch_leaf_reduce(int k, const double* a, const double* b, const int32_t* leaves_a,
                        const int32_t* leaves_b, const double* weight, int count, int mode,
                        double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(leaf_reduce_kernel, dim3(nblocks), dim3(256), 0, s, k * k * k, a, b,
                     leaves_a, leaves_b, weight, count, mode, partial);
  hip_check(hipGetLastError(), "leaf_reduce_kernel");
}

}  // namespace mra
