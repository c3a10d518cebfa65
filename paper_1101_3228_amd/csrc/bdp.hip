// Backward dynamic programming on the quantization tree (Sec. 2), FP64:
//   V_n = phi_n,  V_k(i) = max(phi_k(i), sum_j c_ij V_{k+1}(j) / p_i),
// with pi^k_ij = c_ij / p_i estimated by the forward counts.  The
// conditional expectation on the tree is the row reduction
// sum_j pi_ij f(x_j) of Sec. 2.  One 64-lane wave reduces one row of the
// count block for up to kPay obstacle vectors at once, so the int32 counts
// are read from HBM once per group of payoffs.  Also the obstacle phi_k on
// the grid points.
#include "qtree_batch.hpp"
#include "qtree_internal.hpp"

namespace qtree {

namespace {
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kPay = 16;
constexpr int kRowUnroll = 8;
constexpr int kFewPay = 2;  // payoffs per pass whose V entries are loaded with the counts
constexpr int kFewUnroll = 16;  // ... and the row loads in flight per lane then

// One wave's share of a count row (len entries from row) against nq <= kPay
// value vectors V + (q0 + q) P + col0: the row total p and the sums
// s_q = sum_j c_j V_q(j) of this lane's columns.  kRowUnroll row loads are
// in flight per lane (a long dense row is otherwise one HBM round trip per
// 64 columns); a column whose count is zero adds nothing, and its V entries
// are not read.
template <bool FEW>
__device__ __forceinline__ void row_sums(const int32_t* __restrict__ row, int len,
                                         const double* __restrict__ V, int64_t P, int q0,
                                         int nq, int64_t col0, int lane, int64_t& p,
                                         double (&s)[kPay]) {
  p = 0;
#pragma unroll
  for (int q = 0; q < kPay; ++q) s[q] = 0.0;
  if (FEW && nq <= kFewPay) {
    // few payoffs: the V entries are loaded with the counts, not after them
    // (a load that waits on its count is a second round trip per group);
    // a zero count still adds nothing (a select, not a multiply by zero)
    for (int j0 = lane; j0 < len; j0 += 64 * kFewUnroll) {
      int32_t c[kFewUnroll];
      double v[kFewUnroll][kFewPay];
#pragma unroll
      for (int u = 0; u < kFewUnroll; ++u) {
        const int j = j0 + 64 * u;
        c[u] = j < len ? row[j] : 0;
#pragma unroll
        for (int q = 0; q < kFewPay; ++q)
          v[u][q] = (j < len && q < nq) ? V[(int64_t)(q0 + q) * P + col0 + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kFewUnroll; ++u) {
        p += c[u];
        const double cd = (double)c[u];
#pragma unroll
        for (int q = 0; q < kFewPay; ++q) s[q] = c[u] != 0 ? fma(cd, v[u][q], s[q]) : s[q];
      }
    }
    return;
  }
  for (int j0 = lane; j0 < len; j0 += 64 * kRowUnroll) {
    int32_t c[kRowUnroll];
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) {
      const int j = j0 + 64 * u;
      c[u] = j < len ? row[j] : 0;
    }
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) {
      p += c[u];
      if (c[u] != 0) {
        const double cd = (double)c[u];
        const int64_t col = col0 + j0 + 64 * u;
#pragma unroll
        for (int q = 0; q < kPay; ++q)
          if (q < nq) s[q] = fma(cd, V[(int64_t)(q0 + q) * P + col], s[q]);
      }
    }
  }
}
}  // namespace

// One layer for every payoff: blockIdx.y selects the group of kPay payoffs
// (the count row is re-read per group, from L2 for all but the first).
// FEW: the instance for at most kFewPay payoffs.  The general instance does
// not carry the few-payoff path's registers (98 VGPRs against 119): its
// workgroups, launched beside a sampling pass on another stream, then find
// room on the CUs sooner (the 1-D workload's pipelined step: 1.86 against
// 2.14-2.19 ms with one instance for both).
template <bool FEW>
__global__ __launch_bounds__(kBlock) void bdp_layer_kernel(BdpArgs a, int N_k, int N_k1,
                                                           int64_t pt_k, int64_t pt_k1,
                                                           int64_t cnt_k) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (i >= N_k) return;
  const int q0 = blockIdx.y * kPay;
  const int nq = (a.n_pay - q0) < kPay ? (a.n_pay - q0) : kPay;
  // the row's counts: dense, or the band of columns j0 .. j0 + len - 1
  const int32_t* row;
  int len;
  int64_t col0 = pt_k1;
  if (a.band_off) {
    const int64_t r = pt_k + i;
    const int64_t o = a.band_off[r];
    row = a.counts + o;
    len = (int)(a.band_off[r + 1] - o);
    col0 += a.band_lo[r];
  } else {
    row = a.counts + cnt_k + (int64_t)i * N_k1;
    len = N_k1;
  }
  int64_t p;
  double s[kPay];
  row_sums<FEW>(row, len, a.V, a.P, q0, nq, col0, lane, p, s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    p += __shfl_xor(p, off, 64);
#pragma unroll
    for (int q = 0; q < kPay; ++q) s[q] += __shfl_xor(s[q], off, 64);
  }
  if (lane < nq) {
    // lane q finalises payoff q0 + q
    double sq = s[0];
#pragma unroll
    for (int q = 1; q < kPay; ++q)
      if (lane == q) sq = s[q];
    const double cont = p > 0 ? sq / (double)p : 0.0;
    const int64_t at = (int64_t)(q0 + lane) * a.P + pt_k + i;
    const double f = a.phi[at];
    a.V[at] = f > cont ? f : cont;
  }
}

__global__ void copy_last_layer_kernel(BdpArgs a, int64_t pt_n, int N_n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.n_pay * N_n;
  if (t >= total) return;
  const int64_t q = t / N_n, i = t - q * N_n;
  const int64_t at = q * a.P + pt_n + i;
  a.V[at] = a.phi[at];
}

hipError_t launch_bdp_layer(const BdpArgs& a, int k, int N_k, int N_k1, int64_t pt_k,
                            int64_t pt_k1, int64_t cnt_k, hipStream_t s) {
  (void)k;
  const unsigned blocks = (unsigned)((N_k + kWaves - 1) / kWaves);
  const unsigned groups = (unsigned)((a.n_pay + kPay - 1) / kPay);
  if (a.n_pay <= kFewPay)
    hipLaunchKernelGGL(bdp_layer_kernel<true>, dim3(blocks, groups), dim3(kBlock), 0, s, a, N_k,
                       N_k1, pt_k, pt_k1, cnt_k);
  else
    hipLaunchKernelGGL(bdp_layer_kernel<false>, dim3(blocks, groups), dim3(kBlock), 0, s, a, N_k,
                       N_k1, pt_k, pt_k1, cnt_k);
  return hipGetLastError();
}

hipError_t launch_copy_last_layer(const BdpArgs& a, int64_t pt_n, int N_n, hipStream_t s) {
  const int64_t total = (int64_t)a.n_pay * N_n;
  const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(copy_last_layer_kernel, dim3(blocks), dim3(kBlock), 0, s, a, pt_n, N_n);
  return hipGetLastError();
}

// Batched BDP.  The recursion is sequential in k, so it runs as backward
// steps: step j takes layer n - 1 - j of every contract with n > j, its rows
// cut into tasks of up to kBdpTaskRows rows, one wave per row (as
// bdp_layer_kernel) for the job's up to kPay payoffs; a launch boundary
// separates the steps.  Every contract's work is spread over the whole chip
// at every step.
constexpr int kBdpBlock = 64 * kBdpTaskRows;

__global__ void bdp_batch_copy_kernel(const BdpJob* jobs) {
  const BdpJob& J = jobs[blockIdx.y];
  const LayerDev& Ln = as_global(J.layers)[J.n];
  const double* phi = as_global(J.phi);
  double* V = as_global(J.V);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < J.nq * Ln.N; t += gridDim.x * blockDim.x) {
    const int q = t / Ln.N, i = t - q * Ln.N;
    const int64_t at = (int64_t)(J.q0 + q) * J.P + Ln.pt_off + i;
    V[at] = phi[at];
  }
}

__global__ __launch_bounds__(kBdpBlock) void bdp_step_kernel(const BdpJob* jobs,
                                                             const BdpTask* tasks) {
  const BdpTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave >= T.nrows) return;
  const BdpJob& J = jobs[T.job];
  const LayerDev* layers = as_global(J.layers);
  const LayerDev& L = layers[T.k];
  const LayerDev& L1 = layers[T.k + 1];
  double* V = as_global(J.V);
  const int i = T.row0 + wave;
  const int32_t* row = as_global(J.counts) + L.cnt_off + (int64_t)i * L.N1;
  int64_t p;
  double s[kPay];
  row_sums<true>(row, L.N1, V, J.P, J.q0, J.nq, L1.pt_off, lane, p, s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    p += __shfl_xor(p, off, 64);
#pragma unroll
    for (int q = 0; q < kPay; ++q) s[q] += __shfl_xor(s[q], off, 64);
  }
  if (lane < J.nq) {
    double sq = s[0];
#pragma unroll
    for (int q = 1; q < kPay; ++q)
      if (lane == q) sq = s[q];
    const double cont = p > 0 ? sq / (double)p : 0.0;
    const int64_t at = (int64_t)(J.q0 + lane) * J.P + L.pt_off + i;
    const double f = as_global(J.phi)[at];
    V[at] = f > cont ? f : cont;
  }
}

hipError_t launch_bdp_steps(const BdpJob* jobs, int n_jobs, int max_last, const BdpTask* tasks,
                            const int* step_off, int n_steps, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const unsigned cx = (unsigned)((max_last + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(bdp_batch_copy_kernel, dim3(cx < 1 ? 1 : cx, (unsigned)n_jobs), dim3(kBlock),
                     0, s, jobs);
  for (int j = 0; j < n_steps; ++j) {
    const int cnt = step_off[j + 1] - step_off[j];
    if (cnt > 0)
      hipLaunchKernelGGL(bdp_step_kernel, dim3((unsigned)cnt), dim3(kBdpBlock), 0, s, jobs,
                         tasks + step_off[j]);
  }
  return hipGetLastError();
}

// Discounted obstacle phi_k(x) = exp(-r t_k) payoff(S_{t_k}(x)) on every grid
// point, S^a_t(x) = S0 exp((r - sigma_a^2 / 2) t + sigma_a x_a), FP64, for a
// group of contracts (blockIdx.z).
__global__ void payoff_kernel(PayoffArgs a) {
  const int k = blockIdx.y;
  const Contract& C = a.c[blockIdx.z];
  const LayerDev& L = a.layers[k];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.N) return;
  const double t = C.Tm * (double)k / (double)a.n;
  const double disc = exp(-C.r * t);
  const int64_t at = (int64_t)L.pt_off + i;
  const float4 g = a.d == 1 ? make_float4(a.pts1[at], 0.f, 0.f, 0.f) : a.pts[at];
  const float xs[3] = {g.x, g.y, g.z};
  double y[3];
  for (int c = 0; c < a.d; ++c) {
    if (!C.has_mix) {
      y[c] = (double)xs[c];
      continue;
    }
    y[c] = 0.0;
    for (int e = 0; e < a.d; ++e) y[c] += C.mix[c * a.d + e] * (double)xs[e];
  }
  double v;
  if (C.kind & 1) {
    double smax = -__builtin_huge_val();
    for (int c = 0; c < a.d; ++c) {
      const double sc = C.S0 * exp((C.r - 0.5 * C.sigma[c] * C.sigma[c]) * t + C.sigma[c] * y[c]);
      smax = sc > smax ? sc : smax;
    }
    v = disc * fmax(smax - C.K, 0.0);
  } else {
    const double sc =
        C.S0 * exp((C.r - 0.5 * C.sigma[0] * C.sigma[0]) * t + C.sigma[0] * y[0]);
    v = disc * fmax(C.K - sc, 0.0);
  }
  if ((C.kind & 2) && k < a.n) v = -__builtin_huge_val();
  a.phi[(int64_t)blockIdx.z * a.P + at] = v;
}

hipError_t launch_payoff(const PayoffArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.maxN + kBlock - 1) / kBlock), (unsigned)(a.n + 1),
                  (unsigned)a.count);
  hipLaunchKernelGGL(payoff_kernel, grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}


// ------------------------------------------------- many contracts, one tree
//
// The conditional expectation of the quantized BDP (Sec. 2) is a product of
// the transition matrix pi^k (N_k x N_{k+1}) with the values V_{k+1} of every
// contract priced on the tree; its cost is sum_k N_k N_{k+1} multiply-adds
// per contract.  pi_kernel turns the counts into pi^k_ij = c_ij / p_i once
// (FP64, rows padded with zeros to a multiple of 4 columns) and records the
// range of the nonzero columns of every row; bdp_many_kernel then runs the
// whole backward recursion of 64 contracts per workgroup with their V_{k+1}
// resident in LDS ([j][64]: lane = contract, so every LDS read is one
// conflict-free 512-byte row), the obstacle phi_k computed where it is
// used, and pi read with scalar loads (a wave's rows are uniform).  One
// launch may cover many trees (a table of trees, one per number of layers
// for instance): workgroup b then prices 64 contracts of the tree whose
// range of workgroups holds b, the trees with the most layers first.

__global__ __launch_bounds__(256) void pi_kernel(PiArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // row over layers 0..n-1
  if (r >= a.rows) return;
  int lo = 0, hi = a.n - 1;  // the layer k with pt_off_k <= r < pt_off_k + N_k
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.layers[mid].pt_off <= r) lo = mid; else hi = mid - 1;
  }
  const LayerDev& L = a.layers[lo];
  const int i = (int)(r - L.pt_off);
  const int N1 = L.N1, N1p = (N1 + 3) & ~3;
  const int32_t* row = a.counts + L.cnt_off + (int64_t)i * N1;
  int64_t p = 0;
  int jlo = N1p, jhi = 0;
  for (int j = lane; j < N1; j += 64) {
    const int32_t c = row[j];
    p += c;
    if (c != 0) {
      jlo = j < jlo ? j : jlo;
      jhi = j + 1;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    p += __shfl_xor(p, off, 64);
    const int l2 = __shfl_xor(jlo, off, 64), h2 = __shfl_xor(jhi, off, 64);
    jlo = l2 < jlo ? l2 : jlo;
    jhi = h2 > jhi ? h2 : jhi;
  }
  double* out = a.pi + a.pi_off[lo] + (int64_t)i * N1p;
  const double inv_p = p > 0 ? (double)p : 1.0;
  for (int j = lane; j < N1p; j += 64) {
    const int32_t c = j < N1 ? row[j] : 0;
    out[j] = p > 0 ? (double)c / inv_p : 0.0;
  }
  if (lane == 0) {
    // whole groups of 4 columns; an empty row scans nothing (continuation 0)
    a.band[r] = p > 0 ? make_int2(jlo & ~3, (jhi + 3) & ~3) : make_int2(0, 0);
  }
}

// pi_off[k] = sum_{l < k} N_l N1p_l (one thread; n is at most a few thousand).
__global__ void pi_offsets_kernel(const LayerDev* layers, int n, int64_t* pi_off) {
  int64_t o = 0;
  for (int k = 0; k < n; ++k) {
    pi_off[k] = o;
    o += (int64_t)layers[k].N * (int64_t)((layers[k].N1 + 3) & ~3);
  }
}

hipError_t launch_pi(const PiArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(pi_offsets_kernel, dim3(1), dim3(1), 0, s, a.layers, a.n,
                     const_cast<int64_t*>(a.pi_off));
  hipLaunchKernelGGL(pi_kernel, dim3((unsigned)((a.rows + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

namespace {

// Obstacle of contract C on layer k (the arithmetic of payoff_kernel, so
// both give the same phi bit for bit): the layer's discount and drifts once,
// then one exponential per asset and grid point.
struct LayerObstacle {
  double disc;
  double drift[3];  // (r - sigma_c^2 / 2) t_k
  bool euro;        // European before maturity: phi = -inf
};

template <int D>
__device__ __forceinline__ LayerObstacle layer_obstacle(const Contract& C, int n, int k) {
  LayerObstacle o;
  const double t = C.Tm * (double)k / (double)n;
  o.disc = exp(-C.r * t);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    o.drift[c] = c < D ? (C.r - 0.5 * C.sigma[c] * C.sigma[c]) * t : 0.0;
  o.euro = (C.kind & 2) && k < n;
  return o;
}

template <int D>
__device__ __forceinline__ double obstacle(const Contract& C, const LayerObstacle& o,
                                           const float* xs) {
  double y[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double v = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) v += C.mix[c * D + e] * (double)xs[e];
    y[c] = C.has_mix ? v : (double)xs[c];
  }
  double v;
  if (C.kind & 1) {
    double smax = -__builtin_huge_val();
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double sc = C.S0 * exp(o.drift[c] + C.sigma[c] * y[c]);
      smax = sc > smax ? sc : smax;
    }
    v = o.disc * fmax(smax - C.K, 0.0);
  } else {
    const double sc = C.S0 * exp(o.drift[0] + C.sigma[0] * y[0]);
    v = o.disc * fmax(C.K - sc, 0.0);
  }
  return o.euro ? -__builtin_huge_val() : v;
}

// The grid is read through global pointers: taken from the tree table, the
// generic ones were read with flat loads, which count against the same wait
// counter as the kernel's scalar weight loads.
template <int D>
__device__ __forceinline__ void grid_point(const ManyTree& a, int64_t pt_off, int i,
                                           float* xs) {
  const int64_t at = pt_off + i;
  typedef const float __attribute__((address_space(1)))* GlobalF32;
  if (D == 1) {
    xs[0] = ((GlobalF32)a.pts1)[at];
  } else {
    const GlobalF32 g = (GlobalF32)(a.pts + at);  // the point's x, y (, z)
    xs[0] = g[0];
    xs[1] = g[1];
    if (D == 3) xs[2] = g[2];
  }
}

}  // namespace

// Read-only device memory in the global address space: uniform loads through
// such pointers may become scalar loads (a generic pointer taken from the
// tree table would be read with flat vector loads).
typedef const double __attribute__((address_space(1)))* GlobalF64;
typedef const int32_t __attribute__((address_space(1)))* GlobalI32;
typedef const int64_t __attribute__((address_space(1)))* GlobalI64;
typedef const uint64_t __attribute__((address_space(1)))* GlobalU64;


// Workgroup b prices contracts 64 b .. 64 b + 63 (lane = contract); wave w
// of W owns the rows i = w + W t of every layer, R of them at a time, and
// keeps their new values in registers until every wave has finished reading
// V_{k+1}.  MAXR >= ceil(N_max / W).  The weights of a row group reach the
// FMAs as scalar operands: the loads of the next column group are issued
// once the current group's V_{k+1} values are in (scalar and LDS loads share
// one counter), so they travel while the current group's FMAs run.
template <int D, int W, int MAXR, int R>
__global__ __launch_bounds__(64 * W) void bdp_many_kernel(ManyArgs a) {
  extern __shared__ double Vs[];  // [Np_max][64]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // the workgroup's tree: the one tree, or the last table entry with
  // blk0 <= blockIdx.x
  ManyTree T;
  int64_t qb = (int64_t)blockIdx.x * 64, qe = a.nq;
  if (a.trees) {
    // the table is read through a global pointer, so the record's values are
    // known to be uniform (a generic load could be a per-lane one)
    constexpr int kWords = (int)(sizeof(ManyTree) / 8);
    const GlobalU64 tab = (GlobalU64)a.trees;
    constexpr int kBlk0 = (int)(offsetof(ManyTree, blk0) / 4);
    int lo = 0, hi = a.n_trees - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (((GlobalI32)tab)[mid * 2 * kWords + kBlk0] <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    uint64_t raw[kWords];
#pragma unroll
    for (int w = 0; w < kWords; ++w) raw[w] = tab[lo * kWords + w];
    __builtin_memcpy(&T, raw, sizeof(ManyTree));
    qb = T.q0 + ((int64_t)blockIdx.x - T.blk0) * 64;
    qe = T.q0 + T.nq;
  } else {
    T.layers = a.layers;
    T.pts1 = a.pts1;
    T.pts = a.pts;
    T.pi_off = a.pi_off;
    T.pi = a.pi;
    T.band = a.band;
    T.n = a.n;
  }
  const int64_t q = qb + lane;
  const Contract C = a.specs[q < qe ? q : qe - 1];
  // zero the padding rows once (they meet only zero weights, but must be finite)
  for (int j = wave; j < a.np_max; j += W) Vs[j * 64 + lane] = 0.0;
  __syncthreads();
  // per-layer fields through global pointers (uniform values)
  const GlobalI32 lay = (GlobalI32)T.layers;
  constexpr int kLayWords = (int)(sizeof(LayerDev) / 4);
  constexpr int kN = (int)(offsetof(LayerDev, N) / 4), kN1 = (int)(offsetof(LayerDev, N1) / 4),
                kPt = (int)(offsetof(LayerDev, pt_off) / 4);
  {
    const int Nn = lay[T.n * kLayWords + kN];
    const int64_t pt = lay[T.n * kLayWords + kPt];
    const LayerObstacle ob = layer_obstacle<D>(C, T.n, T.n);
    for (int i = wave; i < Nn; i += W) {
      float xs[3];
      grid_point<D>(T, pt, i, xs);
      Vs[i * 64 + lane] = obstacle<D>(C, ob, xs);
    }
  }
  __syncthreads();
  for (int k = T.n - 1; k >= 0; --k) {
    const int Nk = lay[k * kLayWords + kN], N1p = (lay[k * kLayWords + kN1] + 3) & ~3;
    const int64_t pt = lay[k * kLayWords + kPt];
    const GlobalF64 P = (GlobalF64)T.pi + ((GlobalI64)T.pi_off)[k];
    const GlobalI32 B = (GlobalI32)(T.band + pt);  // (lo, hi) pairs
    const LayerObstacle ob = layer_obstacle<D>(C, T.n, k);
    double res[MAXR];
#pragma unroll
    for (int t0 = 0; t0 < MAXR; t0 += R) {
      const int ib = wave + W * t0;
      if (ib >= Nk) break;
      int jlo = 1 << 30, jhi = 0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = ib + W * t;
        if (i < Nk) {
          const int bx = B[2 * i], by = B[2 * i + 1];
          if (by > bx) {
            jlo = bx < jlo ? bx : jlo;
            jhi = by > jhi ? by : jhi;
          }
        }
      }
      double acc[R];
#pragma unroll
      for (int t = 0; t < R; ++t) acc[t] = 0.0;
      GlobalF64 prow[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = ib + W * t < Nk ? ib + W * t : ib;  // rows past the end repeat row ib
        prow[t] = P + (int64_t)i * N1p;
      }
      if (jlo < jhi) {
        double w[R][4];
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
          for (int u = 0; u < 4; ++u) w[t][u] = prow[t][jlo + u];
        for (int j = jlo; j < jhi; j += 4) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = Vs[(j + u) * 64 + lane];
          // this group's V and weights are in; only then the next group's
          // weights are requested (the last group re-reads its own)
          __builtin_amdgcn_sched_barrier(0);
          __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
          __builtin_amdgcn_sched_barrier(0);
          const int jn = j + 4 < jhi ? j + 4 : j;
          double wn[R][4];
#pragma unroll
          for (int t = 0; t < R; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) wn[t][u] = prow[t][jn + u];
#pragma unroll
          for (int t = 0; t < R; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[t] = fma(w[t][u], v[u], acc[t]);
#pragma unroll
          for (int t = 0; t < R; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) w[t][u] = wn[t][u];
        }
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = ib + W * t;
        if (i < Nk) {
          float xs[3];
          grid_point<D>(T, pt, i, xs);
          const double f = obstacle<D>(C, ob, xs);
          res[t0 + t] = f > acc[t] ? f : acc[t];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXR; ++t) {
      const int i = wave + W * t;
      if (i < Nk) Vs[i * 64 + lane] = res[t];
    }
    __syncthreads();
  }
  if (wave == 0 && q < qe) a.V0[q] = Vs[lane];
}

constexpr int kManyWaves = 8;  // waves per workgroup sharing the LDS of 64 contracts

int bdp_many_maxr(int max_n) {
  const int rows = (max_n + kManyWaves - 1) / kManyWaves;
  return rows <= 8 ? 8 : rows <= 16 ? 16 : rows <= 32 ? 32 : -1;
}

size_t bdp_many_lds(int max_np) { return sizeof(double) * 64 * (size_t)max_np; }

template <int D>
static hipError_t launch_bdp_many_d(const ManyArgs& a, hipStream_t s) {
  const dim3 grid(a.trees ? (unsigned)a.blocks : (unsigned)((a.nq + 63) / 64));
  const size_t lds = bdp_many_lds(a.np_max);
  hipError_t e = hipSuccess;
  switch (bdp_many_maxr(a.max_n)) {
#define QTREE_MANY(MR)                                                                        \
  case MR:                                                                                    \
    if (lds > 65536)                                                                          \
      e = hipFuncSetAttribute(                                                                \
          reinterpret_cast<const void*>(bdp_many_kernel<D, kManyWaves, MR, 4>),               \
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                              \
    if (e != hipSuccess) return e;                                                            \
    hipLaunchKernelGGL((bdp_many_kernel<D, kManyWaves, MR, 4>), grid, dim3(64 * kManyWaves),  \
                       lds, s, a);                                                            \
    break;
    QTREE_MANY(8) QTREE_MANY(16) QTREE_MANY(32)
#undef QTREE_MANY
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bdp_many(const ManyArgs& a, hipStream_t s) {
  if (a.trees ? a.blocks <= 0 : a.nq <= 0) return hipSuccess;
  if (a.d == 1) return launch_bdp_many_d<1>(a, s);
  if (a.d == 2) return launch_bdp_many_d<2>(a, s);
  return launch_bdp_many_d<3>(a, s);
}

}  // namespace qtree
