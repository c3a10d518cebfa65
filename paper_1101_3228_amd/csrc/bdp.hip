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
}  // namespace

// One layer for every payoff: blockIdx.y selects the group of kPay payoffs
// (the count row is re-read per group, from L2 for all but the first).
__global__ __launch_bounds__(kBlock) void bdp_layer_kernel(BdpArgs a, int N_k, int N_k1,
                                                           int64_t pt_k, int64_t pt_k1,
                                                           int64_t cnt_k) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (i >= N_k) return;
  const int q0 = blockIdx.y * kPay;
  const int nq = (a.n_pay - q0) < kPay ? (a.n_pay - q0) : kPay;
  const int32_t* row = a.counts + cnt_k + (int64_t)i * N_k1;
  int64_t p = 0;
  double s[kPay];
#pragma unroll
  for (int q = 0; q < kPay; ++q) s[q] = 0.0;
  for (int j = lane; j < N_k1; j += 64) {
    const int32_t c = row[j];
    p += c;
    if (c != 0) {
      const double cd = (double)c;
#pragma unroll
      for (int q = 0; q < kPay; ++q)
        if (q < nq) s[q] = fma(cd, a.V[(int64_t)(q0 + q) * a.P + pt_k1 + j], s[q]);
    }
  }
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
  hipLaunchKernelGGL(bdp_layer_kernel, dim3(blocks, groups), dim3(kBlock), 0, s, a, N_k, N_k1,
                     pt_k, pt_k1, cnt_k);
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
  const BdpJob J = jobs[blockIdx.y];
  const LayerDev& Ln = J.layers[J.n];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < J.nq * Ln.N; t += gridDim.x * blockDim.x) {
    const int q = t / Ln.N, i = t - q * Ln.N;
    const int64_t at = (int64_t)(J.q0 + q) * J.P + Ln.pt_off + i;
    J.V[at] = J.phi[at];
  }
}

__global__ __launch_bounds__(kBdpBlock) void bdp_step_kernel(const BdpJob* jobs,
                                                             const BdpTask* tasks) {
  const BdpTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave >= T.nrows) return;
  const BdpJob& J = jobs[T.job];
  const LayerDev& L = J.layers[T.k];
  const LayerDev& L1 = J.layers[T.k + 1];
  const int i = T.row0 + wave;
  const int32_t* row = J.counts + L.cnt_off + (int64_t)i * L.N1;
  int64_t p = 0;
  double s[kPay];
#pragma unroll
  for (int q = 0; q < kPay; ++q) s[q] = 0.0;
  for (int j = lane; j < L.N1; j += 64) {
    const int32_t c = row[j];
    p += c;
    if (c != 0) {
      const double cd = (double)c;
#pragma unroll
      for (int q = 0; q < kPay; ++q)
        if (q < J.nq) s[q] = fma(cd, J.V[(int64_t)(J.q0 + q) * J.P + L1.pt_off + j], s[q]);
    }
  }
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
    const double f = J.phi[at];
    J.V[at] = f > cont ? f : cont;
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

}  // namespace qtree
