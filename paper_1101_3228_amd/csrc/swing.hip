// Swing option on the quantization tree (Sec. 2: the stochastic control
// problem whose optimal control is bang-bang) and its obstacle, the forward
// on the sum of the factors of the Gaussian model (Sec. 3), FP64.
//
// The state of the recursion is the volume c consumed before date k, and P
// is stored point major ([point][level]) so that the levels of one grid
// point are contiguous.  A 64-lane wave owns row i of layer k and 63
// consecutive levels (lane = level; neighbouring waves overlap by one level,
// whose value feeds the x = 1 choice of the last lane): it walks the count
// row (the same for every lane, zero counts skipped for the whole wave),
// accumulating cont(i, c) = sum_j c_ij P_{k+1}(j, c) / p_i with one
// coalesced load of 64 levels per nonzero count, and then takes, for every
// c, the best feasible exercise x in {0, 1}:
//   P_k(i, c) = max_x  x v_k(i) + cont(i, c + x),
// x feasible when c + x <= Qmax and c + x + (n - k - 1) >= Qmin.
#include "qtree_internal.hpp"

namespace qtree {

namespace {
constexpr int kBlock = 256;
constexpr int kSpan = 63;  // levels a wave writes
}  // namespace

__global__ void forward_payoff_kernel(ForwardArgs a) {
  const int k = blockIdx.y;
  const LayerDev& L = a.layers[k];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.N) return;
  const int d = a.d;
  // variance of w . X_k under X_k = mu_k + L_k z, and the mean term
  double var = 0.0, wm = 0.0;
  for (int c = 0; c < d; ++c) {
    double u = 0.0;
    for (int b = 0; b < d; ++b) u += a.w[b] * (double)L.L[b * d + c];
    var += u * u;
  }
  for (int b = 0; b < d; ++b) wm += a.w[b] * (double)L.mu[b];
  const int64_t at = (int64_t)L.pt_off + i;
  const float4 g = d == 1 ? make_float4(a.pts1[at], 0.f, 0.f, 0.f) : a.pts[at];
  const float xs[3] = {g.x, g.y, g.z};
  double s = 0.0;
  for (int b = 0; b < d; ++b) s += a.w[b] * (double)xs[b];
  const double t = a.Tm * (double)k / (double)a.n;
  a.v[at] = exp(-a.r * t) * (a.S0 * exp(s - wm - 0.5 * var) - a.K);
}

__global__ void swing_init_kernel(SwingArgs a) {
  const LayerDev& L = a.layers[a.n];
  const int64_t total = (int64_t)(a.Qmax + 1) * L.N;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / L.N), i = (int)(t - (int64_t)c * L.N);
    a.P[((int64_t)L.pt_off + i) * (a.Qmax + 1) + c] =
        (c >= a.Qmin && c <= a.Qmax) ? 0.0 : -__builtin_huge_val();
  }
}

__global__ __launch_bounds__(64) void swing_layer_kernel(SwingArgs a, int k) {
  const int lane = threadIdx.x;
  const LayerDev& L = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  const int i = blockIdx.y;
  const int levels = a.Qmax + 1;
  const int c = kSpan * (int)blockIdx.x + lane;
  const int32_t* row = a.counts + L.cnt_off + (int64_t)i * L.N1;
  int64_t p = 0;
  for (int j = lane; j < L.N1; j += 64) p += row[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, 64);
  const double* next = a.P + (int64_t)L1.pt_off * levels + (c < levels ? c : 0);
  double s = 0.0;
  for (int j = 0; j < L.N1; ++j) {
    const int32_t cij = row[j];  // the same for every lane
    if (cij != 0) s = fma((double)cij, next[(int64_t)j * levels], s);
  }
  const double cont = p > 0 ? s / (double)p : 0.0;
  const double cont1 = __shfl_down(cont, 1, 64);  // level c + 1
  if (lane == kSpan || c >= levels) return;
  const double vi = a.v[(int64_t)L.pt_off + i];
  const int rest = a.n - k - 1;  // dates after this one
  double best = -__builtin_huge_val();
  if (c + rest >= a.Qmin) best = cont;
  if (c + 1 <= a.Qmax && c + 1 + rest >= a.Qmin) {
    const double e = vi + cont1;
    best = e > best ? e : best;
  }
  a.P[((int64_t)L.pt_off + i) * levels + c] = best;
}

hipError_t launch_forward_payoff(const ForwardArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.maxN + kBlock - 1) / kBlock), (unsigned)(a.n + 1));
  hipLaunchKernelGGL(forward_payoff_kernel, grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_swing(const SwingArgs& a, const int32_t* N_host, hipStream_t s) {
  hipLaunchKernelGGL(swing_init_kernel, dim3(256), dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned spans = (unsigned)((a.Qmax + 1 + kSpan - 1) / kSpan);
  for (int k = a.n - 1; k >= 0; --k) {
    hipLaunchKernelGGL(swing_layer_kernel, dim3(spans, (unsigned)N_host[k]), dim3(64), 0, s, a, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qtree
