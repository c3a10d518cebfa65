// Candidate lists of the d = 2 bucketed cell search.  A layer's reachable
// box is cut into buckets; bucket R lists every grid point p that can be the
// FP32 argmin of the half-norm key k_p(x) = h_p - <x, g_p> for some x in R.
// With u = 2^-24 the key carries an error below
// E(x) = 4.1 u (max_p h_p + |x_0| max_p |g_0| + |x_1| max_p |g_1|), so the
// FP32 winner p* for x has |x - g_p*|^2 <= min_q |x - g_q|^2 + 4 E(x) (both
// keys may err by E).  Over R, min_q |x - g_q|^2 <= U = min_q max over R's
// corners of |c - g_q|^2, and |x - g_p|^2 >= lo_p, the squared distance from
// g_p to R; so every p with lo_p <= U + 4 E_R (E_R the bound over R, doubled
// here for margin) is kept.  R is the bucket widened by 1/64 of its width
// on every side, more than the FP32 rounding of the bucket index can move a
// point.  FP64 throughout.  Row t: entry 0 the count c, entries 1..c the
// candidates in increasing index, then the layer's point count N (the
// search's pad record, which never wins) to the end of the last 8-entry
// group; more than kBucketCap candidates mark the bucket full (entry 0 =
// kBucketFull: the search then scans every point).
#include "qtree_internal.hpp"

namespace qtree {

namespace {
constexpr int kBlock = 256;
}

__global__ __launch_bounds__(kBlock) void bucket_build_kernel(const LayerDev* layers, int nl,
                                                              int total, const float4* pts,
                                                              uint16_t* rows) {
  const int t = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (t >= total) return;
  int lo = 0, hi = nl - 1;  // the layer holding bucket t: largest k with bk_off_k <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (layers[mid].bk_off <= t) lo = mid; else hi = mid - 1;
  }
  const LayerDev& L = layers[lo];
  const int r = t - L.bk_off;
  const int i = r / L.bk_B[1], j = r - i * L.bk_B[1];
  const double w0 = 1.0 / (double)L.bk_scale[0], w1 = 1.0 / (double)L.bk_scale[1];
  const double a0 = (double)L.bk_lo[0] + (double)i * w0 - w0 / 64.0;
  const double b0 = (double)L.bk_lo[0] + (double)(i + 1) * w0 + w0 / 64.0;
  const double a1 = (double)L.bk_lo[1] + (double)j * w1 - w1 / 64.0;
  const double b1 = (double)L.bk_lo[1] + (double)(j + 1) * w1 + w1 / 64.0;
  const float4* g = pts + L.pt_off;
  double U = __builtin_huge_val(), hmax = 0.0, G0 = 0.0, G1 = 0.0;
  for (int p = 0; p < L.N; ++p) {
    const float4 q = g[p];
    const double d0 = fmax(fabs(a0 - (double)q.x), fabs(b0 - (double)q.x));
    const double d1 = fmax(fabs(a1 - (double)q.y), fabs(b1 - (double)q.y));
    U = fmin(U, d0 * d0 + d1 * d1);
    hmax = fmax(hmax, (double)q.w);
    G0 = fmax(G0, fabs((double)q.x));
    G1 = fmax(G1, fabs((double)q.y));
  }
  const double X0 = fmax(fabs(a0), fabs(b0)), X1 = fmax(fabs(a1), fabs(b1));
  const double E = 2.0 * 4.1 * 0x1p-24 * (hmax + X0 * G0 + X1 * G1);
  const double thr = U * (1.0 + 1e-9) + 4.0 * E;
  uint16_t* out = rows + (int64_t)t * kBucketRow;
  int c = 0;
  for (int p = 0; p < L.N; ++p) {
    const float4 q = g[p];
    const double e0 = fmax(0.0, fmax(a0 - (double)q.x, (double)q.x - b0));
    const double e1 = fmax(0.0, fmax(a1 - (double)q.y, (double)q.y - b1));
    if (e0 * e0 + e1 * e1 <= thr) {
      if (c < kBucketCap) out[1 + c] = (uint16_t)p;
      ++c;
    }
  }
  if (c > kBucketCap) {
    out[0] = kBucketFull;
    return;
  }
  // c >= 1: the point whose farthest corner distance is U lies within U.
  // The search reads whole groups of 8 entries; the pads all name one
  // record, so the lanes of a wave that read it share one LDS access.
  for (int q = 1 + c; q < ((c + 8) & ~7); ++q) out[q] = (uint16_t)L.N;
  out[0] = (uint16_t)c;
}

hipError_t launch_bucket_build(const LayerDev* layers, int n_layers_total, int total_buckets,
                               const float4* pts, uint16_t* rows, hipStream_t s) {
  if (total_buckets <= 0) return hipSuccess;
  hipLaunchKernelGGL(bucket_build_kernel, dim3((unsigned)((total_buckets + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, layers, n_layers_total, total_buckets, pts, rows);
  return hipGetLastError();
}

}  // namespace qtree
