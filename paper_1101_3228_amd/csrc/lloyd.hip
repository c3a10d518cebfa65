// Grid optimization on the device: randomized Lloyd iteration for the
// quadratic quantization error E min_i |X - x_i|^2 of X = L z, z ~ N(0, I_d)
// (Sec. 2, eq. Qerr).  The paper takes precomputed optimal grids for
// Gaussian marginals and moment-matching grids otherwise; here a grid is
// improved by Lloyd steps, each moving every point to the mean of the
// samples of its Voronoi cell (the stationarity condition of eq. Qerr).
//
// One step on the device:
//   accumulate: a persistent grid of workgroups; each stages the current grid
//     (d >= 2: records (g, |g|^2 / 2); d = 1: midpoints padded with +inf) in
//     LDS, draws samples (Philox counter (m, step, 0, 2), Box-Muller, X = L z
//     as fused multiply-add chains from 0), assigns them with the tree's own
//     cell search, and adds to LDS accumulators: the count, each coordinate
//     as the integer rint(x 2^24) and the squared distance to the cell's
//     point as rint(|x - g|^2 2^16) (FP64).  The workgroup stores its totals,
//     zeros included, as row b of a partial table with plain stores.
//   reduce: each workgroup sums 8 columns of the table over its rows (the
//     step's cell sums, counts and distortion).  Integer sums make the result
//     independent of the order of the samples and of the workgroups (the
//     table replaces device atomics from every workgroup onto the same ~N d
//     words, which serialized at the L2).
//   update: one thread per cell: new point = (sum 2^-24) / count in FP64,
//     rounded once to FP32 (an empty cell keeps its point), or the point
//     moved a fraction gamma of the way there; the distortion of the step.
//     The records or midpoints are then rebuilt from the new grid.
//
// The samples may instead be windows of a caller's sample set (Lloyd's
// method on an empirical measure, for marginals of any law): step t takes
// samples (t batch + j) mod M, and samples with a coordinate outside
// [-64, 64] (or not a number) are skipped and counted.
//
// Moment-matching grids (Sec. 2, the sub-optimal grids for marginals without
// an optimal grid): exact integer sums of x and x x' over the admissible
// samples of a set, then, in one workgroup, the mean, covariance and lower
// Cholesky factor in FP64 and the grid mean + chol base.
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"
#include "qtree_search.hpp"

namespace qtree {

namespace {

constexpr int kBlock = 256;
constexpr int kSamplesNd = 8;  // samples per lane per round, d >= 2 (share each record read)

__device__ __forceinline__ long long fixed_of(double v, double scale) {
  return (long long)__builtin_rint(v * scale);
}

// Sample j of the step's window of the caller's set; false (and x = 0) when
// a coordinate is outside [-64, 64] or not a number.
template <int D>
__device__ __forceinline__ bool set_sample(const LloydArgs& a, uint64_t j, float* x) {
  uint64_t q = a.start + j;
  if (q >= a.Ms) q %= a.Ms;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x[c] = a.xs[q * D + c];
    ok = ok && fabsf(x[c]) <= 64.0f;
  }
  if (!ok) {
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = 0.0f;
  }
  return ok;
}

// X = L z for sample m of the step (z from one Philox block).
template <int D>
__device__ __forceinline__ void lloyd_sample(const LloydArgs& a, uint64_t m, float* x) {
  const U4 r = philox4x32_10(U4{(uint32_t)m, a.it_ctr, 0u, 2u}, a.key0, a.key1);
  float z[4];
  box_muller(r.x, r.y, z[0], z[1]);
  box_muller(r.z, r.w, z[2], z[3]);
#pragma unroll
  for (int row = 0; row < D; ++row) {
    float v = 0.0f;
#pragma unroll
    for (int c = 0; c < D; ++c) v = fmaf(a.L[row * D + c], z[c], v);
    x[row] = v;
  }
}

}  // namespace

// Records or midpoints of the current grid (the start grid, then the grid
// of every step).
__global__ void lloyd_prepare_kernel(LloydArgs a, int first) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (first && i == 0 && a.rej_total) *a.rej_total = 0ull;
  if (a.d == 1) {
    if (i >= a.P) return;
    float m = __builtin_huge_valf();
    if (i + 1 < a.N) {
      m = 0.5f * (a.grid[i] + a.grid[i + 1]);
      if (m == 0.0f) m = 0.0f;
    }
    a.mids[i] = m;
  } else {
    if (i >= a.Npad) return;
    float4 rec = make_float4(0.f, 0.f, 0.f, __builtin_huge_valf());
    if (i < a.N) {
      const float* g = a.grid + (size_t)i * a.d;
      float h = g[0] * g[0];
      for (int c = 1; c < a.d; ++c) h = fmaf(g[c], g[c], h);
      rec = make_float4(g[0], a.d > 1 ? g[1] : 0.f, a.d > 2 ? g[2] : 0.f, 0.5f * h);
    }
    a.recs[i] = rec;
  }
}


// LDS: d = 1: midpoints [P], points [N]; d >= 2: records [Npad]; then the
// counts [N] and the sums [N][d] (8-byte aligned).
template <int D, bool SET>
__global__ __launch_bounds__(kBlock) void lloyd_accum_kernel(LloydArgs a) {
  extern __shared__ float4 lds4[];
  float* ldsf = reinterpret_cast<float*>(lds4);
  float* mids = ldsf;                      // d = 1
  float* pts1 = ldsf + a.P;                // d = 1
  float4* recs = lds4;                     // d >= 2
  const size_t grid_words = D == 1 ? (size_t)a.P + a.N : (size_t)a.Npad * 4;
  unsigned long long* sum =
      reinterpret_cast<unsigned long long*>(ldsf + ((grid_words + 1) & ~(size_t)1));
  unsigned int* cnt = reinterpret_cast<unsigned int*>(sum + (size_t)a.N * D);
  __shared__ unsigned long long part[3][kBlock / 64];

  if (D == 1) {
    for (int i = threadIdx.x; i < a.P; i += kBlock) mids[i] = a.mids[i];
    for (int i = threadIdx.x; i < a.N; i += kBlock) pts1[i] = a.grid[i];
  } else {
    for (int i = threadIdx.x; i < a.Npad; i += kBlock) recs[i] = a.recs[i];
  }
  for (int i = threadIdx.x; i < a.N * D; i += kBlock) sum[i] = 0ull;
  for (int i = threadIdx.x; i < a.N; i += kBlock) cnt[i] = 0u;
  __syncthreads();

  constexpr int S = D == 1 ? 1 : kSamplesNd;
  const uint64_t per_round = (uint64_t)gridDim.x * kBlock * S;
  unsigned long long dist = 0ull, used = 0ull, rej = 0ull;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock * S; base < a.M; base += per_round) {
    float xs[S][D];
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t m = base + (uint64_t)s * kBlock + threadIdx.x;
      live[s] = m < a.M;
      if (SET) {
        const bool ok = set_sample<D>(a, live[s] ? m : 0, xs[s]);
        rej += (live[s] && !ok) ? 1ull : 0ull;
        live[s] = live[s] && ok;
      } else {
        lloyd_sample<D>(a, live[s] ? m : 0, xs[s]);
      }
      used += live[s] ? 1ull : 0ull;
    }
    int idx[S];
    if (D == 1) {
      idx[0] = cell_1d(mids, a.logP, xs[0][0]);
    } else {
      argmin_scan_tiled<D, S, 4>(recs, a.Npad, xs, idx);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (!live[s]) continue;
      const int i = idx[s];
      float g[D];
      if (D == 1) {
        g[0] = pts1[i];
      } else {
        const float4 r = recs[i];
        g[0] = r.x;
        if (D > 1) g[1] = r.y;
        if (D > 2) g[2] = r.z;
      }
      double d2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double dx = (double)xs[s][c] - (double)g[c];
        d2 = d2 + dx * dx;
        atomicAdd(&sum[(size_t)i * D + c],
                  (unsigned long long)fixed_of((double)xs[s][c], 0x1p24));
      }
      atomicAdd(&cnt[i], 1u);
      dist += (unsigned long long)fixed_of(d2, 0x1p16);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dist += __shfl_xor(dist, off, 64);
    used += __shfl_xor(used, off, 64);
    rej += __shfl_xor(rej, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = dist;
    part[1][threadIdx.x >> 6] = used;
    part[2][threadIdx.x >> 6] = rej;
  }
  __syncthreads();
  unsigned long long* row = a.part + (size_t)blockIdx.x * a.E;
  const int nd = a.N * D;
  if (threadIdx.x < 3) {
    unsigned long long t = 0ull;
    for (int w = 0; w < kBlock / 64; ++w) t += part[threadIdx.x][w];
    row[nd + a.N + threadIdx.x] = t;
  }
  for (int i = threadIdx.x; i < nd; i += kBlock) row[i] = sum[i];
  for (int i = threadIdx.x; i < a.N; i += kBlock) row[nd + i] = cnt[i];
}

// Column sums of the partial table over its `rows` rows: workgroup b takes
// columns [8 b, 8 b + 8); lane l adds rows l, l + 256, ...; the 256 lane
// sums of each column are then added in LDS.
constexpr int kReduceCols = 8;
__global__ __launch_bounds__(kBlock) void lloyd_reduce_kernel(LloydArgs a, int rows) {
  __shared__ unsigned long long red[kReduceCols][kBlock];
  const int c0 = (int)blockIdx.x * kReduceCols;
  unsigned long long acc[kReduceCols] = {};
  for (int r = threadIdx.x; r < rows; r += kBlock) {
    const unsigned long long* src = a.part + (size_t)r * a.E + c0;
#pragma unroll
    for (int q = 0; q < kReduceCols; ++q)
      if (c0 + q < a.E) acc[q] += src[q];
  }
#pragma unroll
  for (int q = 0; q < kReduceCols; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < kReduceCols; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < kReduceCols) {
    const int c = c0 + (int)threadIdx.x;
    const int nd = a.N * a.d;
    const unsigned long long v = red[threadIdx.x][0];
    if (c < nd) a.sum[c] = v;
    else if (c < nd + a.N) a.cnt[c - nd] = (unsigned int)v;
    else if (c == nd + a.N) *a.dist = v;
    else if (c == nd + a.N + 1) *a.used = v;
    else if (c == nd + a.N + 2) *a.rej = v;
  }
}

// New point of cell i from the accumulators (the old point when empty):
// the cell mean, or the old point moved the fraction gamma towards it.
__device__ __forceinline__ float lloyd_new(const LloydArgs& a, int i, int c) {
  const float g = a.grid[(size_t)i * a.d + c];
  const unsigned int n = a.cnt[i];
  if (n == 0u) return g;
  const double mean = ((double)(long long)a.sum[(size_t)i * a.d + c] * 0x1p-24) / (double)n;
  return a.gamma == 1.0 ? (float)mean : (float)((double)g + a.gamma * (mean - (double)g));
}

// One thread per cell: its new point (each thread reads and writes only its
// own point), and the step's distortion and sample counts; the records or
// midpoints are rebuilt by lloyd_prepare_kernel afterwards.
__global__ void lloyd_update_kernel(LloydArgs a) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (i == 0) {
    if (a.xs) {
      const unsigned long long used = *a.used;
      if (a.distortion)
        a.distortion[a.it] =
            used > 0ull ? ((double)(long long)*a.dist * 0x1p-16) / (double)(long long)used : 0.0;
      const unsigned long long total = *a.rej_total + *a.rej;
      *a.rej_total = total;
      if (a.rejected) *a.rejected = (long long)total;
    } else if (a.distortion) {
      a.distortion[a.it] = ((double)(long long)*a.dist * 0x1p-16) / (double)a.M;
    }
  }
  if (i >= a.N) return;
  float g[kMaxDim] = {0.f, 0.f, 0.f};
  for (int c = 0; c < a.d; ++c) g[c] = lloyd_new(a, i, c);
  for (int c = 0; c < a.d; ++c) a.grid[(size_t)i * a.d + c] = g[c];
}

size_t lloyd_lds_bytes(int d, int N, int Npad, int P) {
  const size_t grid_words = d == 1 ? (size_t)P + N : (size_t)Npad * 4;
  return sizeof(float) * ((grid_words + 1) & ~(size_t)1) + sizeof(unsigned long long) * N * d +
         sizeof(unsigned int) * N;
}

hipError_t launch_lloyd_prepare(const LloydArgs& a, hipStream_t s) {
  const int n = a.d == 1 ? a.P : a.Npad;
  hipLaunchKernelGGL(lloyd_prepare_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a,
                     1);
  return hipGetLastError();
}

template <int D, bool SET>
static hipError_t launch_accum(const LloydArgs& a, int blocks, size_t lds, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (lds > 65536)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(lloyd_accum_kernel<D, SET>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    hipLaunchKernelGGL((lloyd_accum_kernel<D, SET>), dim3(blocks), dim3(kBlock), lds, s, a);
  return e;
}

hipError_t launch_lloyd_step(const LloydArgs& a, int blocks, hipStream_t s) {
  if (blocks < 1 || blocks > kLloydMaxBlocks) return hipErrorInvalidValue;
  const size_t lds = lloyd_lds_bytes(a.d, a.N, a.Npad, a.P);
  const bool set = a.xs != nullptr;
  hipError_t e;
  if (a.d == 1) e = set ? launch_accum<1, true>(a, blocks, lds, s) : launch_accum<1, false>(a, blocks, lds, s);
  else if (a.d == 2) e = set ? launch_accum<2, true>(a, blocks, lds, s) : launch_accum<2, false>(a, blocks, lds, s);
  else e = set ? launch_accum<3, true>(a, blocks, lds, s) : launch_accum<3, false>(a, blocks, lds, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lloyd_reduce_kernel, dim3((a.E + kReduceCols - 1) / kReduceCols),
                     dim3(kBlock), 0, s, a, blocks);
  hipLaunchKernelGGL(lloyd_update_kernel, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     a);
  const int n = a.d == 1 ? a.P : a.Npad;
  hipLaunchKernelGGL(lloyd_prepare_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a,
                     0);
  return hipGetLastError();
}

// ------------------------------------------------- moment-matching grids

// Exact integer sums over the admissible samples: the count, rint(x_r 2^24)
// and rint(x_r x_c 2^16) (the product exact in FP64); per-lane sums over a
// grid-stride loop, wave sums, one 64-bit device atomic per wave and value
// (integer addition, so the totals do not depend on the order).
template <int D>
__global__ __launch_bounds__(kBlock) void moments_kernel(const float* __restrict__ x, uint64_t M,
                                                         unsigned long long* sums) {
  unsigned long long acc[1 + D + D * D] = {};
  for (uint64_t m = (uint64_t)blockIdx.x * kBlock + threadIdx.x; m < M;
       m += (uint64_t)gridDim.x * kBlock) {
    float v[D];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      v[c] = x[m * D + c];
      ok = ok && fabsf(v[c]) <= 64.0f;
    }
    if (!ok) continue;
    acc[0] += 1ull;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      acc[1 + r] += (unsigned long long)fixed_of((double)v[r], 0x1p24);
#pragma unroll
      for (int c = 0; c < D; ++c)
        acc[1 + D + r * D + c] +=
            (unsigned long long)fixed_of((double)v[r] * (double)v[c], 0x1p16);
    }
  }
#pragma unroll
  for (int q = 0; q < 1 + D + D * D; ++q) {
    unsigned long long t = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0 && t != 0ull) atomicAdd(&sums[q], t);
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (i < n) p[i] = 0ull;
}

// One workgroup: thread 0 forms the mean, covariance and Cholesky factor in
// FP64 (the lower factor column by column; a non-positive pivot gives a zero
// column), then every thread maps grid points base[i] to
// mean + chol base[i] (FP64, left to right, rounded once).
__global__ __launch_bounds__(kBlock) void moment_grid_kernel(int d, const long long* sums,
                                                             const float* base, int N, float* grid,
                                                             double* moments) {
  __shared__ double mean[kMaxDim], chol[kMaxDim * kMaxDim];
  if (threadIdx.x == 0) {
    double cov[kMaxDim * kMaxDim] = {}, L[kMaxDim * kMaxDim] = {}, mu[kMaxDim] = {};
    const long long count = sums[0];
    if (count > 0) {
      for (int r = 0; r < d; ++r) mu[r] = ((double)sums[1 + r] * 0x1p-24) / (double)count;
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
          cov[r * d + c] =
              ((double)sums[1 + d + r * d + c] * 0x1p-16) / (double)count - mu[r] * mu[c];
    }
    for (int r = 0; r < d; ++r) {
      for (int c = 0; c <= r; ++c) {
        double v = cov[r * d + c];
        for (int q = 0; q < c; ++q) v = v - L[r * d + q] * L[c * d + q];
        if (r == c) L[r * d + c] = v > 0.0 ? sqrt(v) : 0.0;
        else L[r * d + c] = L[c * d + c] > 0.0 ? v / L[c * d + c] : 0.0;
      }
    }
    for (int r = 0; r < d; ++r) mean[r] = mu[r];
    for (int q = 0; q < d * d; ++q) chol[q] = L[q];
    if (moments) {
      for (int r = 0; r < d; ++r) moments[r] = mu[r];
      for (int q = 0; q < d * d; ++q) {
        moments[d + q] = cov[q];
        moments[d + d * d + q] = L[q];
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += kBlock) {
    for (int r = 0; r < d; ++r) {
      double v = mean[r];
      for (int c = 0; c <= r; ++c) v = v + chol[r * d + c] * (double)base[(size_t)i * d + c];
      grid[(size_t)i * d + r] = (float)v;
    }
  }
}

hipError_t launch_sample_moments(int d, const float* x, uint64_t M, long long* sums,
                                 hipStream_t s) {
  const int words = 1 + d + d * d;
  auto* u = reinterpret_cast<unsigned long long*>(sums);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(kBlock), 0, s, u, words);
  if (M > 0) {
    const uint64_t want = (M + kBlock - 1) / kBlock;
    const unsigned blocks = (unsigned)(want < 2048 ? want : 2048);
    if (d == 1) hipLaunchKernelGGL(moments_kernel<1>, dim3(blocks), dim3(kBlock), 0, s, x, M, u);
    else if (d == 2) hipLaunchKernelGGL(moments_kernel<2>, dim3(blocks), dim3(kBlock), 0, s, x, M, u);
    else hipLaunchKernelGGL(moments_kernel<3>, dim3(blocks), dim3(kBlock), 0, s, x, M, u);
  }
  return hipGetLastError();
}

hipError_t launch_moment_grid(int d, const long long* sums, const float* base, int N,
                              float* grid, double* moments, hipStream_t s) {
  hipLaunchKernelGGL(moment_grid_kernel, dim3(1), dim3(kBlock), 0, s, d, sums, base, N, grid,
                     moments);
  return hipGetLastError();
}

}  // namespace qtree
