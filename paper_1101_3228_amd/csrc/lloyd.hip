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
//     rounded once to FP32 (an empty cell keeps its point), then its record
//     or the midpoint to its right; the distortion of the step.
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

// Records or midpoints of the start grid.
__global__ void lloyd_prepare_kernel(LloydArgs a) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
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
template <int D>
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
  __shared__ unsigned long long part[kBlock / 64];

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
  unsigned long long dist = 0ull;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock * S; base < a.M; base += per_round) {
    float xs[S][D];
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t m = base + (uint64_t)s * kBlock + threadIdx.x;
      live[s] = m < a.M;
      lloyd_sample<D>(a, live[s] ? m : 0, xs[s]);
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
  for (int off = 32; off > 0; off >>= 1) dist += __shfl_xor(dist, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = dist;
  __syncthreads();
  unsigned long long* row = a.part + (size_t)blockIdx.x * a.E;
  const int nd = a.N * D;
  if (threadIdx.x == 0) {
    unsigned long long t = 0ull;
    for (int w = 0; w < kBlock / 64; ++w) t += part[w];
    row[nd + a.N] = t;
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
  }
}

// New point of cell i from the accumulators (the old point when empty).
__device__ __forceinline__ float lloyd_new(const LloydArgs& a, int i, int c) {
  const unsigned int n = a.cnt[i];
  if (n == 0u) return a.grid[(size_t)i * a.d + c];
  const double s = (double)(long long)a.sum[(size_t)i * a.d + c] * 0x1p-24;
  return (float)(s / (double)n);
}

__global__ void lloyd_update_kernel(LloydArgs a) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (i == 0 && a.distortion)
    a.distortion[a.it] = ((double)(long long)*a.dist * 0x1p-16) / (double)a.M;
  if (i >= a.N) return;
  float g[kMaxDim] = {0.f, 0.f, 0.f};
  for (int c = 0; c < a.d; ++c) g[c] = lloyd_new(a, i, c);
  if (a.d == 1) {
    // the midpoint to the right of point i, from both new points
    if (i + 1 < a.N) {
      float m = 0.5f * (g[0] + lloyd_new(a, i + 1, 0));
      if (m == 0.0f) m = 0.0f;
      a.mids[i] = m;
    }
  } else {
    float h = g[0] * g[0];
    for (int c = 1; c < a.d; ++c) h = fmaf(g[c], g[c], h);
    a.recs[i] = make_float4(g[0], g[1], g[2], 0.5f * h);
  }
  // another thread reads this point only when the cell is empty (d = 1, the
  // cell to its right), and then the value written is the value read
  for (int c = 0; c < a.d; ++c) a.grid[(size_t)i * a.d + c] = g[c];
}

size_t lloyd_lds_bytes(int d, int N, int Npad, int P) {
  const size_t grid_words = d == 1 ? (size_t)P + N : (size_t)Npad * 4;
  return sizeof(float) * ((grid_words + 1) & ~(size_t)1) + sizeof(unsigned long long) * N * d +
         sizeof(unsigned int) * N;
}

hipError_t launch_lloyd_prepare(const LloydArgs& a, hipStream_t s) {
  const int n = a.d == 1 ? a.P : a.Npad;
  hipLaunchKernelGGL(lloyd_prepare_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lloyd_step(const LloydArgs& a, int blocks, hipStream_t s) {
  if (blocks < 1 || blocks > kLloydMaxBlocks) return hipErrorInvalidValue;
  const size_t lds = lloyd_lds_bytes(a.d, a.N, a.Npad, a.P);
  hipError_t e = hipSuccess;
  if (a.d == 1) {
    if (lds > 65536)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(lloyd_accum_kernel<1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      hipLaunchKernelGGL(lloyd_accum_kernel<1>, dim3(blocks), dim3(kBlock), lds, s, a);
  } else if (a.d == 2) {
    if (lds > 65536)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(lloyd_accum_kernel<2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      hipLaunchKernelGGL(lloyd_accum_kernel<2>, dim3(blocks), dim3(kBlock), lds, s, a);
  } else {
    if (lds > 65536)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(lloyd_accum_kernel<3>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      hipLaunchKernelGGL(lloyd_accum_kernel<3>, dim3(blocks), dim3(kBlock), lds, s, a);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lloyd_reduce_kernel, dim3((a.E + kReduceCols - 1) / kReduceCols),
                     dim3(kBlock), 0, s, a, blocks);
  hipLaunchKernelGGL(lloyd_update_kernel, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     a);
  return hipGetLastError();
}

}  // namespace qtree
