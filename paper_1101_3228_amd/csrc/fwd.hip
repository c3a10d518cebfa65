// Forward step of the quantization tree on gfx950: Monte Carlo transition
// counts between the Voronoi cells of consecutive layers.
//
//  - fwd_layer_1d : time-layer parallel estimate (Sec. 4, Algorithm III) for
//                   d = 1.  A block owns one chunk of samples of one layer,
//                   stages the cell midpoints of Gamma_k and Gamma_{k+1} in LDS
//                   and finds both cells by a branch-free binary search.
//  - fwd_layer_nd : the same for d = 2, 3 with the grids staged in LDS as
//                   (g, |g|^2/2) records and a brute-force argmin scan (the
//                   paper's choice over kd-trees, Sec. 3 "Nearest Neighbor
//                   search"), S samples per lane so each LDS broadcast read
//                   feeds S distance evaluations.
//  - fwd_path     : pathwise estimate (Sec. 3, Algorithms I/II), one lane per
//                   path walking all layers.
// Counts are incremented with device-scope atomic adds (Sec. 3, "Updating
// p^k_ij"); integer addition makes the result independent of the order.
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"
#include "qtree_search.hpp"

namespace qtree {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void count_add(int32_t* p) {
  __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Map a workgroup to a (layer, chunk) unit.  Workgroups are dispatched to
// the 8 XCDs round robin (block b runs on XCD b mod 8); with xcd_map the
// units are dealt so that consecutive chunks of one layer -- which hit the
// same count block -- stay on one XCD and its L2.
__device__ __forceinline__ bool unit_of_block(const FwdArgs& a, int& k, int& chunk) {
  int u;
  if (a.xcd_map) {
    const int b = (int)blockIdx.x;
    const int slot = b >> 3;
    if (slot >= a.units_per_xcd) return false;
    u = (b & 7) * a.units_per_xcd + slot;
  } else {
    u = (int)blockIdx.x;
  }
  if (u >= a.units) return false;
  k = u / a.chunks;
  chunk = u - k * a.chunks;
  return true;
}



}  // namespace

__global__ void zero_i32_kernel(int32_t* __restrict__ p, int64_t count) {
  const int64_t n4 = count >> 2;
  int4* p4 = reinterpret_cast<int4*>(p);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    p4[i] = make_int4(0, 0, 0, 0);
  const int64_t t = (n4 << 2) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count && (int64_t)blockIdx.x * blockDim.x + threadIdx.x < 4) p[t] = 0;
}

__global__ __launch_bounds__(kBlock) void fwd_layer_1d(FwdArgs a) {
  extern __shared__ float lds[];
  int k, chunk;
  if (!unit_of_block(a, k, chunk)) return;
  const LayerDev& L0 = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  float* mk = lds;
  float* mk1 = lds + L0.P;
  for (int i = threadIdx.x; i < L0.P; i += kBlock) mk[i] = a.mids[L0.aux_off + i];
  for (int i = threadIdx.x; i < L1.P; i += kBlock) mk1[i] = a.mids[L1.aux_off + i];
  __syncthreads();

  const float mu = L0.mu[0], Lz = L0.L[0], A = L0.A[0], b = L0.b[0], T = L0.T[0];
  const int logP0 = L0.logP, logP1 = L1.logP, N1 = L0.N1;
  int32_t* cnt = a.counts + L0.cnt_off;
  const uint64_t end = a.m0 + a.M;
  const uint64_t lo = a.m0 + (uint64_t)chunk * a.chunk_len;
  const uint64_t hi = (lo + a.chunk_len < end) ? lo + a.chunk_len : end;
  // sample m uses Philox block m >> 1, Box-Muller pair m & 1
  for (uint64_t blk = (lo >> 1) + threadIdx.x; blk < ((hi + 1) >> 1); blk += kBlock) {
    const U4 r = philox4x32_10(U4{(uint32_t)blk, (uint32_t)k, a.contract, 0u}, a.key0, a.key1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t m = 2 * blk + h;
      if (m < lo || m >= hi) continue;
      float z, e;
      box_muller(h ? r.z : r.x, h ? r.w : r.y, z, e);
      const float x = fmaf(Lz, z, mu);
      const float y = fmaf(T, e, fmaf(A, x, b));
      const int i = cell_1d(mk, logP0, x);
      const int j = cell_1d(mk1, logP1, y);
      count_add(cnt + (int64_t)i * N1 + j);
    }
  }
}

template <int D, int S>
__global__ __launch_bounds__(kBlock) void fwd_layer_nd(FwdArgs a) {
  extern __shared__ float4 lds4[];
  int k, chunk;
  if (!unit_of_block(a, k, chunk)) return;
  const LayerDev& L0 = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  const int N0 = L0.N, N1 = L0.N1;
  float4* gk = lds4;
  float4* gk1 = lds4 + N0;
  for (int i = threadIdx.x; i < N0; i += kBlock) gk[i] = a.pts[L0.pt_off + i];
  for (int i = threadIdx.x; i < N1; i += kBlock) gk1[i] = a.pts[L1.pt_off + i];
  __syncthreads();

  int32_t* cnt = a.counts + L0.cnt_off;
  const uint64_t end = a.m0 + a.M;
  const uint64_t lo = a.m0 + (uint64_t)chunk * a.chunk_len;
  const uint64_t hi = (lo + a.chunk_len < end) ? lo + a.chunk_len : end;
  for (uint64_t base = lo; base < hi; base += (uint64_t)kBlock * S) {
    float xs[S][D], ys[S][D];
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t m = base + (uint64_t)s * kBlock + threadIdx.x;
      live[s] = m < hi;
      float z[D], e[D];
      layer_normals<D>(a.key0, a.key1, a.contract, k, live[s] ? m : lo, z, e);
      layer_pair<D>(L0, z, e, xs[s], ys[s]);
    }
    int ii[S], jj[S];
    argmin_scan<D, S>(gk, N0, xs, ii);
    argmin_scan<D, S>(gk1, N1, ys, jj);
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (live[s]) count_add(cnt + (int64_t)ii[s] * N1 + jj[s]);
  }
}

// Pathwise (Algorithm I/II): one lane per path.  d = 1 keeps the midpoints of
// every layer in LDS when they fit (ws_mids_in_lds), d >= 2 stages the grid
// of the next layer in LDS at every step (the whole block walks the layers
// together).
template <int D>
__global__ __launch_bounds__(kBlock) void fwd_path(FwdArgs a, int mids_in_lds) {
  extern __shared__ float lds[];
  const uint64_t m = a.m0 + (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool live = m < a.m0 + a.M;
  const uint32_t mc = (uint32_t)(live ? m : a.m0);
  float x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = a.layers[0].x0[c];
  int i = 0;
  if (D == 1) {
    const float* mids = a.mids;
    if (mids_in_lds) {
      for (int64_t t = threadIdx.x; t < a.mids_total; t += kBlock) lds[t] = a.mids[t];
      __syncthreads();
      mids = lds;
    }
    float zb[4];
    for (int k = 0; k < a.n; ++k) {
      const LayerDev& L = a.layers[k];
      if ((k & 3) == 0) {
        const U4 r = philox4x32_10(U4{mc, (uint32_t)(k >> 2), a.contract, 1u}, a.key0, a.key1);
        box_muller(r.x, r.y, zb[0], zb[1]);
        box_muller(r.z, r.w, zb[2], zb[3]);
      }
      const float e = zb[k & 3];
      const float y = fmaf(L.T[0], e, fmaf(L.A[0], x[0], L.b[0]));
      const LayerDev& L1 = a.layers[k + 1];
      const int j = cell_1d(mids + L1.aux_off, L1.logP, y);
      if (live) count_add(a.counts + L.cnt_off + (int64_t)i * L.N1 + j);
      i = j;
      x[0] = y;
    }
  } else {
    float4* g = reinterpret_cast<float4*>(lds);
    float eb[4];
    for (int k = 0; k < a.n; ++k) {
      const LayerDev& L = a.layers[k];
      const LayerDev& L1 = a.layers[k + 1];
      __syncthreads();
      for (int t = threadIdx.x; t < L1.N; t += kBlock) g[t] = a.pts[L1.pt_off + t];
      __syncthreads();
      float e[D];
      if (D == 2) {
        if ((k & 1) == 0) {
          const U4 r = philox4x32_10(U4{mc, (uint32_t)(k >> 1), a.contract, 1u}, a.key0, a.key1);
          box_muller(r.x, r.y, eb[0], eb[1]);
          box_muller(r.z, r.w, eb[2], eb[3]);
        }
        e[0] = eb[(k & 1) * 2];
        e[1] = eb[(k & 1) * 2 + 1];
      } else {
        const U4 r = philox4x32_10(U4{mc, (uint32_t)k, a.contract, 1u}, a.key0, a.key1);
        float unused;
        box_muller(r.x, r.y, e[0], e[1]);
        box_muller(r.z, r.w, e[D - 1], unused);
      }
      float y[D];
#pragma unroll
      for (int r = 0; r < D; ++r) {
        float v = L.b[r];
#pragma unroll
        for (int c = 0; c < D; ++c) v = fmaf(L.A[r * D + c], x[c], v);
#pragma unroll
        for (int c = 0; c < D; ++c) v = fmaf(L.T[r * D + c], e[c], v);
        y[r] = v;
      }
      float yq[1][D];
#pragma unroll
      for (int c = 0; c < D; ++c) yq[0][c] = y[c];
      int j;
      argmin_scan<D, 1>(g, L1.N, yq, &j);
      if (live) count_add(a.counts + L.cnt_off + (int64_t)i * L.N1 + j);
      i = j;
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] = y[c];
    }
  }
}

hipError_t launch_zero_i32(int32_t* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = ((count >> 2) + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, count);
  return hipGetLastError();
}

// Allow dynamic LDS beyond the 64 KiB default (gfx950 has 160 KiB per CU).
template <typename F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static dim3 unit_grid(const FwdArgs& a) {
  return a.xcd_map ? dim3((unsigned)(8 * a.units_per_xcd)) : dim3((unsigned)a.units);
}

hipError_t launch_fwd_layer_1d(const FwdArgs& a, hipStream_t s) {
  const size_t lds = sizeof(float) * 2 * (size_t)a.maxP;
  hipError_t e = allow_lds(fwd_layer_1d, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fwd_layer_1d, unit_grid(a), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_fwd_layer_nd(const FwdArgs& a, hipStream_t s) {
  const size_t lds = sizeof(float4) * 2 * (size_t)a.maxN;
  hipError_t e;
  if (a.d == 2) {
    e = allow_lds(fwd_layer_nd<2, 4>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_layer_nd<2, 4>), unit_grid(a), dim3(kBlock), lds, s, a);
  } else {
    e = allow_lds(fwd_layer_nd<3, 4>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_layer_nd<3, 4>), unit_grid(a), dim3(kBlock), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fwd_path(const FwdArgs& a, hipStream_t s) {
  const uint64_t blocks = (a.M + kBlock - 1) / kBlock;
  if (a.d == 1) {
    // midpoints of every layer in LDS when they fit in 64 KiB
    const int in_lds = a.mids_total * 4 <= 65536;
    const size_t lds = in_lds ? sizeof(float) * (size_t)a.mids_total : 0;
    hipLaunchKernelGGL((fwd_path<1>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a, in_lds);
  } else {
    const size_t lds = sizeof(float4) * (size_t)a.maxN;
    if (a.d == 2)
      hipLaunchKernelGGL((fwd_path<2>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a, 0);
    else
      hipLaunchKernelGGL((fwd_path<3>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a, 0);
  }
  return hipGetLastError();
}

}  // namespace qtree
