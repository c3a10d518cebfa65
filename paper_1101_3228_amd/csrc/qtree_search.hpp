// Device-side sample construction and cell search shared by the forward
// kernels and the per-sample diagnostics.
#pragma once
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"

namespace qtree {

// Number of midpoints strictly below x in a sorted array padded with +inf to
// 2^logP entries (2^logP >= N > number of real midpoints).
__device__ __forceinline__ int cell_1d(const float* mids, int logP, float x) {
  int c = 0;
  for (int s = (1 << logP) >> 1; s > 0; s >>= 1) {
    c = (mids[c + s - 1] < x) ? c + s : c;
  }
  return c;
}

// X_k = mu + L z and X_{k+1} = b + A X_k + T eps, row by row, left-to-right
// chains of fused multiply-adds (the AR(1) proposition of Sec. 3).
template <int D>
__device__ __forceinline__ void layer_pair(const LayerDev& L, const float* z, const float* e,
                                           float* x, float* y) {
#pragma unroll
  for (int r = 0; r < D; ++r) {
    float v = L.mu[r];
#pragma unroll
    for (int c = 0; c < D; ++c) v = fmaf(L.L[r * D + c], z[c], v);
    x[r] = v;
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    float v = L.b[r];
#pragma unroll
    for (int c = 0; c < D; ++c) v = fmaf(L.A[r * D + c], x[c], v);
#pragma unroll
    for (int c = 0; c < D; ++c) v = fmaf(L.T[r * D + c], e[c], v);
    y[r] = v;
  }
}

// Argmin over N grid records (g_0..g_{D-1}, h) of h - <x, g>, lowest index on
// ties, for S query points at once.
template <int D, int S>
__device__ __forceinline__ void argmin_scan(const float4* __restrict__ g, int N,
                                            const float (*xs)[D], int* idx) {
  float best[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    best[s] = __builtin_huge_valf();
    idx[s] = 0;
  }
  for (int p = 0; p < N; ++p) {
    const float4 q = g[p];
    const float gc[3] = {q.x, q.y, q.z};
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float key = q.w;
#pragma unroll
      for (int c = 0; c < D; ++c) key = fmaf(-xs[s][c], gc[c], key);
      const bool lt = key < best[s];
      best[s] = lt ? key : best[s];
      idx[s] = lt ? p : idx[s];
    }
  }
}

// The same argmin, by tiles of TL records: a running minimum per tile
// (fminf chains -> v_min3_f32) and only the index of the first tile whose
// minimum is strictly smaller than the best so far; the winning tile is then
// rescanned for the first record whose key equals the minimum.  Bit-identical
// to argmin_scan (same keys, lowest index among the minimal ones).  The
// record array must be padded to a multiple of TL with records whose key is
// +inf for every x (g = 0, h = +inf).
template <int D, int S, int TL>
__device__ __forceinline__ void argmin_scan_tiled(const float4* __restrict__ g, int Npad,
                                                  const float (*xs)[D], int* idx) {
  float best[S];
  int tile[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    best[s] = __builtin_huge_valf();
    tile[s] = 0;
  }
  for (int p0 = 0; p0 < Npad; p0 += TL) {
    float m[S];
#pragma unroll
    for (int s = 0; s < S; ++s) m[s] = __builtin_huge_valf();
#pragma unroll
    for (int q = 0; q < TL; ++q) {
      const float4 r = g[p0 + q];
      const float gc[3] = {r.x, r.y, r.z};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        float key = r.w;
#pragma unroll
        for (int c = 0; c < D; ++c) key = fmaf(-xs[s][c], gc[c], key);
        m[s] = fminf(m[s], key);
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const bool lt = m[s] < best[s];
      best[s] = lt ? m[s] : best[s];
      tile[s] = lt ? p0 : tile[s];
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    int found = tile[s] + TL - 1;
#pragma unroll
    for (int q = TL - 1; q >= 0; --q) {
      const float4 r = g[tile[s] + q];
      const float gc[3] = {r.x, r.y, r.z};
      float key = r.w;
#pragma unroll
      for (int c = 0; c < D; ++c) key = fmaf(-xs[s][c], gc[c], key);
      found = key == best[s] ? tile[s] + q : found;
    }
    idx[s] = found;
  }
}

// Standard normals z (for X_k) and eps (for the innovation) of LAYERWISE
// sample m of layer k.  Philox counter (block, k, contract, tag): d = 1 uses
// block m >> 1 and the Box-Muller pair m & 1; d = 2 block m; d = 3 blocks
// (m, tag 0) and (m, tag 16).
template <int D>
__device__ __forceinline__ void layer_normals(uint32_t key0, uint32_t key1, uint32_t contract,
                                              int k, uint64_t m, float* z, float* e) {
  if (D == 1) {
    const U4 r = philox4x32_10(U4{(uint32_t)(m >> 1), (uint32_t)k, contract, 0u}, key0, key1);
    if (m & 1) box_muller(r.z, r.w, z[0], e[0]);
    else box_muller(r.x, r.y, z[0], e[0]);
  } else if (D == 2) {
    const U4 r = philox4x32_10(U4{(uint32_t)m, (uint32_t)k, contract, 0u}, key0, key1);
    box_muller(r.x, r.y, z[0], z[1]);
    box_muller(r.z, r.w, e[0], e[1]);
  } else {
    const U4 r = philox4x32_10(U4{(uint32_t)m, (uint32_t)k, contract, 0u}, key0, key1);
    box_muller(r.x, r.y, z[0], z[1]);
    box_muller(r.z, r.w, z[2], e[0]);
    const U4 r2 = philox4x32_10(U4{(uint32_t)m, (uint32_t)k, contract, 16u}, key0, key1);
    box_muller(r2.x, r2.y, e[1], e[2]);
  }
}

}  // namespace qtree
