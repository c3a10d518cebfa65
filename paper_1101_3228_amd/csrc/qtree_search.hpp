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

// Breadth-first (Eytzinger) order of the 2^LOGP padded midpoints of a layer:
// node i (1 <= i < 2^LOGP) at depth t = floor(log2 i) holds the sorted
// midpoint (2 (i - 2^t) + 1) 2^(LOGP-t-1) - 1, so binary lifting from the
// root visits the same midpoints as cell_1d.  Nodes of one depth are
// adjacent in LDS: the lanes of a wave at a shallow depth read a few
// consecutive words instead of words one power of two apart (which share a
// bank).  Slot 0 is unused.
template <int LOGP>
__device__ __forceinline__ int bfs_source(int i) {
  const int t = 31 - __clz(i);
  return ((2 * (i - (1 << t)) + 1) << (LOGP - t - 1)) - 1;
}

// cell_1d over a breadth-first LDS copy, the depth fixed at compile time:
// i <- 2 i + (e_i < x) from the root, count = i - 2^LOGP.  The comparison is
// the sign bit of e_i - x, which equals (e_i < x) for every finite x and
// every midpoint that is +inf or finite and not -0 (zero midpoints are stored
// as +0): with denormals kept the difference of two distinct floats never
// rounds to zero, and m - m = +0.  The LDS address a = base + 4 i is carried:
// the child's address is 2 a + (4 b - base), b the sign bit.  A step after
// the load is five vector operations (subtract, arithmetic shift, and, add,
// and one shift-add, the only half-rate one) instead of a compare and a
// select; they form one asm block so that the compiler keeps these forms and
// puts no wait states between them (plain VALU dependences interlock).
template <int LOGP>
__device__ __forceinline__ int cell_1d_bfs(const float* e, float x) {
  typedef __attribute__((address_space(3))) const float lds_float;
  const uint32_t base = (uint32_t)(uintptr_t)(lds_float*)e;
  const uint32_t nbase = vgpr_copy(0u - base);
  uint32_t addr = base + 4;
#pragma unroll
  for (int t = 0; t < LOGP; ++t) {
    const float m = *(lds_float*)(uintptr_t)addr;
    uint32_t tmp;
    asm("v_sub_f32_e32 %[t], %[m], %[x]\n\t"
        "v_ashrrev_i32_e32 %[t], 31, %[t]\n\t"
        "v_and_b32_e32 %[t], 4, %[t]\n\t"
        "v_add_u32_e32 %[t], %[t], %[nb]\n\t"
        "v_lshl_add_u32 %[a], %[a], 1, %[t]"
        : [a] "+v"(addr), [t] "=&v"(tmp)
        : [m] "v"(m), [x] "v"(x), [nb] "v"(nbase));
  }
  return (int)((addr - base) >> 2) - (1 << LOGP);
}

// cell_1d by a guide table: bucket b = (int)clamp(fma(x, scale, shift), 0,
// B - 1) (bmax = B - 1), then c = tab[b] + #{r < K : m[tab[b] + r] < x}.
// Exact when tab[b] counts the midpoints below the first float of bucket b
// and K bounds the midpoints inside any bucket (the host builds both from
// the same float formula), with m padded by K entries of +inf.  The clamp is
// one median-of-three (x is finite, so it equals max then min); each
// comparison is the sign bit of m - x (subtract, shift: full-rate
// operations, where a compare and select issue at half rate).  Written as
// plain arithmetic, the searches of neighbouring samples are free to be
// scheduled together: the compiler issues the table reads of several samples,
// then their paired candidate reads, before the first wait.
template <int K>
__device__ __forceinline__ int cell_1d_guide(const float* m, const uint16_t* tab, float scale,
                                             float shift, float bmax, float x) {
  const float t = __builtin_amdgcn_fmed3f(fmaf(x, scale, shift), 0.0f, bmax);
  const int c0 = tab[(int)t];
  int c = c0;
#pragma unroll
  for (int r = 0; r < K; ++r) c += (int)(__float_as_uint(m[c0 + r] - x) >> 31);
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
  // the records of the next tile are loaded while the current one is
  // scanned (the last iteration reloads its own tile, which stays in bounds)
  float4 cur[TL];
#pragma unroll
  for (int q = 0; q < TL; ++q) cur[q] = g[q];
  for (int p0 = 0; p0 < Npad; p0 += TL) {
    float4 nxt[TL];
    const int pn = p0 + TL < Npad ? p0 + TL : p0;
#pragma unroll
    for (int q = 0; q < TL; ++q) nxt[q] = g[pn + q];
    float m[S];
#pragma unroll
    for (int s = 0; s < S; ++s) m[s] = __builtin_huge_valf();
#pragma unroll
    for (int q = 0; q < TL; ++q) {
      const float4 r = cur[q];
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
#pragma unroll
    for (int q = 0; q < TL; ++q) cur[q] = nxt[q];
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    int found = tile[s] + TL - 1;
    // rolled: unrolled, the loads of every record of every sample's tile
    // would be hoisted together (TL x S float4 registers)
#pragma unroll 1
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

// d = 2 cells by the layer's bucket tables, in two steps so that the row
// loads of many points are in flight together.  A bucket's row (kBucketRow
// uint16, 16-byte aligned) holds its candidate count c in entry 0 and, in
// entries 1..c, every point that can be the FP32 argmin of h - <x, g>
// anywhere in the bucket, in increasing index, then the pad index N to the
// end of its last 8-entry group.  The first minimum over the list is the
// full scan's cell (the lowest index of the minimal key).  Outside the box,
// in a bucket whose candidates did not fit (c = kBucketFull), or in a layer
// without tables, the full scan over the N points decides.
//
// The points are (x, y) pairs in LDS, 8 bytes each, with a pad pair (NaN,
// NaN) at index N: its key is NaN, which never wins a comparison, and the
// lanes that read it share one LDS access.  Consecutive points fall in
// different bank pairs, where 16-byte records would share a quarter of the
// banks (and 12-byte (x, y, h) triples take two reads).  The half norm is
// recomputed as h = (x x + y y) / 2 with one product, one fma and one
// halving, the order in which the records' own half norms are formed, so
// the key is bit for bit the scan's.
__device__ __forceinline__ float half_norm_key(float2 r, float x0, float x1) {
  const float h = 0.5f * fmaf(r.y, r.y, r.x * r.x);
  return fmaf(-x1, r.y, fmaf(-x0, r.x, h));
}

// bucket_rows: the row index of each of S points (-1: full scan) and the
// first 16 bytes of its row (count and candidates 1..7).  Every point loads
// a row (row 0 when it has none, so that the load is not under a branch and
// all S stay in flight); bucket_argmin ignores what a -1 point loaded.
template <int S>
__device__ __forceinline__ void bucket_rows(const LayerDev& L, const uint4* __restrict__ rows,
                                            const float (*xs)[2], int* slot, uint4* w) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float f0 = (xs[s][0] - L.bk_lo[0]) * L.bk_scale[0];
    const float f1 = (xs[s][1] - L.bk_lo[1]) * L.bk_scale[1];
    // false for a layer without tables (bk_B = 0) and for NaN
    const bool in =
        f0 >= 0.0f && f1 >= 0.0f && f0 < (float)L.bk_B[0] && f1 < (float)L.bk_B[1];
    const int r = in ? L.bk_off + (int)f0 * L.bk_B[1] + (int)f1 : 0;
    slot[s] = in ? r : -1;
    w[s] = rows[(int64_t)r * (kBucketRow / 8)];
  }
}

// One 8-entry group of a row: entries e0..7 (candidates or pads).
__device__ __forceinline__ void bucket_group(const float2* __restrict__ g, uint4 w, int e0,
                                             float x0, float x1, float& best, int& idx) {
  const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int e = e0; e < 8; ++e) {
    const int p = (int)((ww[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu);
    const float key = half_norm_key(g[p], x0, x1);
    const bool lt = key < best;
    best = lt ? key : best;
    idx = lt ? p : idx;
  }
}

// bucket_first: the minimum over the first group of each of S points'
// rows, in straight-line code so that the LDS reads of all S points can be
// in flight together.  A point without a row (outside the box) walks pads
// only; a full row's first entries are valid points of the layer, and
// bucket_rest replaces what they give.
template <int S>
__device__ __forceinline__ void bucket_first(const float2* __restrict__ g, int N,
                                             const float (*xs)[2], const int* slot,
                                             const uint4* w, float* best, int* idx) {
  const uint32_t pads = (uint32_t)N | ((uint32_t)N << 16);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const uint4 v = slot[s] >= 0 ? w[s] : make_uint4(pads, pads, pads, pads);
    best[s] = __builtin_huge_valf();
    idx[s] = 0;
    bucket_group(g, v, 1, xs[s][0], xs[s][1], best[s], idx[s]);
  }
}

// bucket_rest: the further groups of rows longer than 7 candidates, and the
// full scan for points outside the box or in a full bucket; idx then holds
// the cells.
template <int S>
__device__ __forceinline__ void bucket_rest(const float2* __restrict__ g, int N,
                                            const uint4* __restrict__ rows,
                                            const float (*xs)[2], const int* slot,
                                            const uint4* w, float* best, int* idx) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int c = slot[s] >= 0 ? (int)(w[s].x & 0xFFFFu) : (int)kBucketFull;
    if (c == (int)kBucketFull) {
      float b = __builtin_huge_valf();
      int bi = 0;
      for (int p = 0; p < N; ++p) {
        const float key = half_norm_key(g[p], xs[s][0], xs[s][1]);
        const bool lt = key < b;
        b = lt ? key : b;
        bi = lt ? p : bi;
      }
      idx[s] = bi;
    } else {
      for (int q = 8; q <= c; q += 8)
        bucket_group(g, rows[(int64_t)slot[s] * (kBucketRow / 8) + (q >> 3)], 0, xs[s][0],
                     xs[s][1], best[s], idx[s]);
    }
  }
}

// bucket_argmin: the cells of the S points whose rows bucket_rows fetched.
template <int S>
__device__ __forceinline__ void bucket_argmin(const float2* __restrict__ g, int N,
                                              const uint4* __restrict__ rows,
                                              const float (*xs)[2], const int* slot,
                                              const uint4* w, int* idx) {
  float best[S];
  bucket_first<S>(g, N, xs, slot, w, best, idx);
  bucket_rest<S>(g, N, rows, xs, slot, w, best, idx);
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
