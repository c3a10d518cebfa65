// Two-pass transition counting for the time-layer parallel estimate
// (Sec. 4, Algorithm III) without device-wide atomics on the hot path.
//
// The paper increments p^k_ij with atomicAdd in global memory (Sec. 3,
// "Updating p^k_ij").  On MI355X a device-scope atomic per sample caps the
// forward step near 2e10 samples/s, an order of magnitude below what the
// sampling and the cell searches sustain, and a count block of N_k x N_{k+1}
// int32 (1 MB at N = 500) does not fit in LDS.  So:
//
//  pass A (fwd_keys_*): a workgroup draws a chunk of kChunk samples of one
//    layer (Philox -> Box-Muller -> AR(1) -> two cell searches, as in the
//    one-pass kernels), forms the flat index key = i N_{k+1} + j, and sorts
//    the keys by tile t = key >> kTileBits with a counting sort in LDS (count
//    per tile, scan, place; 4096-entry tiles keep the LDS counters of a wave
//    apart).  The chunk writes each key as its 16-bit offset inside its
//    16384-entry super tile, tile by tile, with 16-byte stores, plus the
//    segment starts.
//  pass B (count_tiles): one workgroup per (layer, super tile) walks that
//    super tile's segment (four consecutive tiles) in every chunk of the
//    layer, increments a 16384-bin LDS histogram, and stores the super tile
//    into the count block.  Each count is
//    owned by exactly one workgroup, so the store is plain (it also replaces
//    zeroing).  Integer counting makes the order of keys irrelevant.
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"
#include "qtree_search.hpp"

namespace qtree {

namespace {

constexpr int kBlock = 256;
constexpr int kKeys = kChunk / kBlock;  // keys per lane in pass A
constexpr int kCountBlock = 1024;

__device__ __forceinline__ bool unit_of_block_keys(const FwdArgs& a, int& k, int& chunk) {
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

// Counting sort of a chunk's keys by tile, in LDS.  `tcount` holds T + 1
// counters, `cursor` T, `stage` kChunk 16-bit slots.  Phase 1 counts keys
// per tile; the exclusive scan gives each tile's segment start; phase 2
// places every key at its tile's cursor; the staged chunk is then copied to
// its scratch slot with wide stores, and the segment starts with it.
__device__ __forceinline__ void count_keys(const uint32_t* key, uint32_t* tcount) {
#pragma unroll
  for (int e = 0; e < kKeys; ++e)
    if (key[e] != 0xFFFFFFFFu) atomicAdd(&tcount[key[e] >> kTileBits], 1u);
}

// Exclusive scan of tcount[0..T) in place (tcount[T] = total), copied to
// cursor, by wave 0 alone: each lane sums a run of consecutive counters, the
// 64 run sums are scanned with shuffles, then the runs are rewritten.  Must
// sit between two barriers.
__device__ __forceinline__ void scan_tiles(uint32_t* tcount, uint32_t* cursor, int T) {
  if (threadIdx.x >= 64) return;
  const int lane = (int)threadIdx.x;
  const int per = (T + 63) / 64;
  const int t0 = lane * per;
  uint32_t sum = 0;
  for (int t = t0; t < t0 + per && t < T; ++t) sum += tcount[t];
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  uint32_t run = incl - sum;
  for (int t = t0; t < t0 + per && t < T; ++t) {
    const uint32_t v = tcount[t];
    tcount[t] = run;
    cursor[t] = run;
    run += v;
  }
  if (lane == 63) tcount[T] = incl;
}

__device__ __forceinline__ void place_keys(const uint32_t* key, uint32_t* cursor,
                                           uint16_t* stage) {
#pragma unroll
  for (int e = 0; e < kKeys; ++e) {
    if (key[e] != 0xFFFFFFFFu) {
      const uint32_t pos = atomicAdd(&cursor[key[e] >> kTileBits], 1u);
      stage[pos] = (uint16_t)(key[e] & (kSuper - 1));
    }
  }
}

__device__ __forceinline__ void write_chunk(const FwdArgs& a, int k, int c, int T,
                                            const uint32_t* tcount, const uint16_t* stage) {
  uint32_t* seg = a.segs + ((size_t)k * a.chunks + c) * a.seg_stride;
  for (int t = threadIdx.x; t <= T; t += kBlock) seg[t] = tcount[t];
  const uint32_t total = tcount[T];
  uint4* out = reinterpret_cast<uint4*>(a.keys + ((size_t)k * a.chunks + c) * kChunk);
  const uint4* src = reinterpret_cast<const uint4*>(stage);
  const uint32_t vecs = (total + 7) / 8;  // 8 keys per 16-byte store
  for (uint32_t v = threadIdx.x; v < vecs; v += kBlock) out[v] = src[v];
}

}  // namespace

// Pass A, d = 1.  Chunk c of the batch covers the Philox blocks
// [lo/2 + c kChunk/2, lo/2 + (c+1) kChunk/2); sample m = 2 block + h is live
// when it lies in the batch [lo, hi).
__global__ __launch_bounds__(kBlock) void fwd_keys_1d(FwdArgs a) {
  extern __shared__ float lds[];
  int k, c;
  if (!unit_of_block_keys(a, k, c)) return;
  const LayerDev& L0 = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  const int T = L0.tiles;
  float* mk = lds;
  float* mk1 = lds + L0.P;
  // 16-byte aligned staging (it is copied out with 16-byte accesses)
  uint16_t* stage = reinterpret_cast<uint16_t*>(lds + ((L0.P + L1.P + 3) & ~3));
  uint32_t* tcount = reinterpret_cast<uint32_t*>(stage + kChunk);
  uint32_t* cursor = tcount + (T + 1);
  for (int i = threadIdx.x; i < L0.P; i += kBlock) mk[i] = a.mids[L0.aux_off + i];
  for (int i = threadIdx.x; i < L1.P; i += kBlock) mk1[i] = a.mids[L1.aux_off + i];
  for (int t = threadIdx.x; t <= T; t += kBlock) tcount[t] = 0;
  __syncthreads();

  const float mu = L0.mu[0], Lz = L0.L[0], A = L0.A[0], b = L0.b[0], Tk = L0.T[0];
  const int logP0 = L0.logP, logP1 = L1.logP;
  const uint32_t N1 = (uint32_t)L0.N1;
  const uint64_t lo = a.m0, hi = a.m0 + a.M;
  const uint64_t pb = (lo >> 1) + (uint64_t)c * (kChunk / 2);
  uint32_t key[kKeys];
#pragma unroll
  for (int e = 0; e < kKeys / 2; ++e) {
    const uint64_t blk = pb + (uint64_t)e * kBlock + threadIdx.x;
    const U4 r = philox4x32_10(U4{(uint32_t)blk, (uint32_t)k, a.contract, 0u}, a.key0, a.key1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t m = 2 * blk + h;
      const bool live = m >= lo && m < hi;
      float z, eps;
      box_muller(h ? r.z : r.x, h ? r.w : r.y, z, eps);
      const float x = fmaf(Lz, z, mu);
      const float y = fmaf(Tk, eps, fmaf(A, x, b));
      const uint32_t kk = (uint32_t)cell_1d(mk, logP0, x) * N1 + (uint32_t)cell_1d(mk1, logP1, y);
      key[2 * e + h] = live ? kk : 0xFFFFFFFFu;
    }
  }
  count_keys(key, tcount);
  __syncthreads();
  scan_tiles(tcount, cursor, T);
  __syncthreads();
  place_keys(key, cursor, stage);
  __syncthreads();
  write_chunk(a, k, c, T, tcount, stage);
}

// Pass A, d = 2, 3: S samples per lane share each LDS grid read.
template <int D, int S>
__global__ __launch_bounds__(kBlock) void fwd_keys_nd(FwdArgs a) {
  extern __shared__ float4 lds4[];
  int k, c;
  if (!unit_of_block_keys(a, k, c)) return;
  const LayerDev& L0 = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  const int N0 = L0.N, N1 = L0.N1, T = L0.tiles;
  float4* gk = lds4;
  float4* gk1 = lds4 + N0;
  uint16_t* stage = reinterpret_cast<uint16_t*>(lds4 + N0 + N1);
  uint32_t* tcount = reinterpret_cast<uint32_t*>(stage + kChunk);
  uint32_t* cursor = tcount + (T + 1);
  for (int i = threadIdx.x; i < N0; i += kBlock) gk[i] = a.pts[L0.pt_off + i];
  for (int i = threadIdx.x; i < N1; i += kBlock) gk1[i] = a.pts[L1.pt_off + i];
  for (int t = threadIdx.x; t <= T; t += kBlock) tcount[t] = 0;
  __syncthreads();

  const uint64_t lo = a.m0 + (uint64_t)c * kChunk;
  const uint64_t hi = a.m0 + a.M;
  uint32_t key[kKeys];
#pragma unroll
  for (int r = 0; r < kKeys / S; ++r) {
    float xs[S][D], ys[S][D];
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t m = lo + (uint64_t)(r * S + s) * kBlock + threadIdx.x;
      live[s] = m < hi;
      float z[D], e[D];
      layer_normals<D>(a, k, live[s] ? m : a.m0, z, e);
      layer_pair<D>(L0, z, e, xs[s], ys[s]);
    }
    int ii[S], jj[S];
    argmin_scan<D, S>(gk, N0, xs, ii);
    argmin_scan<D, S>(gk1, N1, ys, jj);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t kk = (uint32_t)ii[s] * (uint32_t)N1 + (uint32_t)jj[s];
      key[r * S + s] = live[s] ? kk : 0xFFFFFFFFu;
    }
  }
  count_keys(key, tcount);
  __syncthreads();
  scan_tiles(tcount, cursor, T);
  __syncthreads();
  place_keys(key, cursor, stage);
  __syncthreads();
  write_chunk(a, k, c, T, tcount, stage);
}

// Pass B: workgroup b owns super tile t of layer k (b = tile_off_k + t),
// i.e. tiles [t kTilesPerSuper, (t+1) kTilesPerSuper) whose keys are one
// contiguous segment of every chunk.  Segment bounds of kCountBlock chunks at
// a time are fetched with one load per lane into LDS; each wave then walks
// whole segments, 8 keys per lane per 16-byte load, adding into the
// kSuper-bin LDS histogram.
__global__ __launch_bounds__(kCountBlock) void count_tiles(FwdArgs a) {
  extern __shared__ uint32_t hist[];
  uint32_t* sb = hist + kSuper;
  uint32_t* se = sb + kCountBlock;
  const int b = (int)blockIdx.x;
  int lo = 0, hi = a.n - 1;  // largest k with tile_off_k <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.layers[mid].tile_off <= b) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const LayerDev& L0 = a.layers[k];
  const int t = b - L0.tile_off;
  const int f0 = t * kTilesPerSuper;
  const int f1 = (f0 + kTilesPerSuper) < L0.tiles ? (f0 + kTilesPerSuper) : L0.tiles;
  for (int i = threadIdx.x; i < kSuper; i += kCountBlock) hist[i] = 0;
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const uint32_t* segk = a.segs + (size_t)k * a.chunks * a.seg_stride;
  const uint16_t* keysk = a.keys + (size_t)k * a.chunks * kChunk;
  for (int c0 = 0; c0 < a.chunks; c0 += kCountBlock) {
    __syncthreads();
    const int c = c0 + (int)threadIdx.x;
    if (c < a.chunks) {
      sb[threadIdx.x] = segk[(size_t)c * a.seg_stride + f0];
      se[threadIdx.x] = segk[(size_t)c * a.seg_stride + f1];
    }
    __syncthreads();
    const int cn = (a.chunks - c0) < kCountBlock ? (a.chunks - c0) : kCountBlock;
    // each wave takes kInFlight chunks at a time so that several segment
    // loads are outstanding per lane; 16-byte loads of 8 keys each (a chunk's
    // key block is 16-byte aligned), keys outside [s0, s1) skipped
    constexpr int kWaves = kCountBlock / 64;
    constexpr int kInFlight = 4;
    for (int g = wave * kInFlight; g < cn; g += kWaves * kInFlight) {
      uint32_t s0[kInFlight], s1[kInFlight], v[kInFlight];
      const uint4* kv[kInFlight];
#pragma unroll
      for (int u = 0; u < kInFlight; ++u) {
        const int cc = g + u < cn ? g + u : g;
        s0[u] = g + u < cn ? sb[cc] : 0u;
        s1[u] = g + u < cn ? se[cc] : 0u;
        kv[u] = reinterpret_cast<const uint4*>(keysk + (size_t)(c0 + cc) * kChunk);
        v[u] = (s0[u] >> 3) + lane;
      }
      bool more = true;
      while (more) {
        uint4 w[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u)
          w[u] = v[u] * 8 < s1[u] ? kv[u][v[u]] : make_uint4(0, 0, 0, 0);
        more = false;
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
          if (v[u] * 8 < s1[u]) {
            const uint32_t words[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const uint32_t q = v[u] * 8 + e;
              const uint32_t key = (words[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu;
              if (q >= s0[u] && q < s1[u]) atomicAdd(&hist[key], 1u);
            }
          }
          v[u] += 64;
          more = more || (v[u] * 8 < s1[u]);
        }
        more = __any(more);
      }
    }
  }
  __syncthreads();
  const int64_t total = (int64_t)L0.N * L0.N1;
  const int64_t base = (int64_t)t * kSuper;
  const int bins = (int)((total - base) < kSuper ? (total - base) : kSuper);
  int32_t* dst = a.counts + L0.cnt_off + base;
  if (a.first_batch) {
    for (int i = threadIdx.x; i < bins; i += kCountBlock) dst[i] = (int32_t)hist[i];
  } else {
    for (int i = threadIdx.x; i < bins; i += kCountBlock) dst[i] += (int32_t)hist[i];
  }
}

static dim3 keys_grid(const FwdArgs& a) {
  return a.xcd_map ? dim3((unsigned)(8 * a.units_per_xcd)) : dim3((unsigned)a.units);
}

template <typename F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_fwd_keys(const FwdArgs& a, hipStream_t s) {
  // staged keys + tile counters + cursors + scan partials
  const size_t tiles_bytes =
      sizeof(uint16_t) * kChunk + sizeof(uint32_t) * (size_t)(2 * a.max_tiles + 1);
  hipError_t e;
  if (a.d == 1) {
    const size_t lds = sizeof(float) * (2 * (size_t)a.maxP + 4) + tiles_bytes;
    if ((e = allow_lds(fwd_keys_1d, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(fwd_keys_1d, keys_grid(a), dim3(kBlock), lds, s, a);
  } else if (a.d == 2) {
    const size_t lds = sizeof(float4) * 2 * (size_t)a.maxN + tiles_bytes;
    if ((e = allow_lds(fwd_keys_nd<2, 4>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_keys_nd<2, 4>), keys_grid(a), dim3(kBlock), lds, s, a);
  } else {
    const size_t lds = sizeof(float4) * 2 * (size_t)a.maxN + tiles_bytes;
    if ((e = allow_lds(fwd_keys_nd<3, 4>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_keys_nd<3, 4>), keys_grid(a), dim3(kBlock), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_count_tiles(const FwdArgs& a, hipStream_t s) {
  const size_t lds = sizeof(uint32_t) * (kSuper + 2 * kCountBlock);
  hipError_t e = allow_lds(count_tiles, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(count_tiles, dim3((unsigned)a.total_tiles), dim3(kCountBlock), lds, s, a);
  return hipGetLastError();
}

}  // namespace qtree
