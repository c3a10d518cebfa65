// Two-pass transition counting for the time-layer parallel estimate
// (Sec. 4, Algorithm III) without device-wide atomics on the hot path.
//
// The paper increments p^k_ij with atomicAdd in global memory (Sec. 3,
// "Updating p^k_ij").  On MI355X a device-scope atomic per sample caps the
// forward step near 2e10 samples/s, an order of magnitude below what the
// sampling and the cell searches sustain, and a count block of N_k x N_{k+1}
// int32 (1 MB at N = 500) does not fit in LDS.  So:
//
//  pass A (keys_chunk_*): a workgroup draws a chunk of kChunk samples of one
//    layer (Philox -> Box-Muller -> AR(1) -> two cell searches, as in the
//    one-pass kernels), forms the flat index key = i N_{k+1} + j, and sorts
//    the keys by tile t = key >> kTileBits with a counting sort in LDS (count
//    per tile, scan, place; 4096-entry tiles keep the LDS counters of a wave
//    apart).  The chunk writes each key as its 16-bit offset inside its
//    16384-entry super tile, tile by tile, with 16-byte stores, plus the
//    segment starts.
//  pass B (count_tile): one workgroup per (layer, super tile) walks that
//    super tile's segment (four consecutive tiles) in every chunk of the
//    layer, increments a 16384-bin LDS histogram, and stores the super tile
//    into the count block.  Each count is owned by exactly one workgroup, so
//    the store is plain (it also replaces zeroing).  Integer counting makes
//    the order of keys irrelevant.
//
// The same device routines serve one plan (fwd_keys_*, count_tiles) and a
// batch of contracts (batch_keys, batch_count): the batch kernel takes one
// chunk of a device work list of (contract, layer, chunks) units, longest
// first, per workgroup.
#include "qtree_batch.hpp"
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"
#include "qtree_search.hpp"

namespace qtree {

namespace {

constexpr int kBlock = 256;      // pass-A workgroup, d = 1
constexpr int kBlockNd = 512;    // pass-A workgroup, d >= 2 (two waves per SIMD under one grid pair)
// samples per lane sharing each LDS record read of the d = 2 scan (8: half
// the LDS reads of 4 at 90 VGPRs, 9 % faster on the 2-D workload); d = 3
// keeps 4 (three coordinates per sample)
constexpr int kSamplesNd2 = 8;
// samples per lane of the d = 2 bucketed search (the tuned choice between
// the two): the first-group reads of all 2 S searches of a round are in
// flight together, so S sets the registers and the overlap of LDS reads
constexpr int kBkSamplesLo = 1, kBkSamplesHi = 2;
constexpr int kStageLoads = 4;  // grid records in flight per lane while staging (bucketed)
constexpr int kCountBlock = 1024;
constexpr int kGuideSub = 4;         // sub-counters per tile in the guide kernel's sort
constexpr int kGuideSubTiles = 256;  // ... when a layer has at most this many tiles
// The same for the d >= 2 sort, where the tiles of a wave's keys are few (the
// samples of a row band of the count block share one tile)
constexpr int kNdSub = 4;
constexpr int kNdSubTiles = 256;
__host__ __device__ constexpr int nd_subs(int max_tiles) {
  return max_tiles <= kNdSubTiles ? kNdSub : 1;
}

// One pass-A job: chunk c of the samples [lo, hi) of layer k.
struct KeysJob {
  const LayerDev* L0;
  const LayerDev* L1;
  const float* mids;
  const uint16_t* guide;
  const float4* pts;
  uint32_t key0, key1, contract;
  int k, c;
  uint64_t lo, hi;
  uint16_t* keys;  // kChunk slots of this chunk
  uint32_t* seg;   // T + 1 segment starts of this chunk
  const uint4* bk_rows;  // d = 2 bucket rows (bucketed search only)
  int nd_sub;            // d >= 2: sub-counters per tile in the sort (kNdSub or 1)
};

// One pass-B job: super tile t of a layer whose chunks start at keys / seg.
struct TileJob {
  const LayerDev* L0;
  const uint16_t* keys;
  const uint32_t* seg;
  int seg_stride;
  int chunks;
  int c_lo, c_hi;     // the chunks [c_lo, c_hi) of this job
  int t;
  int32_t* counts_k;  // count block of the layer
  int first;
  int atomic;         // one part of a split super tile: add nonzero bins atomically
};

// Counting sort of a chunk's keys by tile, in LDS.  `tcount` holds T S + 1
// counters, `cursor` T S, `stage` kChunk 16-bit slots.  Each tile has S
// sub-counters, taken by lane & (S - 1): the lanes of a wave whose keys share
// a tile then mostly update different words (same-word LDS atomics of one
// wave are serialized), and tile t's segment is the concatenation of its S
// sub-segments.  Phase 1 counts keys per (tile, sub-counter); the exclusive
// scan gives each its start; phase 2 places every key at its cursor; the
// staged chunk is then copied to its scratch slot with wide stores, and the
// tile segment starts with it.  ALL: every key of the chunk is valid (no
// 0xFFFFFFFF slots).
template <int S>
__device__ __forceinline__ uint32_t sub_counter(uint32_t key) {
  return (key >> kTileBits) * S + (threadIdx.x & (S - 1));
}

template <int KB, bool ALL = false, int S = 1>
__device__ __forceinline__ void count_keys(const uint32_t* key, uint32_t* tcount) {
#pragma unroll
  for (int e = 0; e < kChunk / KB; ++e)
    if (ALL || key[e] != 0xFFFFFFFFu) atomicAdd(&tcount[sub_counter<S>(key[e])], 1u);
}

// Exclusive scan of tcount[0..T) in place (tcount[T] = total), copied to
// cursor: each lane sums a run of consecutive counters, the run sums are
// scanned with shuffles, then the runs are rewritten.  Up to kWaveScan
// counters, wave 0 alone (runs of at most 4); beyond, the whole workgroup,
// the wave sums meeting in LDS (wave 0 alone, with runs of 16 counters at
// the 2-D workload's 980, left the other waves idle behind 32 dependent LDS
// round trips per chunk; at the 1-D workload's 64 counters the extra
// barrier cost more than it saved).  T is uniform over the workgroup; every
// lane must call it, between two barriers.
constexpr int kWaveScan = 256;
template <int KB>
__device__ __forceinline__ void scan_tiles(uint32_t* tcount, uint32_t* cursor, int T) {
  if (T <= kWaveScan) {
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
    return;
  }
  __shared__ uint32_t wave_total[KB / 64];
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (T + KB - 1) / KB;
  const int t0 = tid * per;
  uint32_t sum = 0;
  for (int t = t0; t < t0 + per && t < T; ++t) sum += tcount[t];
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wave_total[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int w = 0; w < KB / 64; ++w) before += w < wave ? wave_total[w] : 0u;
  uint32_t run = before + incl - sum;
  for (int t = t0; t < t0 + per && t < T; ++t) {
    const uint32_t v = tcount[t];
    tcount[t] = run;
    cursor[t] = run;
    run += v;
  }
  if (tid == KB - 1) tcount[T] = before + incl;
}

template <int KB, bool ALL = false, int S = 1>
__device__ __forceinline__ void place_keys(const uint32_t* key, uint32_t* cursor,
                                           uint16_t* stage) {
#pragma unroll
  for (int e = 0; e < kChunk / KB; ++e) {
    if (ALL || key[e] != 0xFFFFFFFFu) {
      const uint32_t pos = atomicAdd(&cursor[sub_counter<S>(key[e])], 1u);
      stage[pos] = (uint16_t)(key[e] & (kSuper - 1));
    }
  }
}

template <int KB, bool ALL = false, int S = 1>
__device__ __forceinline__ void sort_and_write(const KeysJob& j, const uint32_t* key, int T,
                                               uint16_t* stage, uint32_t* tcount,
                                               uint32_t* cursor) {
  count_keys<KB, ALL, S>(key, tcount);
  __syncthreads();
  scan_tiles<KB>(tcount, cursor, T * S);
  __syncthreads();
  place_keys<KB, ALL, S>(key, cursor, stage);
  __syncthreads();
  for (int t = threadIdx.x; t <= T; t += KB) j.seg[t] = tcount[t * S];
  const uint32_t total = tcount[T * S];
  uint4* out = reinterpret_cast<uint4*>(j.keys);
  const uint4* src = reinterpret_cast<const uint4*>(stage);
  const uint32_t vecs = (total + 7) / 8;  // 8 keys per 16-byte store
  for (uint32_t v = threadIdx.x; v < vecs; v += KB) out[v] = src[v];
}

// Pass A, d = 1.  Chunk c covers the Philox blocks
// [lo/2 + c kChunk/2, lo/2 + (c+1) kChunk/2); sample m = 2 block + h is live
// when it lies in [lo, hi).  LOGP > 0: both layers' midpoints are staged in
// breadth-first order, padded with +inf to 2^LOGP entries (LOGP >= the
// layers' own logP), and searched at that fixed depth; the uniform model coefficients and the
// Philox key are kept in vector registers.  LOGP = 0: searches of each
// layer's own depth.
template <int KB, int LOGP>
__device__ __forceinline__ void keys_chunk_1d(const KeysJob& j, float* lds) {
  constexpr int kKeys = kChunk / KB;
  const LayerDev& L0 = *j.L0;
  const LayerDev& L1 = *j.L1;
  const int T = L0.tiles;
  const int P0 = LOGP > 0 ? (1 << LOGP) : L0.P;
  const int P1 = LOGP > 0 ? (1 << LOGP) : L1.P;
  float* mk = lds;
  float* mk1 = lds + P0;
  // 16-byte aligned staging (it is copied out with 16-byte accesses)
  uint16_t* stage = reinterpret_cast<uint16_t*>(lds + ((P0 + P1 + 3) & ~3));
  uint32_t* tcount = reinterpret_cast<uint32_t*>(stage + kChunk);
  uint32_t* cursor = tcount + (T + 1);
  if (LOGP > 0) {
    // breadth-first order, padded with +inf beyond each layer's own midpoints
    constexpr int LG = LOGP > 0 ? LOGP : 1;
    const float inf = __builtin_huge_valf();
    for (int i = threadIdx.x; i < P0; i += KB) {
      const int src = i > 0 ? bfs_source<LG>(i) : 0;
      mk[i] = (i > 0 && src < L0.P) ? j.mids[L0.aux_off + src] : inf;
    }
    for (int i = threadIdx.x; i < P1; i += KB) {
      const int src = i > 0 ? bfs_source<LG>(i) : 0;
      mk1[i] = (i > 0 && src < L1.P) ? j.mids[L1.aux_off + src] : inf;
    }
  } else {
    for (int i = threadIdx.x; i < P0; i += KB) mk[i] = j.mids[L0.aux_off + i];
    for (int i = threadIdx.x; i < P1; i += KB) mk1[i] = j.mids[L1.aux_off + i];
  }
  for (int t = threadIdx.x; t <= T; t += KB) tcount[t] = 0;
  __syncthreads();

  float mu = L0.mu[0], Lz = L0.L[0], A = L0.A[0], b = L0.b[0], Tk = L0.T[0];
  if (LOGP > 0) {
    mu = vgpr_copy(mu);
    Lz = vgpr_copy(Lz);
    A = vgpr_copy(A);
    b = vgpr_copy(b);
    Tk = vgpr_copy(Tk);
  }
  const int logP0 = L0.logP, logP1 = L1.logP;
  const uint32_t N1 = (uint32_t)L0.N1;
  const uint64_t pb = (j.lo >> 1) + (uint64_t)j.c * (kChunk / 2);
  uint32_t key[kKeys];
#pragma unroll
  for (int e = 0; e < kKeys / 2; ++e) {
    const uint64_t blk = pb + (uint64_t)e * KB + threadIdx.x;
    const U4 ctr = U4{(uint32_t)blk, (uint32_t)j.k, j.contract, 0u};
    const U4 r = LOGP > 0 ? philox4x32_10_vk(ctr, j.key0, j.key1)
                          : philox4x32_10(ctr, j.key0, j.key1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t m = 2 * blk + h;
      const bool live = m >= j.lo && m < j.hi;
      float z, eps;
      box_muller(h ? r.z : r.x, h ? r.w : r.y, z, eps);
      const float x = fmaf(Lz, z, mu);
      const float y = fmaf(Tk, eps, fmaf(A, x, b));
      int c0, c1;
      if (LOGP > 0) {
        c0 = cell_1d_bfs<(LOGP > 0 ? LOGP : 1)>(mk, x);
        c1 = cell_1d_bfs<(LOGP > 0 ? LOGP : 1)>(mk1, y);
      } else {
        c0 = cell_1d(mk, logP0, x);
        c1 = cell_1d(mk1, logP1, y);
      }
      const uint32_t kk = (uint32_t)c0 * N1 + (uint32_t)c1;
      key[2 * e + h] = live ? kk : 0xFFFFFFFFu;
    }
  }
  sort_and_write<KB>(j, key, T, stage, tcount, cursor);
}

// Pass A, d = 1, with the guide tables of both layers (every layer's K <= GK):
// the LDS holds the sorted midpoints of both layers (padded with +inf to
// maxP + kGuideKMax entries) and their tables (maxB 16-bit entries each).

struct GuideLds {
  float *mk, *mk1;
  uint16_t *tk, *tk1, *stage;
  uint32_t *tcount, *cursor;
};

__device__ __forceinline__ GuideLds guide_lds(float* lds, int maxP, int maxB, int TS) {
  GuideLds g;
  const int PM = maxP + kGuideKMax;
  g.mk = lds;
  g.mk1 = lds + PM;
  g.tk = reinterpret_cast<uint16_t*>(lds + 2 * PM);
  g.tk1 = g.tk + maxB;
  // 16-byte aligned staging (it is copied out with 16-byte accesses)
  g.stage = reinterpret_cast<uint16_t*>(lds + ((2 * PM + maxB + 3) & ~3));
  g.tcount = reinterpret_cast<uint32_t*>(g.stage + kChunk);
  g.cursor = g.tcount + (TS + 1);
  return g;
}

template <int KB>
__device__ __forceinline__ void guide_stage(const KeysJob& j, const GuideLds& g, int maxP) {
  const LayerDev& L0 = *j.L0;
  const LayerDev& L1 = *j.L1;
  const int PM = maxP + kGuideKMax;
  const float inf = __builtin_huge_valf();
  for (int i = threadIdx.x; i < PM; i += KB) {
    g.mk[i] = i < L0.P ? j.mids[L0.aux_off + i] : inf;
    g.mk1[i] = i < L1.P ? j.mids[L1.aux_off + i] : inf;
  }
  for (int i = threadIdx.x; i < L0.gt_B; i += KB) g.tk[i] = j.guide[L0.gt_off + i];
  for (int i = threadIdx.x; i < L1.gt_B; i += KB) g.tk1[i] = j.guide[L1.gt_off + i];
}

// The keys of one chunk, whose samples are m0 + [0, kChunk) with
// m0 = 2 pb: sample 2 (pb + e KB + lane) + h is key slot 2 e + h of the lane.
// Every slot gets its key; the chunks at the ends of [lo, hi) then mark
// their dead slots (guide_chunk).  The Philox key and the coefficients are
// copied to vector registers once per chunk.
template <int KB, int GK>
__device__ __forceinline__ void guide_keys(const KeysJob& j, const GuideLds& g,
                                           uint32_t (&key)[kChunk / KB]) {
  constexpr int kKeys = kChunk / KB;
  const LayerDev& L0 = *j.L0;
  const LayerDev& L1 = *j.L1;
  const float mu = vgpr_copy(L0.mu[0]), Lz = vgpr_copy(L0.L[0]), A = vgpr_copy(L0.A[0]);
  const float b = vgpr_copy(L0.b[0]), Tk = vgpr_copy(L0.T[0]);
  const float s0 = vgpr_copy(L0.gt_scale), h0 = vgpr_copy(L0.gt_shift);
  const float s1 = vgpr_copy(L1.gt_scale), h1 = vgpr_copy(L1.gt_shift);
  const uint32_t k0 = vgpr_copy(j.key0), k1 = vgpr_copy(j.key1);
  const float bm0 = (float)(L0.gt_B - 1), bm1 = (float)(L1.gt_B - 1);
  const uint32_t N1 = (uint32_t)L0.N1;
  // the low word of the chunk's first Philox block (the counter's word 0)
  const uint32_t pb = (uint32_t)((j.lo >> 1) + (uint64_t)j.c * (kChunk / 2));
  const uint32_t lane = threadIdx.x;
#pragma unroll
  for (int e = 0; e < kKeys / 2; ++e) {
    const U4 r = philox4x32_10(U4{pb + (uint32_t)(e * KB) + lane, (uint32_t)j.k, j.contract, 0u},
                               k0, k1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float z, eps;
      box_muller(h ? r.z : r.x, h ? r.w : r.y, z, eps);
      const float x = fmaf(Lz, z, mu);
      const float y = fmaf(Tk, eps, fmaf(A, x, b));
      const int c0 = cell_1d_guide<GK>(g.mk, g.tk, s0, h0, bm0, x);
      const int c1 = cell_1d_guide<GK>(g.mk1, g.tk1, s1, h1, bm1, y);
      key[2 * e + h] = (uint32_t)c0 * N1 + (uint32_t)c1;
    }
  }
}

template <int KB, int GK, int S>
__device__ __forceinline__ void guide_chunk(const KeysJob& j, const GuideLds& g) {
  const int T = j.L0->tiles;
  for (int t = threadIdx.x; t <= T * S; t += KB) g.tcount[t] = 0;
  __syncthreads();
  const uint64_t m0 = 2 * ((j.lo >> 1) + (uint64_t)j.c * (kChunk / 2));
  uint32_t key[kChunk / KB];
  guide_keys<KB, GK>(j, g, key);
  if (m0 >= j.lo && m0 + kChunk <= j.hi) {
    sort_and_write<KB, true, S>(j, key, T, g.stage, g.tcount, g.cursor);
  } else {
    // slot 2 e + h holds sample m0 + rel, rel = 2 (e KB + lane) + h; it is
    // live when rel - rlo < rhi - rlo (unsigned), [rlo, rhi) = [lo, hi) - m0
    // clamped to [0, kChunk]
    const uint64_t lo = j.lo > m0 ? j.lo - m0 : 0;
    const uint64_t hi = j.hi > m0 ? j.hi - m0 : 0;
    const uint32_t rlo = (uint32_t)(lo < kChunk ? lo : kChunk);
    const uint32_t rhi = (uint32_t)(hi < kChunk ? hi : kChunk);
#pragma unroll
    for (int e = 0; e < kChunk / KB / 2; ++e)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t rel = 2u * ((uint32_t)(e * KB) + threadIdx.x) + (uint32_t)h;
        if (rel - rlo >= rhi - rlo) key[2 * e + h] = 0xFFFFFFFFu;
      }
    sort_and_write<KB, false, S>(j, key, T, g.stage, g.tcount, g.cursor);
  }
}

// Pass A, d = 2, 3: S samples per lane share each LDS grid read, in
// kChunk / (KB S) rounds whose keys stay in registers.  The grid scans take
// tiles of kScanTile records, the padding unit, loaded one tile ahead: one
// compare and two selects per tile and sample for the running best, then a
// rescan of the winning tile (with 4-record tiles that bookkeeping was ~a
// third of the scan's issue time; 8 records: 5 % faster; tiles of 16 and
// groups of 2 or 4 tiles per running-best update: 2.5 %, 3.4 % and 20 %
// slower at N = 2000).
template <int D, int S, int KB, bool BK = false>
__device__ __forceinline__ void keys_chunk_nd(const KeysJob& j, float4* lds4) {
  constexpr int kKeys = kChunk / KB;
  constexpr int kNdTile = kScanTile;
  const LayerDev& L0 = *j.L0;
  const LayerDev& L1 = *j.L1;
  const int N0 = L0.N, N1 = L0.N1, T = L0.tiles;
  // both grids padded to whole scan tiles with records whose key is +inf
  const int P0 = (N0 + kScanTile - 1) / kScanTile * kScanTile;
  const int P1 = (N1 + kScanTile - 1) / kScanTile * kScanTile;
  // the scan: 16-byte records (x, .., h); the bucketed search: (x, y)
  // pairs and the pad pair at N, each layer's block a whole number of 16
  // bytes
  constexpr bool kXY = BK && D == 2;
  const int Q0 = kXY ? (N0 + 2) / 2 : P0, Q1 = kXY ? (N1 + 2) / 2 : P1;
  float4* gk = lds4;
  float4* gk1 = lds4 + Q0;
  float2* xy0 = reinterpret_cast<float2*>(gk);
  float2* xy1 = reinterpret_cast<float2*>(gk1);
  uint16_t* stage = reinterpret_cast<uint16_t*>(lds4 + Q0 + Q1);
  uint32_t* tcount = reinterpret_cast<uint32_t*>(stage + kChunk);
  uint32_t* cursor = tcount + (T + 1);
  if constexpr (kXY) {
    // kStageLoads records of each layer in flight per lane
    const float2 nan2 = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    const int Nm = N0 > N1 ? N0 : N1;
    for (int i0 = threadIdx.x; i0 <= Nm; i0 += KB * kStageLoads) {
      float4 r0[kStageLoads], r1[kStageLoads];
#pragma unroll
      for (int u = 0; u < kStageLoads; ++u) {
        const int i = i0 + u * KB;
        r0[u] = i < N0 ? j.pts[L0.pt_off + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        r1[u] = i < N1 ? j.pts[L1.pt_off + i] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kStageLoads; ++u) {
        const int i = i0 + u * KB;
        if (i <= N0) xy0[i] = i < N0 ? make_float2(r0[u].x, r0[u].y) : nan2;
        if (i <= N1) xy1[i] = i < N1 ? make_float2(r1[u].x, r1[u].y) : nan2;
      }
    }
  } else {
    const float4 pad = make_float4(0.f, 0.f, 0.f, __builtin_huge_valf());
    for (int i = threadIdx.x; i < P0; i += KB) gk[i] = i < N0 ? j.pts[L0.pt_off + i] : pad;
    for (int i = threadIdx.x; i < P1; i += KB) gk1[i] = i < N1 ? j.pts[L1.pt_off + i] : pad;
  }
  for (int t = threadIdx.x; t <= T * j.nd_sub; t += KB) tcount[t] = 0;
  __syncthreads();

  const uint64_t lo = j.lo + (uint64_t)j.c * kChunk;
  uint32_t key[kKeys];
#pragma unroll
  for (int e = 0; e < kKeys; ++e) key[e] = 0xFFFFFFFFu;
#pragma unroll 1
  for (int r = 0; r < kKeys / S; ++r) {
    float xs[S][D], ys[S][D];
    bool live[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t m = lo + (uint64_t)(r * S + s) * KB + threadIdx.x;
      live[s] = m < j.hi;
      float z[D], e[D];
      layer_normals<D>(j.key0, j.key1, j.contract, j.k, live[s] ? m : j.lo, z, e);
      layer_pair<D>(L0, z, e, xs[s], ys[s]);
    }
    int ii[S], jj[S];
    if constexpr (BK && D == 2) {
      // each sample's own bucket list (the same cells as the full scan); the
      // rows of all 2 S searches are fetched before the first is walked
      int sx[S], sy[S];
      uint4 wx[S], wy[S];
      bucket_rows<S>(L0, j.bk_rows, xs, sx, wx);
      bucket_rows<S>(L1, j.bk_rows, ys, sy, wy);
      float bx[S], by[S];
      bucket_first<S>(xy0, N0, xs, sx, wx, bx, ii);
      bucket_first<S>(xy1, N1, ys, sy, wy, by, jj);
      bucket_rest<S>(xy0, N0, j.bk_rows, xs, sx, wx, bx, ii);
      bucket_rest<S>(xy1, N1, j.bk_rows, ys, sy, wy, by, jj);
    } else {
      argmin_scan_tiled<D, S, kNdTile>(gk, P0, xs, ii);
      argmin_scan_tiled<D, S, kNdTile>(gk1, P1, ys, jj);
    }
    // the round is not unrolled, so its keys go to fixed registers by a
    // uniform select (a dynamic index would put the array in scratch)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t kk = (uint32_t)ii[s] * (uint32_t)N1 + (uint32_t)jj[s];
      const uint32_t v = live[s] ? kk : 0xFFFFFFFFu;
#pragma unroll
      for (int q = 0; q < kKeys / S; ++q) key[q * S + s] = q == r ? v : key[q * S + s];
    }
  }
  // tcount holds T nd_sub + 1 counters and cursor T nd_sub; a chunk inside
  // [lo, hi) has no dead slots
  const bool all = lo + kChunk <= j.hi;
  if (j.nd_sub == kNdSub) {
    uint32_t* cur = tcount + (T * kNdSub + 1);
    if (all) sort_and_write<KB, true, kNdSub>(j, key, T, stage, tcount, cur);
    else sort_and_write<KB, false, kNdSub>(j, key, T, stage, tcount, cur);
  } else {
    if (all) sort_and_write<KB, true>(j, key, T, stage, tcount, cursor);
    else sort_and_write<KB, false>(j, key, T, stage, tcount, cursor);
  }
}

// Pass B for one super tile: tiles [t kTilesPerSuper, (t+1) kTilesPerSuper)
// are one contiguous segment of every chunk, walked with 16-byte loads of 8
// keys (a chunk's key block is 16-byte aligned) into the kSuper-bin LDS
// histogram; keys outside [s0, s1) are skipped.  Long segments (a layer of
// few super tiles): segment bounds of kCountBlock chunks at a time are
// fetched with one load per lane into LDS, then each wave walks kInFlight
// segments at once, 8 keys per lane.  Short segments (under kShortSegment
// keys on average, a layer of many super tiles, where a wave would leave
// most lanes idle): each lane walks whole segments of its own chunks, two
// loads at a time.
constexpr int kShortSegment = 64;
__device__ __forceinline__ void count_tile(const TileJob& j, uint32_t* hist, uint32_t* sb,
                                           uint32_t* se) {
  const LayerDev& L0 = *j.L0;
  const int f0 = j.t * kTilesPerSuper;
  const int f1 = (f0 + kTilesPerSuper) < L0.tiles ? (f0 + kTilesPerSuper) : L0.tiles;
  for (int i = threadIdx.x; i < kSuper; i += kCountBlock) hist[i] = 0;
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  constexpr int kWaves = kCountBlock / 64;
  constexpr int kInFlight = 4;
  const int64_t supers = ((int64_t)L0.N * L0.N1 + kSuper - 1) / kSuper;
  const bool lanes = (int64_t)kChunk < (int64_t)kShortSegment * supers;
  if (lanes) {
    __syncthreads();  // the cleared histogram
    for (int c = j.c_lo + (int)threadIdx.x; c < j.c_hi; c += kCountBlock) {
      const uint32_t s0 = j.seg[(size_t)c * j.seg_stride + f0];
      const uint32_t s1 = j.seg[(size_t)c * j.seg_stride + f1];
      const uint4* kv = reinterpret_cast<const uint4*>(j.keys + (size_t)c * kChunk);
      for (uint32_t v = s0 >> 3; v * 8 < s1; v += 2) {
        const uint4 w0 = kv[v];
        const uint4 w1 = (v + 1) * 8 < s1 ? kv[v + 1] : make_uint4(0, 0, 0, 0);
        const uint32_t words[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const uint32_t q = v * 8 + e;
          const uint32_t key = (words[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu;
          if (q >= s0 && q < s1) atomicAdd(&hist[key], 1u);
        }
      }
    }
  }
  for (int c0 = j.c_lo; !lanes && c0 < j.c_hi; c0 += kCountBlock) {
    __syncthreads();
    const int c = c0 + (int)threadIdx.x;
    if (c < j.c_hi) {
      sb[threadIdx.x] = j.seg[(size_t)c * j.seg_stride + f0];
      se[threadIdx.x] = j.seg[(size_t)c * j.seg_stride + f1];
    }
    __syncthreads();
    const int cn = (j.c_hi - c0) < kCountBlock ? (j.c_hi - c0) : kCountBlock;
    for (int g = wave * kInFlight; g < cn; g += kWaves * kInFlight) {
      uint32_t s0[kInFlight], s1[kInFlight], v[kInFlight];
      const uint4* kv[kInFlight];
#pragma unroll
      for (int u = 0; u < kInFlight; ++u) {
        const int cc = g + u < cn ? g + u : g;
        s0[u] = g + u < cn ? sb[cc] : 0u;
        s1[u] = g + u < cn ? se[cc] : 0u;
        kv[u] = reinterpret_cast<const uint4*>(j.keys + (size_t)(c0 + cc) * kChunk);
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
  const int64_t base = (int64_t)j.t * kSuper;
  const int bins = (int)((total - base) < kSuper ? (total - base) : kSuper);
  int32_t* dst = j.counts_k + base;
  if (j.atomic) {
    for (int i = threadIdx.x; i < bins; i += kCountBlock)
      if (hist[i] != 0u) atomicAdd(&dst[i], (int32_t)hist[i]);
  } else if (j.first) {
    for (int i = threadIdx.x; i < bins; i += kCountBlock) dst[i] = (int32_t)hist[i];
  } else {
    for (int i = threadIdx.x; i < bins; i += kCountBlock) dst[i] += (int32_t)hist[i];
  }
}

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
  const int kl = u / a.chunks;
  chunk = u - kl * a.chunks;
  k = a.layer0 + kl;
  return true;
}

__device__ __forceinline__ KeysJob plan_job(const FwdArgs& a, int k, int c) {
  KeysJob j;
  j.L0 = &a.layers[k];
  j.L1 = &a.layers[k + 1];
  j.mids = a.mids;
  j.guide = a.guide;
  j.pts = a.pts;
  j.key0 = a.key0;
  j.key1 = a.key1;
  j.contract = a.contract;
  j.k = k;
  j.c = c;
  j.lo = a.m0;
  j.hi = a.m0 + a.M;
  j.keys = a.keys + ((size_t)k * a.chunks + c) * kChunk;
  j.seg = a.segs + ((size_t)k * a.chunks + c) * a.seg_stride;
  j.bk_rows = a.bk_rows;
  j.nd_sub = nd_subs(a.max_tiles);
  return j;
}

}  // namespace

// ------------------------------------------------------------- one plan

template <int LOGP>
__global__ __launch_bounds__(kBlock) void fwd_keys_1d(FwdArgs a) {
  extern __shared__ float lds[];
  int k, c;
  if (!unit_of_block_keys(a, k, c)) return;
  keys_chunk_1d<kBlock, LOGP>(plan_job(a, k, c), lds);
}

template <int GK, int S>
__global__ __launch_bounds__(kBlock) void fwd_keys_1d_guide(FwdArgs a) {
  extern __shared__ float lds[];
  int k, c;
  if (!unit_of_block_keys(a, k, c)) return;
  const KeysJob j = plan_job(a, k, c);
  const GuideLds g = guide_lds(lds, a.maxP, a.gt_Bmax, a.layers[k].tiles * S);
  guide_stage<kBlock>(j, g, a.maxP);
  guide_chunk<kBlock, GK, S>(j, g);
}

template <int D, int S, bool BK = false>
__global__ __launch_bounds__(kBlockNd) void fwd_keys_nd(FwdArgs a) {
  extern __shared__ float4 lds4[];
  int k, c;
  if (!unit_of_block_keys(a, k, c)) return;
  keys_chunk_nd<D, S, kBlockNd, BK>(plan_job(a, k, c), lds4);
}

// The bucketed search with one sample per lane and round, held to 80 VGPRs
// (six waves per SIMD): with its smaller LDS, three workgroups per CU.
__global__ __launch_bounds__(kBlockNd) __attribute__((amdgpu_waves_per_eu(6)))
void fwd_keys_nd_bk1(FwdArgs a) {
  extern __shared__ float4 lds4[];
  int k, c;
  if (!unit_of_block_keys(a, k, c)) return;
  keys_chunk_nd<2, kBkSamplesLo, kBlockNd, true>(plan_job(a, k, c), lds4);
}

// Workgroup b owns histogram unit tile0 + u (super tile t of layer k, or
// one part of it).  With the XCD map, workgroup b runs on XCD b mod 8 and
// takes unit u = (b mod 8) per + b / 8: consecutive units -- the super tiles
// of one layer, whose key segments share cache lines in every chunk -- run on
// one XCD and meet those lines in its L2.
__global__ __launch_bounds__(kCountBlock) void count_tiles(FwdArgs a) {
  extern __shared__ uint32_t hist[];
  int u = (int)blockIdx.x;
  if (a.xcd_map) {
    const int per = (a.total_tiles + 7) / 8;
    const int slot = (int)blockIdx.x >> 3;
    if (slot >= per) return;
    u = ((int)blockIdx.x & 7) * per + slot;
    if (u >= a.total_tiles) return;
  }
  const int b = a.tile0 + u;
  int lo = 0, hi = a.n - 1;  // largest k with unit_off_k <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.layers[mid].unit_off <= b) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  TileJob j;
  j.L0 = &a.layers[k];
  j.keys = a.keys + (size_t)k * a.chunks * kChunk;
  j.seg = a.segs + (size_t)k * a.chunks * a.seg_stride;
  j.seg_stride = a.seg_stride;
  j.chunks = a.chunks;
  // unit = super tile * split + part; part p takes chunks [p C / split, (p+1) C / split)
  const int split = a.layers[k].split > 1 ? a.layers[k].split : 1;
  const int r = b - a.layers[k].unit_off;
  j.t = r / split;
  const int part = r - j.t * split;
  j.c_lo = (int)((int64_t)a.chunks * part / split);
  j.c_hi = (int)((int64_t)a.chunks * (part + 1) / split);
  j.counts_k = a.counts + a.layers[k].cnt_off;
  j.first = a.first_batch;
  j.atomic = split > 1;
  count_tile(j, hist, hist + kSuper, hist + kSuper + kCountBlock);
}

// ------------------------------------------------------------- a batch

// Pass A over a work list of (contract, layer, chunk range) units sorted by
// decreasing cost: workgroup b takes chunk b of the list (the chunks of unit
// u are [chunk_off[u], chunk_off[u + 1])), so the costly units are dispatched
// first.  One workgroup per chunk, as in the single-plan kernels, keeps the
// register allocation of the chunk routine alone (a persistent claim loop
// around it held ~40 more).  One launch takes the 1-D units (256 lanes),
// another the d >= 2 units (512 lanes under one grid pair).
template <int KB, typename Body>
__device__ __forceinline__ void batch_loop(const BatchArgs& a, Body body) {
  const int b = (int)blockIdx.x;
  const int* chunk_off = as_global(a.chunk_off);
  int lo = 0, hi = a.n_units - 1;  // largest u with chunk_off[u] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chunk_off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int u = lo;
  const BatchUnit U = as_global(a.units)[u];
  const BatchContract& C = as_global(a.contracts)[U.c];
  {
    const int c = U.chunk0 + (b - chunk_off[u]);
    {
      KeysJob j;
      const LayerDev* layers = as_global(C.layers);
      j.L0 = &layers[U.k];
      j.L1 = &layers[U.k + 1];
      j.mids = as_global(C.mids);
      j.guide = as_global(C.guide);
      j.pts = as_global(C.pts);
      j.key0 = C.key0;
      j.key1 = C.key1;
      j.contract = C.contract;
      j.k = U.k;
      j.c = c;
      j.lo = 0;
      j.hi = C.M;
      j.keys = as_global(a.keys) + ((size_t)C.chunk_base + (size_t)U.k * C.chunks + c) * kChunk;
      j.seg = as_global(a.segs) + (size_t)C.seg_base +
              ((size_t)U.k * C.chunks + c) * (size_t)C.seg_stride;
      j.bk_rows = as_global(C.bk_rows);
      j.nd_sub = a.sub;
      body(C, j);
    }
  }
}

// LG > 0: every unit is searched at depth LG (the largest padded midpoint
// count of the batch's 1-D contracts; shallower layers are padded with +inf).
// One depth per launch: instances switched inside one kernel would share one
// register allocation (the union of their live ranges).
template <int LG>
__global__ __launch_bounds__(kBlock) void batch_keys_1d(BatchArgs a) {
  extern __shared__ float lds[];
  batch_loop<kBlock>(a, [&](const BatchContract&, const KeysJob& j) {
    keys_chunk_1d<kBlock, LG>(j, lds);
  });
}

// The same with guide tables (the chunk routine of fwd_keys_1d_guide).
template <int GK, int S>
__global__ __launch_bounds__(kBlock) void batch_keys_1d_guide(BatchArgs a) {
  extern __shared__ float lds[];
  batch_loop<kBlock>(a, [&](const BatchContract&, const KeysJob& j) {
    const GuideLds g = guide_lds(lds, a.maxP, a.gt_Bmax, j.L0->tiles * S);
    guide_stage<kBlock>(j, g, a.maxP);
    guide_chunk<kBlock, GK, S>(j, g);
  });
}

template <int DMAX, int S2, bool BK>
__device__ __forceinline__ void batch_keys_nd_body(const BatchArgs& a) {
  extern __shared__ float4 lds4[];
  batch_loop<kBlockNd>(a, [&](const BatchContract& C, const KeysJob& j) {
    if (DMAX < 3 || C.d == 2) keys_chunk_nd<2, S2, kBlockNd, BK>(j, lds4);
    else keys_chunk_nd<3, 4, kBlockNd>(j, lds4);
  });
}

template <int DMAX, int S2>
__global__ __launch_bounds__(kBlockNd) void batch_keys_nd(BatchArgs a) {
  batch_keys_nd_body<DMAX, S2, false>(a);
}

// The bucketed d = 2 search, held to 128 VGPRs (four waves per SIMD) so that
// two workgroups share a CU: the contract table's registers otherwise leave
// room for one.
template <int S2>
__global__ __launch_bounds__(kBlockNd) __attribute__((amdgpu_waves_per_eu(4)))
void batch_keys_nd_bk(BatchArgs a) {
  batch_keys_nd_body<2, S2, true>(a);
}

// One sample per lane and round, held to 80 VGPRs (six waves per SIMD): with
// the pairs-only LDS block, three workgroups per CU.
__global__ __launch_bounds__(kBlockNd) __attribute__((amdgpu_waves_per_eu(6)))
void batch_keys_nd_bk1(BatchArgs a) {
  batch_keys_nd_body<2, kBkSamplesLo, true>(a);
}

// Pass B of a batch: workgroup b handles tile record b.
__global__ __launch_bounds__(kCountBlock) void batch_count(BatchArgs a) {
  extern __shared__ uint32_t hist[];
  const BatchTile T = as_global(a.tiles)[blockIdx.x];
  const BatchContract& C = as_global(a.contracts)[T.c];
  TileJob j;
  j.L0 = &as_global(C.layers)[T.k];
  j.keys = as_global(a.keys) + ((size_t)C.chunk_base + (size_t)T.k * C.chunks) * kChunk;
  j.seg = as_global(a.segs) + (size_t)C.seg_base + (size_t)T.k * C.chunks * (size_t)C.seg_stride;
  j.seg_stride = C.seg_stride;
  j.chunks = C.chunks;
  j.c_lo = 0;
  j.c_hi = C.chunks;
  j.atomic = 0;
  j.t = T.t;
  j.counts_k = as_global(C.counts) + j.L0->cnt_off;
  j.first = 1;
  count_tile(j, hist, hist + kSuper, hist + kSuper + kCountBlock);
}


// ------------------------------------------------------------- launchers

static dim3 keys_grid(const FwdArgs& a) {
  return a.xcd_map ? dim3((unsigned)(8 * a.units_per_xcd)) : dim3((unsigned)a.units);
}

template <typename F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int guide_sub_counters(int max_tiles) { return max_tiles <= kGuideSubTiles ? kGuideSub : 1; }

int nd_sub_counters(int max_tiles) { return nd_subs(max_tiles); }

size_t keys_lds_1d_guide(int maxP, int maxB, int max_tiles) {
  const size_t words = (2 * (size_t)(maxP + kGuideKMax) + (size_t)maxB + 3) & ~(size_t)3;
  const size_t ts = (size_t)max_tiles * guide_sub_counters(max_tiles);
  return sizeof(float) * words + sizeof(uint16_t) * kChunk + sizeof(uint32_t) * (2 * ts + 1);
}

size_t keys_lds_1d(int maxP, int max_tiles) {
  return sizeof(float) * (2 * (size_t)maxP + 4) + sizeof(uint16_t) * kChunk +
         sizeof(uint32_t) * (size_t)(2 * max_tiles + 1);
}

size_t keys_lds_nd(int maxN, int max_tiles) {
  const size_t ts = (size_t)max_tiles * nd_subs(max_tiles);
  return sizeof(float4) * 2 * (size_t)(maxN + kScanTile) + sizeof(uint16_t) * kChunk +
         sizeof(uint32_t) * (2 * ts + 1);
}

// The bucketed d = 2 search stages (x, y) pairs and a pad pair per layer, a
// whole number of 16 bytes each: a third less LDS than the scan's records,
// so a CU holds three workgroups where their registers allow.
size_t keys_lds_nd_bk(int maxN, int max_tiles) {
  const size_t ts = (size_t)max_tiles * nd_subs(max_tiles);
  return sizeof(float4) * 2 * (size_t)((maxN + 2) / 2) + sizeof(uint16_t) * kChunk +
         sizeof(uint32_t) * (2 * ts + 1);
}

hipError_t launch_fwd_keys(const FwdArgs& a, hipStream_t s) {
  hipError_t e;
  if (a.d == 1 && a.gt_Kmax >= 0) {
    // guide tables: one instance per bound K on the midpoints a bucket adds
    const size_t lds = keys_lds_1d_guide(a.maxP, a.gt_Bmax, a.max_tiles);
    const FwdArgs& g = a;
    switch (a.gt_Kmax) {
#define QTREE_KEYS_1D_GUIDE(K, GK)                                                        \
  case K:                                                                                 \
    if (guide_sub_counters(a.max_tiles) == kGuideSub) {                                   \
      if ((e = allow_lds(fwd_keys_1d_guide<GK, kGuideSub>, lds)) != hipSuccess) return e; \
      hipLaunchKernelGGL((fwd_keys_1d_guide<GK, kGuideSub>), keys_grid(g), dim3(kBlock),  \
                         lds, s, g);                                                      \
    } else {                                                                              \
      if ((e = allow_lds(fwd_keys_1d_guide<GK, 1>, lds)) != hipSuccess) return e;         \
      hipLaunchKernelGGL((fwd_keys_1d_guide<GK, 1>), keys_grid(g), dim3(kBlock), lds, s,  \
                         g);                                                              \
    }                                                                                     \
    break;
      QTREE_KEYS_1D_GUIDE(0, 1) QTREE_KEYS_1D_GUIDE(1, 1) QTREE_KEYS_1D_GUIDE(2, 2)
      QTREE_KEYS_1D_GUIDE(3, 3) QTREE_KEYS_1D_GUIDE(4, 4)
#undef QTREE_KEYS_1D_GUIDE
      default:
        return hipErrorInvalidValue;
    }
  } else if (a.d == 1) {
    // one instance per search depth: the plan's largest padded midpoint count
    const size_t lds = keys_lds_1d(a.maxP, a.max_tiles);
    switch (a.maxP) {
#define QTREE_KEYS_1D(LG)                                                              \
  case 1 << LG:                                                                        \
    if ((e = allow_lds(fwd_keys_1d<LG>, lds)) != hipSuccess) return e;                 \
    hipLaunchKernelGGL(fwd_keys_1d<LG>, keys_grid(a), dim3(kBlock), lds, s, a);        \
    break;
      QTREE_KEYS_1D(1) QTREE_KEYS_1D(2) QTREE_KEYS_1D(3) QTREE_KEYS_1D(4) QTREE_KEYS_1D(5)
      QTREE_KEYS_1D(6) QTREE_KEYS_1D(7) QTREE_KEYS_1D(8) QTREE_KEYS_1D(9) QTREE_KEYS_1D(10)
      QTREE_KEYS_1D(11) QTREE_KEYS_1D(12) QTREE_KEYS_1D(13)
#undef QTREE_KEYS_1D
      default:
        if ((e = allow_lds(fwd_keys_1d<0>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(fwd_keys_1d<0>, keys_grid(a), dim3(kBlock), lds, s, a);
    }
  } else if (a.d == 2 && a.bucketed && a.nd_samples == 4) {
    const size_t lds = keys_lds_nd_bk(a.maxN, a.max_tiles);
    if ((e = allow_lds(fwd_keys_nd_bk1, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(fwd_keys_nd_bk1, keys_grid(a), dim3(kBlockNd), lds, s, a);
  } else if (a.d == 2 && a.bucketed) {
    const size_t lds = keys_lds_nd_bk(a.maxN, a.max_tiles);
    if ((e = allow_lds(fwd_keys_nd<2, kBkSamplesHi, true>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_keys_nd<2, kBkSamplesHi, true>), keys_grid(a), dim3(kBlockNd), lds, s,
                       a);
  } else if (a.d == 2 && a.nd_samples == 4) {
    const size_t lds = keys_lds_nd(a.maxN, a.max_tiles);
    if ((e = allow_lds(fwd_keys_nd<2, 4>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_keys_nd<2, 4>), keys_grid(a), dim3(kBlockNd), lds, s, a);
  } else if (a.d == 2) {
    const size_t lds = keys_lds_nd(a.maxN, a.max_tiles);
    if ((e = allow_lds(fwd_keys_nd<2, kSamplesNd2>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_keys_nd<2, kSamplesNd2>), keys_grid(a), dim3(kBlockNd), lds, s, a);
  } else {
    const size_t lds = keys_lds_nd(a.maxN, a.max_tiles);
    if ((e = allow_lds(fwd_keys_nd<3, 4>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_keys_nd<3, 4>), keys_grid(a), dim3(kBlockNd), lds, s, a);
  }
  return hipGetLastError();
}

// One workgroup per layer of [layer0, layer0 + gridDim.x): a split layer's
// count block is cleared before its histogram parts add into it.
// Clears the count blocks of the split layers: layer layer0 + blockIdx.y,
// kZeroBlocks workgroups per layer, each a strided share of the block.
constexpr int kZeroBlocks = 16;
__global__ __launch_bounds__(256) void zero_split_kernel(FwdArgs a) {
  const LayerDev& L = a.layers[a.layer0 + (int)blockIdx.y];
  if (L.split <= 1) return;
  const int64_t n = (int64_t)L.N * L.N1;
  int32_t* dst = a.counts + L.cnt_off;
  const int64_t stride = (int64_t)kZeroBlocks * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = 0;
}

hipError_t launch_zero_split(const FwdArgs& a, int nl, hipStream_t s) {
  if (nl <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_split_kernel, dim3(kZeroBlocks, (unsigned)nl), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_count_tiles(const FwdArgs& a, hipStream_t s) {
  const size_t lds = sizeof(uint32_t) * (kSuper + 2 * kCountBlock);
  hipError_t e = allow_lds(count_tiles, lds);
  if (e != hipSuccess) return e;
  if (a.total_tiles <= 0) return hipSuccess;
  const unsigned grid =
      a.xcd_map ? 8u * (unsigned)((a.total_tiles + 7) / 8) : (unsigned)a.total_tiles;
  hipLaunchKernelGGL(count_tiles, dim3(grid), dim3(kCountBlock), lds, s, a);
  return hipGetLastError();
}

// The kernel instance of a 1-D search depth (0: each layer's own depth).
#define QTREE_BATCH_1D_SWITCH(LG, CALL) \
  switch (LG) {                         \
    case 1: CALL(1); break;             \
    case 2: CALL(2); break;             \
    case 3: CALL(3); break;             \
    case 4: CALL(4); break;             \
    case 5: CALL(5); break;             \
    case 6: CALL(6); break;             \
    case 7: CALL(7); break;             \
    case 8: CALL(8); break;             \
    case 9: CALL(9); break;             \
    case 10: CALL(10); break;           \
    case 11: CALL(11); break;           \
    case 12: CALL(12); break;           \
    case 13: CALL(13); break;           \
    default: CALL(0);                   \
  }

hipError_t launch_batch_keys(const BatchArgs& a, int dmax, int lg1, int grid, size_t lds,
                             hipStream_t s) {
  hipError_t e = hipSuccess;
  if (a.n_units == 0 || grid <= 0) return hipSuccess;
  if (dmax <= 1 && a.gk >= 0) {
#define QTREE_LAUNCH_1DG(GK, S)                                                             \
  if ((e = allow_lds(batch_keys_1d_guide<GK, S>, lds)) == hipSuccess)                       \
    hipLaunchKernelGGL((batch_keys_1d_guide<GK, S>), dim3((unsigned)grid), dim3(kBlock), lds, \
                       s, a);
#define QTREE_LAUNCH_1DG_S(GK)            \
  if (a.sub == kGuideSub) {               \
    QTREE_LAUNCH_1DG(GK, kGuideSub)       \
  } else {                                \
    QTREE_LAUNCH_1DG(GK, 1)               \
  }
    switch (a.gk) {
      case 0:
      case 1: QTREE_LAUNCH_1DG_S(1) break;
      case 2: QTREE_LAUNCH_1DG_S(2) break;
      case 3: QTREE_LAUNCH_1DG_S(3) break;
      default: QTREE_LAUNCH_1DG_S(4) break;
    }
#undef QTREE_LAUNCH_1DG_S
#undef QTREE_LAUNCH_1DG
    if (e != hipSuccess) return e;
  } else if (dmax <= 1) {
#define QTREE_LAUNCH_1D(LG)                                                                 \
  if ((e = allow_lds(batch_keys_1d<LG>, lds)) == hipSuccess)                                \
    hipLaunchKernelGGL(batch_keys_1d<LG>, dim3((unsigned)grid), dim3(kBlock), lds, s, a);
    QTREE_BATCH_1D_SWITCH(lg1, QTREE_LAUNCH_1D)
#undef QTREE_LAUNCH_1D
    if (e != hipSuccess) return e;
  } else {
#define QTREE_LAUNCH_ND(KER)                                                                 \
  if ((e = allow_lds(KER, lds)) != hipSuccess) return e;                                     \
  hipLaunchKernelGGL((KER), dim3((unsigned)grid), dim3(kBlockNd), lds, s, a);
    if (dmax == 2 && a.bucketed && a.nd_samples == 4) {
      QTREE_LAUNCH_ND(batch_keys_nd_bk1)
    } else if (dmax == 2 && a.bucketed) {
      QTREE_LAUNCH_ND(batch_keys_nd_bk<kBkSamplesHi>)
    } else if (dmax == 2 && a.nd_samples == 4) {
      QTREE_LAUNCH_ND((batch_keys_nd<2, 4>))
    } else if (dmax == 2) {
      QTREE_LAUNCH_ND((batch_keys_nd<2, kSamplesNd2>))
    } else if (a.nd_samples == 4) {
      QTREE_LAUNCH_ND((batch_keys_nd<3, 4>))
    } else {
      QTREE_LAUNCH_ND((batch_keys_nd<3, kSamplesNd2>))
    }
#undef QTREE_LAUNCH_ND
  }
  return hipGetLastError();
}

int batch_keys_occupancy(int dmax, int lg1, int gk, size_t lds, int nd_samples, int bucketed) {
  int blocks = 0;
  hipError_t e = hipSuccess;
  if (dmax <= 1 && gk >= 0) {
    e = allow_lds(batch_keys_1d_guide<2, kGuideSub>, lds);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_keys_1d_guide<2, kGuideSub>,
                                                       kBlock, lds);
  } else if (dmax <= 1) {
#define QTREE_OCC_1D(LG)                                                                   \
  if ((e = allow_lds(batch_keys_1d<LG>, lds)) == hipSuccess)                               \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_keys_1d<LG>, kBlock, lds);
    QTREE_BATCH_1D_SWITCH(lg1, QTREE_OCC_1D)
#undef QTREE_OCC_1D
  } else {
#define QTREE_OCC_ND(KER)                                                                   \
  e = allow_lds(KER, lds);                                                                   \
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, KER, kBlockNd, lds);
    if (dmax == 2 && bucketed && nd_samples == 4) {
      QTREE_OCC_ND(batch_keys_nd_bk1)
    } else if (dmax == 2 && bucketed) {
      QTREE_OCC_ND(batch_keys_nd_bk<kBkSamplesHi>)
    } else if (dmax == 2 && nd_samples == 4) {
      QTREE_OCC_ND((batch_keys_nd<2, 4>))
    } else if (dmax == 2) {
      QTREE_OCC_ND((batch_keys_nd<2, kSamplesNd2>))
    } else if (nd_samples == 4) {
      QTREE_OCC_ND((batch_keys_nd<3, 4>))
    } else {
      QTREE_OCC_ND((batch_keys_nd<3, kSamplesNd2>))
    }
#undef QTREE_OCC_ND
  }
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

hipError_t launch_batch_count(const BatchArgs& a, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  const size_t lds_b = sizeof(uint32_t) * (kSuper + 2 * kCountBlock);
  hipError_t e = allow_lds(batch_count, lds_b);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_count, dim3((unsigned)a.n_tiles), dim3(kCountBlock), lds_b, s, a);
  return hipGetLastError();
}

}  // namespace qtree
