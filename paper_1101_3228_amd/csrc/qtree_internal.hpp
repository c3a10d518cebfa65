// Internal layout shared by the host side of the library and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtree {

constexpr int kMaxDim = 3;

// Two-pass LAYERWISE counting.  Pass A sorts each chunk of kChunk samples of
// a layer by tile (kTile consecutive entries of the layer's count block) and
// stores every key as its 16-bit offset inside its super tile (kSuper
// consecutive entries, kSuper / kTile tiles); pass B gives every (layer,
// super tile) to one workgroup that histograms its keys in LDS and writes the
// super tile with plain stores.
// One tile per super tile: the sort's scan and a chunk's segment table have
// one entry per super tile, all that pass B reads.
constexpr int kTileBits = 14;
constexpr int kTile = 1 << kTileBits;
constexpr int kSuperBits = 14;
constexpr int kSuper = 1 << kSuperBits;
constexpr int kTilesPerSuper = kSuper / kTile;
constexpr int kChunk = 4096;          // samples per pass-A workgroup

// A pointer read from device memory (a batch or job record, a kernel
// argument's struct field) is a generic address to the compiler, which then
// loads through it with flat instructions: a 64-bit address in VGPRs, no
// scalar loads of uniform fields, and waits shared with LDS operations.
// Every table such a field points to is device memory: reading the field as
// a global pointer and converting it gives global and scalar loads.
template <class T>
__device__ __forceinline__ T* as_global(T* const& field) {
  typedef __attribute__((address_space(1))) T* G;
  return (T*)*reinterpret_cast<const G*>(&field);
}
constexpr int kMaxTiles = 4096;       // larger count blocks use direct atomics
constexpr int kDefaultBatch = 1 << 22;  // samples per layer per pass by default
constexpr int kScanTile = 8;            // records per tile of the d >= 2 argmin scan
constexpr int kGuideMax = 8192;         // largest guide table of a 1-D layer (entries)
constexpr int kGuideKMax = 4;           // most midpoints one guide bucket may add

// One record per layer k = 0..n, stored in the plan's device workspace.
// Model coefficients are the FP32 inputs of the AR(1) proposition (Sec. 3);
// A, b, T are unused on the last layer.
struct alignas(16) LayerDev {
  int64_t cnt_off;  // first entry of counts block k (k < n)
  int32_t N;        // N_k
  int32_t N1;       // N_{k+1} (0 on the last layer)
  int32_t pt_off;   // first point of layer k in the point array
  int32_t aux_off;  // 1-D: first padded midpoint of layer k
  int32_t P;        // 1-D: padded midpoint slots, a power of two >= N_k
  int32_t logP;     // log2(P)
  int32_t tiles;    // ceil(N_k N_{k+1} / kTile) (0 on the last layer)
  int32_t tile_off; // super tiles of the layers before k
  // Histogram pass: each super tile of layer k is split into `split` parts
  // over the chunks (layers with few super tiles, such as a one-point first
  // layer, would otherwise give all their keys to a few workgroups); the
  // parts of a split layer add into its count block atomically, zeroed first.
  int32_t split;    // parts per super tile (1: one workgroup stores the tile)
  int32_t unit_off; // histogram-pass units (super tiles x parts) of the layers before k
  int32_t edge_off; // 1-D: first of the N_k + 1 cell-edge probabilities of layer k
  // 1-D guide table of the cell search: bucket b = (int)clamp(fma(x, gt_scale,
  // gt_shift), 0, gt_B - 1); the cell is tab[b] + #{r < K : m[tab[b] + r] < x}
  // for K >= gt_K (the table holds the count of midpoints below the bucket's
  // first float; gt_K bounds the midpoints a bucket can add).
  int32_t gt_off;   // first entry of the layer's table (16-bit entries)
  int32_t gt_B, gt_K;
  float gt_scale, gt_shift;
  float A[9], b[3], T[9], mu[3], L[9];
  float x0[3];      // start point of the pathwise mode (layer 0 record)
  // d = 2 bucketed cell search (bk_B[0] = 0: none): the layer's reachable box
  // from bk_lo in bk_B[0] x bk_B[1] buckets; x is in bucket
  // (floor((x_0 - bk_lo[0]) bk_scale[0]), floor((x_1 - bk_lo[1]) bk_scale[1]))
  // in FP32, and bucket (i, j) owns row bk_off + i bk_B[1] + j of the row
  // array: entry 0 its candidate count c (kBucketFull: more than kBucketCap,
  // the full scan decides), entries 1..c every point that can be the FP32
  // argmin anywhere in it, in increasing index, padded to a whole 8-entry
  // group with N (the search's pad record, whose key is NaN)
  float bk_lo[2], bk_scale[2];
  int32_t bk_B[2];
  int32_t bk_off;
};
constexpr int kBucketRow = 32;            // uint16 entries of a bucket row (64 bytes)
constexpr int kBucketCap = kBucketRow - 1; // candidates a row holds
constexpr uint16_t kBucketFull = 0xFFFF;  // row count: candidates did not fit
// Buckets per side of a d = 2 layer of N points: about 64 buckets per point,
// at most 512 per side, 4 KB of rows per point (the 2-D workload, N = 2000:
// a step of 3.82 ms at 64 per point, 3.89 at 96, 3.97 at 128, 4.15 at 32;
// its first form's sampling pass 5.16 ms at 32, 5.68 at 24, 6.28 at 16,
// 8.42 at 8).  Denser buckets list fewer candidates, so fewer waves walk a
// second group; beyond 64 the rows no longer stay in the caches.
inline int bucket_side(int N) {
  if (N <= 1) return 1;
  int b = 1;
  while ((double)b * b < 64.0 * N) ++b;
  return b < 512 ? b : 512;
}

// Workspace layout (byte offsets from the workspace base).
struct WsLayout {
  size_t layers;   // LayerDev[n+1]
  size_t points;   // d == 1: float[sum N]; d >= 2: float4[sum N] = (g0, g1, g2, h)
  size_t aux;      // d == 1: float[sum P] midpoints padded with +inf
  size_t edges;    // d == 1: double[sum (N_k + 1)] marginal probabilities below the cell edges
  size_t guide;    // d == 1: uint16[(n + 1) kGuideMax] guide tables of the cell search
  size_t band;     // d == 1: int64[R + 1] band offsets, then int32[R] first band columns
                   // of the R = sum_{k<n} N_k count rows (banded stratified counts)
  size_t bk_rows;  // d == 2: uint16[buckets][kBucketRow] bucket rows (count, candidates)
  size_t keys;     // uint16[n][batch chunks][kChunk] pass-A keys
  size_t segs;     // uint32[n][batch chunks][max tiles + 1] segment starts
  size_t total;
};

// Layout for a scratch that holds `batch_chunks` chunks per layer (0: none).
WsLayout ws_layout(int d, int n, const int32_t* N, int64_t batch_chunks);
bool two_pass_fits(int d, int n, const int32_t* N);

struct FwdArgs {
  const LayerDev* layers;
  const float* mids;     // 1-D midpoints (padded per layer)
  const uint16_t* guide; // 1-D guide tables (kGuideMax entries per layer)
  int gt_Kmax;           // 1-D: largest guide K over the layers, -1 without tables
  int gt_Bmax;           // 1-D: largest guide table
  const float4* pts;     // d >= 2 points with half norm
  const float* pts1;     // 1-D points
  int32_t* counts;
  uint64_t m0, M;
  uint32_t key0, key1, contract;
  int32_t n, d;
  // launch decomposition: unit u = (layer, chunk); `chunks` per layer
  int32_t chunks;
  int32_t units;          // n * chunks
  int32_t units_per_xcd;  // ceil(units / 8)
  int32_t xcd_map;        // 1: keep a layer's chunks on one XCD
  uint64_t chunk_len;     // samples per chunk (even)
  int32_t maxP;           // largest padded midpoint count (1-D LDS sizing)
  int32_t maxN;           // largest layer size (d >= 2 LDS sizing)
  int64_t mids_total;     // 1-D: padded midpoints over all layers
  // two-pass counting
  uint16_t* keys;
  uint32_t* segs;
  int32_t seg_stride;     // max tiles + 1
  int32_t max_tiles;
  int32_t total_tiles;    // histogram units of this launch (pass-B grid)
  int32_t first_batch;    // pass B overwrites instead of adding
  int32_t layer0;         // first layer of this launch (units and tiles)
  int32_t nd_samples;     // d >= 2: samples per lane sharing each grid read (8 or 4)
  int32_t tile0;          // first histogram unit of this launch
  // d = 2 bucketed cell search (bucketed = 0: the full scan)
  int32_t bucketed;
  const uint4* bk_rows;
};

// Forward obstacle on the sum of the factors (see qtree_payoff_forward).
struct ForwardArgs {
  const LayerDev* layers;
  const float* pts1;
  const float4* pts;
  double* v;
  int32_t n, d, maxN;
  double S0, K, r, Tm;
  double w[kMaxDim];  // mix' sigma
};

// Swing BDP: P is [Pts][Qmax + 1] (point major, the levels of a point
// contiguous).
constexpr int kSwingMaxQ = 2046;
struct SwingArgs {
  const LayerDev* layers;
  const int32_t* counts;
  const double* v;
  double* P;
  int64_t Pts;
  int32_t n, Qmin, Qmax;
};

hipError_t launch_forward_payoff(const ForwardArgs& a, hipStream_t s);
hipError_t launch_swing(const SwingArgs& a, const int32_t* N_host, hipStream_t s);

hipError_t launch_zero_i32(int32_t* p, int64_t count, hipStream_t s);
hipError_t launch_fwd_layer_1d(const FwdArgs& a, hipStream_t s);
hipError_t launch_fwd_layer_nd(const FwdArgs& a, hipStream_t s);
hipError_t launch_fwd_path(const FwdArgs& a, hipStream_t s);
hipError_t launch_fwd_keys(const FwdArgs& a, hipStream_t s);
hipError_t launch_count_tiles(const FwdArgs& a, hipStream_t s);
// Zero the count blocks of the split layers in [layer0, layer0 + nl).
hipError_t launch_zero_split(const FwdArgs& a, int nl, hipStream_t s);

struct BdpArgs {
  const LayerDev* layers;
  const int32_t* counts;
  const double* phi;
  double* V;
  int64_t P;  // points per payoff vector (sum N_k)
  int32_t n_pay;
  // banded counts (else null): row r = pt_off_k + i holds columns
  // band_lo[r] + w, w < band_off[r + 1] - band_off[r], at counts[band_off[r] + w]
  const int64_t* band_off;
  const int32_t* band_lo;
};
hipError_t launch_bdp_layer(const BdpArgs& a, int k, int N_k, int N_k1, int64_t pt_k,
                            int64_t pt_k1, int64_t cnt_k, hipStream_t s);
hipError_t launch_copy_last_layer(const BdpArgs& a, int64_t pt_n, int N_n, hipStream_t s);

struct Contract {
  double S0, K, r, Tm;
  double sigma[kMaxDim];
  double mix[kMaxDim * kMaxDim];  // Brownian factors y = mix x (row-major d x d)
  int32_t kind;
  int32_t has_mix;                // 0: y = x
};
constexpr int kPayoffGroup = 16;  // contracts per payoff launch (kernel-argument size)

struct PayoffArgs {
  const LayerDev* layers;
  const float* pts1;
  const float4* pts;
  double* phi;      // [count][P]
  int64_t P;
  int32_t n, d, maxN, count;
  Contract c[kPayoffGroup];
};
hipError_t launch_payoff(const PayoffArgs& a, hipStream_t s);

// Transition weights pi^k = c / p (FP64, rows padded to N1p = multiple of 4)
// and the nonzero column range of every row, for the many-contract BDP.
struct PiArgs {
  const LayerDev* layers;
  const int32_t* counts;
  const int64_t* pi_off;  // [n] first weight of layer k (device)
  double* pi;
  int2* band;             // [rows] columns [x, y) hold every nonzero weight of the row
  int64_t rows;           // sum_{k<n} N_k
  int32_t n;
};
hipError_t launch_pi(const PiArgs& a, hipStream_t s);

// Backward recursion of many contracts on one tree (64 per workgroup).
// One tree of a many-tree launch: its tables and weights, and the contracts
// q0 .. q0 + nq - 1 it prices (workgroups blk0 .. blk0 + ceil(nq / 64) - 1).
struct alignas(16) ManyTree {
  const LayerDev* layers;
  const float* pts1;
  const float4* pts;
  const int64_t* pi_off;
  const double* pi;
  const int2* band;
  int64_t q0, nq;
  int32_t blk0, n;
};
struct ManyArgs {
  const LayerDev* layers;
  const float* pts1;
  const float4* pts;
  const int64_t* pi_off;
  const double* pi;
  const int2* band;
  const Contract* specs;  // [nq] (device)
  double* V0;             // [nq] (device)
  int64_t nq;
  int32_t n, d, max_n, np_max;  // np_max: largest N_k rounded up to a multiple of 4
  // many trees (else null): the table of n_trees trees, ordered by blk0;
  // the fields above then come from the workgroup's tree (max_n, np_max: the
  // largest over the trees)
  const ManyTree* trees;
  int32_t n_trees, blocks;
};
int bdp_many_maxr(int max_n);  // -1: beyond the supported 256 points per layer
size_t bdp_many_lds(int max_np);
hipError_t launch_bdp_many(const ManyArgs& a, hipStream_t s);

// Stratified time-layer counts (d = 1): Ms samples per cell of layer k.
struct StratArgs {
  const LayerDev* layers;
  const float* mids;      // sorted midpoints, padded per layer
  const uint16_t* guide;  // guide tables of the cell search (kGuideMax entries per layer)
  int gt_Kmax, gt_Bmax;   // largest guide K (-1: no tables) and table over the layers
  const double* edges;    // cell-edge probabilities per layer
  uint32_t key0, key1, contract;
  uint64_t M;             // samples per row (alloc 0) or per layer (alloc 1)
  int alloc;              // 0 equal, 1 proportional allocation
  int32_t* counts;        // the plan's count blocks, or the band values
  int n, maxP, maxN;      // layers; largest padded midpoint count; largest N_k
  // banded output (else null): row r = pt_off_k + i keeps columns
  // band_lo[r] .. band_lo[r] + W_r - 1 at counts[band_off[r] ..], W_r =
  // band_off[r + 1] - band_off[r]; counts outside the band go to *overflow
  const int64_t* band_off;
  const int32_t* band_lo;
  uint32_t* overflow;
};
constexpr int kStratRows = 4;            // rows (strata) per tile
constexpr uint64_t kStratSegment = 65536;  // samples per workgroup at most
// A workgroup's share: samples [s0, s1) of the tile of rows [i0, i0 + 4) of
// layer k (in the tile's own order: row by row); split: the tile is shared
// by several workgroups (its counts are added with atomics onto zeros).
struct alignas(16) StratUnit {
  int32_t k, i0, split, pad;
  uint64_t s0, s1;
};
size_t strat_lds_bytes(int maxP, int maxN);
hipError_t launch_strat(const StratArgs& a, const StratUnit* units, int n_units, hipStream_t s);
hipError_t launch_strat_samples(const StratArgs& a, int k, int i, uint64_t t0, int64_t count,
                                float* x, float* y, hipStream_t s);

// Randomized Lloyd iteration (Sec. 2, eq. Qerr) on a device grid.
struct LloydArgs {
  int d, N;
  int Npad;                  // d >= 2: records padded to whole scan tiles
  int P, logP;               // d = 1: midpoint slots (power of two >= N)
  float L[9];                // X = L z, row-major [d][d]
  uint32_t key0, key1;       // Philox key (seed)
  uint32_t it_ctr;           // counter word 1 of the step (the step, or 0)
  int it;                    // step index (distortion slot)
  uint64_t M;                // samples per step
  float* grid;               // [N][d], updated in place
  float4* recs;              // d >= 2: [Npad] (g, |g|^2 / 2)
  float* mids;               // d = 1: [P] midpoints padded with +inf
  unsigned int* cnt;         // [N]
  unsigned long long* sum;   // [N][d] two's complement sums of rint(x 2^24)
  unsigned long long* dist;  // sum of rint(|x - g|^2 2^16)
  double* distortion;        // [steps] or null
  // per-workgroup partials of the accumulation: row b holds workgroup b's
  // sums [N d], counts [N], distortion, admissible and inadmissible samples
  // (E = N d + N + 3 words)
  unsigned long long* part;
  int E;
  // samples of a caller's set instead of Philox draws: step window
  // (start + m) mod Ms, m < M; samples with a coordinate outside [-64, 64]
  // (or NaN) are skipped and counted
  const float* xs;           // [Ms][d] device, or null (Philox samples)
  uint64_t Ms;
  uint64_t start;
  double gamma;              // new point g + gamma (mean - g); 1: the mean
  unsigned long long* used;  // admissible samples of the step
  unsigned long long* rej;   // inadmissible samples of the step
  unsigned long long* rej_total;  // running total over the steps
  long long* rejected;       // caller's copy of the total, or null
};
constexpr int kLloydMaxBlocks = 512;  // accumulation workgroups per step at most
size_t lloyd_lds_bytes(int d, int N, int Npad, int P);
// Bucket rows of the d = 2 bucketed cell search of every layer (records
// and LayerDev already in the workspace).
hipError_t launch_bucket_build(const LayerDev* layers, int n_layers_total, int total_buckets,
                               const float4* pts, uint16_t* rows, hipStream_t s);
hipError_t launch_lloyd_prepare(const LloydArgs& a, hipStream_t s);
hipError_t launch_lloyd_step(const LloydArgs& a, int blocks, hipStream_t s);
// Moment-matching grids: exact integer moment sums of a device sample set,
// sums = [count, s1 (d), s2 (d d)], and the grid mean + chol(cov) base.
hipError_t launch_sample_moments(int d, const float* x, uint64_t M, long long* sums,
                                 hipStream_t s);
hipError_t launch_moment_grid(int d, const long long* sums, const float* base, int N,
                              float* grid, double* moments, hipStream_t s);

hipError_t launch_pi_quarter_disc(uint32_t key0, uint32_t key1, uint32_t rep0, int reps,
                                  uint64_t blocks, unsigned long long* inside, hipStream_t s);
hipError_t launch_box_muller(const uint32_t* ra, const uint32_t* rb, int64_t count, float* z0,
                             float* z1, hipStream_t s);
hipError_t launch_layer_samples(const FwdArgs& a, int k, int64_t count, float* x, float* y,
                                hipStream_t s);
hipError_t launch_cells(const FwdArgs& a, int k, const float* x, int64_t count, int32_t* cell,
                        hipStream_t s);

}  // namespace qtree
