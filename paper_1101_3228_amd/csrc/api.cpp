// C-ABI of the qtree library: argument checks, plan/workspace layout and
// kernel dispatch.  Declarations and contracts are in include/qtree.h.
#include "qtree.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qtree_batch.hpp"
#include "qtree_internal.hpp"
#include "qtree_plan.hpp"

namespace {

thread_local std::string g_last_error;

qtree_status fail(qtree_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

}  // namespace

namespace qtree {
qtree_status set_error(qtree_status s, const std::string& msg) { return fail(s, msg); }
}  // namespace qtree

namespace {

qtree_status hip_fail(hipError_t e, const char* what) {
  return fail(QTREE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

int log2i(int p) {
  int l = 0;
  while ((1 << l) < p) ++l;
  return l;
}

// LDS limits of the kernels (160 KiB per CU; the 1-D layerwise kernel stages
// two padded midpoint arrays, the d >= 2 kernel two point arrays of 16 B).
constexpr int kMaxN1d = 16384;
constexpr int64_t kManySuperTiles = 2048;  // histogram units that fill the chip unsplit
constexpr int kMaxNnd = 4096;

}  // namespace


namespace qtree {

int max_tiles_of(int n, const int32_t* N) {
  int64_t mt = 0;
  for (int k = 0; k < n; ++k) {
    const int64_t t = ((int64_t)N[k] * N[k + 1] + kTile - 1) / kTile;
    if (t > mt) mt = t;
  }
  return (int)(mt > (1 << 30) ? (1 << 30) : mt);
}

// LDS bytes of the pass-A kernel (grids or midpoints, staged keys, tile
// counters, cursors and scan partials); two-pass counting needs it to fit.
size_t keys_lds_bytes(int d, int n, const int32_t* N) {
  int maxN = 0, maxP = 0;
  for (int k = 0; k <= n; ++k) {
    maxN = N[k] > maxN ? N[k] : maxN;
    maxP = next_pow2(N[k]) > maxP ? next_pow2(N[k]) : maxP;
  }
  const size_t grids =
      d == 1 ? sizeof(float) * (2 * (size_t)maxP + 4) : 16 * 2 * (size_t)(maxN + kScanTile);
  const int mt = max_tiles_of(n, N);
  const size_t sub = d == 1 ? 1 : (size_t)nd_sub_counters(mt);  // the d >= 2 sort's sub-counters
  return grids + sizeof(uint16_t) * kChunk + sizeof(uint32_t) * (2 * (size_t)mt * sub + 1 + 256);
}

bool two_pass_fits(int d, int n, const int32_t* N) {
  return max_tiles_of(n, N) <= kMaxTiles && keys_lds_bytes(d, n, N) <= 160 * 1024;
}

// Buckets of the d = 2 cell search over all layers (layers of one point
// have none).
// Layers take bucket tables in order while the rows so far stay within
// int32 indices; later layers (beyond about 8000 layers of 4096 points)
// keep the full scan.  bucket_boxes follows the same rule.
constexpr int64_t kMaxBuckets = 0x7FFFFFFF;
int64_t total_buckets(int n, const int32_t* N) {
  int64_t b = 0;
  for (int k = 0; k <= n; ++k) {
    if (N[k] <= 1) continue;
    const int64_t b2 = (int64_t)bucket_side(N[k]) * bucket_side(N[k]);
    if (b + b2 <= kMaxBuckets) b += b2;
  }
  return b;
}

WsLayout ws_layout(int d, int n, const int32_t* N, int64_t batch_chunks) {
  WsLayout l{};
  size_t off = 0;
  l.layers = off;
  off = align_up(off + sizeof(LayerDev) * (size_t)(n + 1), 256);
  int64_t pts = 0, mids = 0;
  for (int k = 0; k <= n; ++k) {
    pts += N[k];
    mids += next_pow2(N[k]);
  }
  l.points = off;
  off = align_up(off + (size_t)pts * (d == 1 ? sizeof(float) : sizeof(float4)), 256);
  l.aux = off;
  if (d == 1) off = align_up(off + (size_t)mids * sizeof(float), 256);
  l.edges = off;
  if (d == 1) off = align_up(off + (size_t)(pts + n + 1) * sizeof(double), 256);
  l.guide = off;
  if (d == 1) off = align_up(off + (size_t)(n + 1) * kGuideMax * sizeof(uint16_t), 256);
  l.band = off;
  if (d == 1) {
    const int64_t rows = pts - N[n];
    off = align_up(off + sizeof(int64_t) * (size_t)(rows + 1) + sizeof(int32_t) * (size_t)rows,
                   256);
  }
  const int64_t buckets = d == 2 ? total_buckets(n, N) : 0;
  l.bk_rows = off;
  off = align_up(off + sizeof(uint16_t) * kBucketRow * (size_t)buckets, 256);
  // scratch of the two-pass counting (only when every count block has at
  // most kMaxTiles tiles)
  const int mt = max_tiles_of(n, N);
  l.keys = off;
  if (batch_chunks > 0 && two_pass_fits(d, n, N)) {
    off = align_up(off + sizeof(uint16_t) * (size_t)n * (size_t)batch_chunks * kChunk, 256);
    l.segs = off;
    off = align_up(off + sizeof(uint32_t) * (size_t)n * (size_t)batch_chunks * (size_t)(mt + 1),
                   256);
  } else {
    l.segs = off;
  }
  l.total = off;
  return l;
}

// Chunks per layer a scratch for `samples` samples per layer needs (a d = 1
// batch may start on an odd sample, so it spans one more Philox block).
int64_t chunks_for(int d, uint64_t samples) {
  if (samples == 0) return 0;
  if (d == 1) return (int64_t)((samples / 2 + 1 + kChunk / 2 - 1) / (kChunk / 2));
  return (int64_t)((samples + kChunk - 1) / kChunk);
}

}  // namespace qtree

// Guide table of a sorted 1-D midpoint array m[0 .. nm) (the cell search of
// the forward kernels).  The device maps x to bucket
//   b = (int)fminf(fmaxf(fmaf(x, scale, shift), 0), B - 1),
// a non-decreasing function of x, so every bucket is an interval of floats;
// the table stores c(first float of the bucket), c(x) = #{r : m_r < x}, and
// K bounds c(last float) - c(first float) over the buckets.  The table size is
// the smallest power of two in 256 .. kGuideMax with K <= 2, else with
// K <= kGuideKMax; K = -1 when none qualifies (the kernels then use the
// breadth-first binary search).
namespace {
int64_t float_order(float x) {
  uint32_t u;
  std::memcpy(&u, &x, sizeof u);
  return (u & 0x80000000u) ? -(int64_t)(u & 0x7FFFFFFFu) : (int64_t)u;
}
float order_float(int64_t v) {
  const uint32_t u = v >= 0 ? (uint32_t)v : (0x80000000u | (uint32_t)(-v));
  float x;
  std::memcpy(&x, &u, sizeof x);
  return x;
}
int guide_bucket(float x, float scale, float shift, int B) {
  float t = std::fmaf(x, scale, shift);
  t = std::fmax(t, 0.0f);
  t = std::fmin(t, (float)(B - 1));
  return (int)t;
}
struct Guide {
  int B = 1, K = 0;
  float scale = 0.f, shift = 0.f;
  std::vector<uint16_t> tab;
};
Guide build_guide(const float* m, int nm) {
  Guide best;
  best.tab.assign(1, 0);
  if (nm <= 0) return best;  // one cell: bucket 0, nothing to add
  auto count_below = [&](float x) {
    return (int)(std::lower_bound(m, m + nm, x) - m);  // #{m_r < x}
  };
  const int64_t lo_o = float_order(-FLT_MAX), hi_o = float_order(FLT_MAX);
  for (int cap : {2, qtree::kGuideKMax}) {
    for (int B = 256; B <= qtree::kGuideMax; B *= 2) {
      Guide g;
      g.B = B;
      const float span = m[nm - 1] - m[0];
      g.scale = span > 0.0f ? (float)B / span : 0.0f;
      g.shift = -m[0] * g.scale;
      if (!std::isfinite(g.scale) || !std::isfinite(g.shift)) continue;
      // first float of every bucket (or past the end when a bucket is empty)
      std::vector<int64_t> first(B + 1, hi_o + 1);
      first[0] = lo_o;
      for (int b = 1; b < B; ++b) {
        int64_t lo = first[b - 1], hi = hi_o + 1;  // smallest v with bucket >= b
        while (lo < hi) {
          const int64_t mid = lo + (hi - lo) / 2;
          if (guide_bucket(order_float(mid), g.scale, g.shift, B) >= b) hi = mid;
          else lo = mid + 1;
        }
        first[b] = lo;
      }
      g.tab.assign(B, 0);
      g.K = 0;
      for (int b = 0; b < B; ++b) {
        const int64_t f = first[b], l = first[b + 1] - 1;  // floats of bucket b
        if (f > hi_o) {  // empty bucket: no float maps here
          g.tab[b] = (uint16_t)nm;
          continue;
        }
        const int c0 = count_below(order_float(f));
        const int c1 = count_below(order_float(std::min(l, hi_o)));
        g.tab[b] = (uint16_t)c0;
        g.K = std::max(g.K, c1 - c0);
      }
      if (g.K <= cap) return g;
    }
  }
  best.K = -1;  // no table: binary search
  return best;
}
}  // namespace

extern "C" {

const char* qtree_status_string(qtree_status s) {
  switch (s) {
    case QTREE_OK: return "ok";
    case QTREE_EINVAL: return "invalid argument";
    case QTREE_ENOMEM: return "workspace too small";
    case QTREE_EOVERFLOW: return "count overflow (M >= 2^31 or m0 + M > 2^32)";
    case QTREE_EDEVICE: return "HIP runtime error";
    case QTREE_EUNSUPPORTED: return "unsupported by the library";
  }
  return "unknown status";
}

const char* qtree_last_error(void) { return g_last_error.c_str(); }

const char* qtree_version(void) { return "qtree 0.1 gfx950"; }


static qtree_status check_shape(int32_t d, int32_t n, const int32_t* N) {
  if (d < 1 || d > 3) return fail(QTREE_EINVAL, "d must be 1, 2 or 3");
  if (n < 1) return fail(QTREE_EINVAL, "n must be >= 1");
  if (!N) return fail(QTREE_EINVAL, "N is NULL");
  if (N[0] != 1) return fail(QTREE_EINVAL, "N[0] must be 1 (layer 0 is the start point)");
  for (int k = 0; k <= n; ++k) {
    if (N[k] < 1) return fail(QTREE_EINVAL, "N[k] must be >= 1 (layer " + std::to_string(k) + ")");
    if (d == 1 && N[k] > kMaxN1d)
      return fail(QTREE_EUNSUPPORTED, "1-D layers are limited to 16384 points");
    if (d > 1 && N[k] > kMaxNnd)
      return fail(QTREE_EUNSUPPORTED, "2-D/3-D layers are limited to 4096 points");
  }
  return QTREE_OK;
}

qtree_status qtree_workspace_size(int32_t d, int32_t n, const int32_t* N, uint64_t batch_samples,
                                  size_t* bytes) {
  if (!bytes) return fail(QTREE_EINVAL, "bytes is NULL");
  qtree_status s = check_shape(d, n, N);
  if (s != QTREE_OK) return s;
  if (batch_samples == 0) batch_samples = qtree::kDefaultBatch;
  if (batch_samples > (1ull << 31)) return fail(QTREE_EINVAL, "batch_samples must be <= 2^31");
  *bytes = qtree::ws_layout(d, n, N, qtree::chunks_for(d, batch_samples)).total;
  return QTREE_OK;
}

static bool all_finite(const float* p, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Banded layout of the stratified counts (d = 1): the columns of layer k+1
// that the samples of row i of layer k can reach.  X_k lies in cell i
// (between the FP32 midpoints m_{i-1} and m_i; the end cells reach
// mu_k - 38.5 L_k and mu_k + 8.3 L_k, the normal quantiles of the clamped
// probabilities 2^-1074 and 1 - 2^-53), and eps within +-5.769 (the largest
// Box-Muller radius), so X_{k+1} = A_k X_k + b_k + T_k eps lies in an
// interval, widened by a margin for the FP32 rounding of the samples, whose
// cells (layer k+1's midpoints strictly below its ends) form the band.
// Writes int64 offsets [R + 1] then int32 first columns [R] at `dst` and
// keeps host copies in the plan.
static void band_table(qtree_plan& p, const qtree_model* model, const float* mids, char* dst) {
  const int n = p.n;
  const int64_t R = p.pt_off[n];
  p.band_off.assign((size_t)R + 1, 0);
  p.band_lo.assign((size_t)R, 0);
  int64_t o = 0;
  for (int k = 0; k < n; ++k) {
    const float* m0 = mids + p.aux_off[k];
    const float* m1 = mids + p.aux_off[k + 1];
    const int n1 = p.N[k + 1] - 1;  // midpoints of layer k+1
    const double mu = model->mu[k], L = std::fabs((double)model->L[k]);
    const double A = model->A[k], b = model->b[k], T = std::fabs((double)model->T[k]);
    for (int i = 0; i < p.N[k]; ++i) {
      double xl = i == 0 ? mu - 38.5 * L : (double)m0[i - 1];
      double xh = i == p.N[k] - 1 ? mu + 8.3 * L : (double)m0[i];
      const double mx = 1e-6 * (1.0 + std::fabs(mu) + 40.0 * L + std::fabs(xl) + std::fabs(xh));
      xl -= mx;
      xh += mx;
      double yl = (A >= 0.0 ? A * xl : A * xh) + b - 5.769 * T;
      double yh = (A >= 0.0 ? A * xh : A * xl) + b + 5.769 * T;
      const double my = 1e-6 * (1.0 + std::fabs(yl) + std::fabs(yh));
      yl -= my;
      yh += my;
      const int lo = (int)(std::lower_bound(m1, m1 + n1, yl,
                                            [](float m, double y) { return (double)m < y; }) -
                           m1);
      const int hi = (int)(std::lower_bound(m1, m1 + n1, yh,
                                            [](float m, double y) { return (double)m < y; }) -
                           m1) + 1;
      const int64_t r = p.pt_off[k] + i;
      p.band_lo[(size_t)r] = lo;
      p.band_off[(size_t)r] = o;
      o += hi - lo;
    }
  }
  p.band_off[(size_t)R] = o;
  std::memcpy(dst, p.band_off.data(), sizeof(int64_t) * (size_t)(R + 1));
  std::memcpy(dst + sizeof(int64_t) * (size_t)(R + 1), p.band_lo.data(),
              sizeof(int32_t) * (size_t)R);
}

// Boxes of the d = 2 bucketed cell search.  Layer k's time-layer samples
// are X_k = mu_k + L_k z (as the first point of a pair) and
// A_{k-1} X_{k-1} + b_{k-1} + T_{k-1} eps (as the second), every normal
// within +-5.7684 (the largest Box-Muller radius), so X_k lies in the union
// of two boxes (interval arithmetic, FP64); with the layer's own points and
// a margin for FP32 rounding, that union is cut into bucket_side(N_k)^2
// buckets.  A point outside the box (a pathwise state, a diagnostic query)
// is found by the full scan.
static void bucket_boxes(qtree_plan& p, const qtree_model* model, const float* grid,
                         qtree::LayerDev* layers) {
  constexpr double kZ = 5.7684;
  const int n = p.n;
  std::vector<double> slo((size_t)(n + 1) * 2), shi((size_t)(n + 1) * 2);
  for (int k = 0; k <= n; ++k)
    for (int r = 0; r < 2; ++r) {
      double w = 0.0;
      for (int c = 0; c < 2; ++c) w += std::fabs((double)model->L[(size_t)k * 4 + r * 2 + c]);
      slo[(size_t)k * 2 + r] = (double)model->mu[(size_t)k * 2 + r] - kZ * w;
      shi[(size_t)k * 2 + r] = (double)model->mu[(size_t)k * 2 + r] + kZ * w;
    }
  int64_t off = 0;
  for (int k = 0; k <= n; ++k) {
    qtree::LayerDev& L = layers[k];
    L.bk_B[0] = L.bk_B[1] = 0;
    L.bk_off = (int32_t)off;
    if (p.N[k] <= 1) continue;
    const int B = qtree::bucket_side(p.N[k]);
    if (off + (int64_t)B * B > qtree::kMaxBuckets) continue;
    double lo[2], hi[2];
    for (int r = 0; r < 2; ++r) {
      lo[r] = slo[(size_t)k * 2 + r];
      hi[r] = shi[(size_t)k * 2 + r];
    }
    if (k > 0) {
      const float* A = model->A + (size_t)(k - 1) * 4;
      const float* T = model->T + (size_t)(k - 1) * 4;
      for (int r = 0; r < 2; ++r) {
        double c = (double)model->b[(size_t)(k - 1) * 2 + r], w = 0.0;
        for (int q = 0; q < 2; ++q) {
          const double m = 0.5 * (slo[(size_t)(k - 1) * 2 + q] + shi[(size_t)(k - 1) * 2 + q]);
          const double h = 0.5 * (shi[(size_t)(k - 1) * 2 + q] - slo[(size_t)(k - 1) * 2 + q]);
          c += (double)A[r * 2 + q] * m;
          w += std::fabs((double)A[r * 2 + q]) * h + kZ * std::fabs((double)T[r * 2 + q]);
        }
        lo[r] = std::min(lo[r], c - w);
        hi[r] = std::max(hi[r], c + w);
      }
    }
    const float* g = grid + (size_t)p.pt_off[k] * 2;
    for (int i = 0; i < p.N[k]; ++i)
      for (int r = 0; r < 2; ++r) {
        lo[r] = std::min(lo[r], (double)g[(size_t)i * 2 + r]);
        hi[r] = std::max(hi[r], (double)g[(size_t)i * 2 + r]);
      }
    for (int r = 0; r < 2; ++r) {
      const double m = 1e-3 * (hi[r] - lo[r]) + 1e-6 * (1.0 + std::fabs(lo[r]) + std::fabs(hi[r]));
      lo[r] -= m;
      hi[r] += m;
      L.bk_lo[r] = (float)lo[r];
      L.bk_scale[r] = (float)((double)B / (hi[r] - (double)L.bk_lo[r]));
      L.bk_B[r] = B;
    }
    off += (int64_t)B * B;
  }
  p.buckets = off;
  // with the bucket tables, one sample per lane and round runs at six waves
  // per SIMD and beats two per round's shared grid reads
  if (off > 0) p.tune_nd_samples = 4;
}

qtree_status qtree_plan_create(const qtree_model* model, const float* grid, const int32_t* N,
                               void* workspace, size_t workspace_bytes, qtree_plan** out) {
  if (!out) return fail(QTREE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!model) return fail(QTREE_EINVAL, "model is NULL");
  const int d = model->d, n = model->n;
  qtree_status s = check_shape(d, n, N);
  if (s != QTREE_OK) return s;
  if (!model->A || !model->b || !model->T || !model->mu || !model->L || !model->x0)
    return fail(QTREE_EINVAL, "model array is NULL");
  if (!grid) return fail(QTREE_EINVAL, "grid is NULL");
  if (!workspace) return fail(QTREE_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 16)
    return fail(QTREE_EINVAL, "workspace must be 16-byte aligned");
  const size_t dd = (size_t)d * d;
  if (!all_finite(model->A, dd * n) || !all_finite(model->b, (size_t)d * n) ||
      !all_finite(model->T, dd * n) || !all_finite(model->mu, (size_t)d * (n + 1)) ||
      !all_finite(model->L, dd * (n + 1)) || !all_finite(model->x0, d))
    return fail(QTREE_EINVAL, "model coefficients must be finite");

  qtree_plan p;
  p.d = d;
  p.n = n;
  p.N.assign(N, N + n + 1);
  p.pt_off.resize(n + 2);
  p.cnt_off.resize(n + 1);
  p.aux_off.resize(n + 2);
  p.P.resize(n + 1);
  p.pt_off[0] = 0;
  p.cnt_off[0] = 0;
  p.aux_off[0] = 0;
  for (int k = 0; k <= n; ++k) {
    p.pt_off[k + 1] = p.pt_off[k] + N[k];
    p.P[k] = next_pow2(N[k]);
    p.aux_off[k + 1] = p.aux_off[k] + p.P[k];
    if (k < n) p.cnt_off[k + 1] = p.cnt_off[k] + (int64_t)N[k] * N[k + 1];
    if (N[k] > p.maxN) p.maxN = N[k];
    if (p.P[k] > p.maxP) p.maxP = p.P[k];
  }
  p.points = p.pt_off[n + 1];
  p.entries = p.cnt_off[n];
  p.mids_total = p.aux_off[n + 1];
  if (!all_finite(grid, (size_t)p.points * d)) return fail(QTREE_EINVAL, "grid must be finite");
  if (d == 1) {
    for (int k = 0; k <= n; ++k) {
      const float* g = grid + p.pt_off[k];
      for (int r = 0; r + 1 < N[k]; ++r)
        if (!(g[r] < g[r + 1]))
          return fail(QTREE_EINVAL, "1-D grid of layer " + std::to_string(k) +
                                        " must be strictly increasing");
    }
  }
  // the scratch takes whatever the workspace holds beyond the layer tables
  p.max_tiles = qtree::max_tiles_of(n, N);
  const qtree::WsLayout base = qtree::ws_layout(d, n, N, 0);
  if (workspace_bytes < base.total)
    return fail(QTREE_ENOMEM, "workspace needs at least " + std::to_string(base.total) + " bytes");
  p.batch_chunks = 0;
  if (qtree::two_pass_fits(d, n, N)) {
    const size_t per = (size_t)n * (sizeof(uint16_t) * qtree::kChunk +
                                    sizeof(uint32_t) * (size_t)(p.max_tiles + 1));
    int64_t c = (int64_t)((workspace_bytes - base.total) / per);
    while (c > 0 && qtree::ws_layout(d, n, N, c).total > workspace_bytes) --c;
    p.batch_chunks = c;
  }
  p.two_pass_ok = p.batch_chunks > 0;
  p.two_pass_shape = qtree::two_pass_fits(d, n, N);
  p.lay = qtree::ws_layout(d, n, N, p.batch_chunks);

  // host image of the workspace
  std::vector<char> img(p.lay.total, 0);
  auto* layers = reinterpret_cast<qtree::LayerDev*>(img.data() + p.lay.layers);
  // histogram parts: a layer with fewer super tiles than the largest layer
  // is split over the chunks into up to that ratio (at most 16), so that no
  // workgroup of the histogram pass takes many times the keys of another (a
  // one-point first layer has a single super tile).  With few super tiles
  // in all, every super tile is split in two besides, so that the last
  // layer group's histogram, which no sampling pass hides, has twice the
  // workgroups (1-D workload, n = 50, N = 500, M = 1e7: 1.835 ms per step
  // against 1.899 unsplit and 1.838 with four parts); with many, splitting
  // only costs the clearing of the split blocks (the parts add into them).
  int64_t st_max = 1, st_all = 0;
  for (int k = 0; k < n; ++k) {
    const int64_t st = ((int64_t)N[k] * N[k + 1] + qtree::kSuper - 1) / qtree::kSuper;
    st_max = std::max<int64_t>(st_max, st);
    st_all += st;
  }
  const int64_t split_base = st_all >= kManySuperTiles ? 1 : 2;
  int32_t total_units = 0;
  for (int k = 0; k <= n; ++k) {
    qtree::LayerDev L{};
    L.cnt_off = k < n ? p.cnt_off[k] : 0;
    L.N = N[k];
    L.N1 = k < n ? N[k + 1] : 0;
    L.pt_off = (int32_t)p.pt_off[k];
    L.aux_off = (int32_t)p.aux_off[k];
    L.P = p.P[k];
    L.logP = log2i(p.P[k]);
    const int64_t entries_k = k < n ? (int64_t)N[k] * N[k + 1] : 0;
    L.tiles = (int32_t)((entries_k + qtree::kTile - 1) / qtree::kTile);
    L.tile_off = p.total_tiles;
    L.edge_off = (int32_t)(p.pt_off[k] + k);
    p.tile_off.push_back(p.total_tiles);
    const int64_t st_k = (entries_k + qtree::kSuper - 1) / qtree::kSuper;
    p.total_tiles += (int32_t)st_k;
    L.split = st_k > 0
                  ? (int32_t)std::min<int64_t>(16, split_base * std::max<int64_t>(1, st_max / st_k))
                  : 1;
    L.unit_off = total_units;
    p.split.push_back(L.split);
    p.unit_off.push_back(total_units);
    total_units += (int32_t)(st_k * L.split);
    if (k < n) {
      std::memcpy(L.A, model->A + dd * k, sizeof(float) * dd);
      std::memcpy(L.b, model->b + (size_t)d * k, sizeof(float) * d);
      std::memcpy(L.T, model->T + dd * k, sizeof(float) * dd);
    }
    std::memcpy(L.mu, model->mu + (size_t)d * k, sizeof(float) * d);
    std::memcpy(L.L, model->L + dd * k, sizeof(float) * dd);
    std::memcpy(L.x0, model->x0, sizeof(float) * d);
    layers[k] = L;
  }
  if (d == 1) {
    std::memcpy(img.data() + p.lay.points, grid, sizeof(float) * (size_t)p.points);
    float* mids = reinterpret_cast<float*>(img.data() + p.lay.aux);
    for (int k = 0; k <= n; ++k) {
      const float* g = grid + p.pt_off[k];
      float* m = mids + p.aux_off[k];
      // cell edges of Gamma_k: FP32 midpoints (x_r + x_{r+1}) / 2, padded with
      // +inf; a zero midpoint is stored as +0 (the device search reads the
      // sign bit of m - x, and -0 < x is the same comparison as +0 < x)
      for (int r = 0; r < p.P[k]; ++r) {
        float v = (r + 1 < N[k]) ? 0.5f * (g[r] + g[r + 1]) : INFINITY;
        if (v == 0.0f) v = 0.0f;
        m[r] = v;
      }
    }
    p.marg_L.assign(model->L, model->L + n + 1);
    // guide tables of the cell search, from the stored midpoints
    uint16_t* guide = reinterpret_cast<uint16_t*>(img.data() + p.lay.guide);
    p.gt_Kmax = 0;
    p.gt_Bmax = 1;
    for (int k = 0; k <= n; ++k) {
      const Guide g = build_guide(mids + p.aux_off[k], N[k] - 1);
      qtree::LayerDev& L = layers[k];
      L.gt_off = k * qtree::kGuideMax;
      L.gt_B = g.B;
      L.gt_K = g.K;
      L.gt_scale = g.scale;
      L.gt_shift = g.shift;
      std::memcpy(guide + (size_t)k * qtree::kGuideMax, g.tab.data(),
                  sizeof(uint16_t) * g.tab.size());
      if (g.K < 0) p.gt_Kmax = -1;
      if (p.gt_Kmax >= 0) p.gt_Kmax = std::max(p.gt_Kmax, g.K);
      p.gt_Bmax = std::max(p.gt_Bmax, g.B);
    }
    // stratified sampling: probabilities of the marginal N(mu_k, L_k^2) below
    // the cell edges, e_0 = 0, e_{r+1} = Phi(((double)m_r - mu_k) / L_k),
    // e_N = 1, with Phi(a) = erfc(-a / sqrt 2) / 2
    double* edges = reinterpret_cast<double*>(img.data() + p.lay.edges);
    for (int k = 0; k <= n; ++k) {
      const float* g = grid + p.pt_off[k];
      double* e = edges + p.pt_off[k] + k;
      e[0] = 0.0;
      e[N[k]] = 1.0;
      for (int r = 0; r + 1 < N[k]; ++r) {
        const float m = 0.5f * (g[r] + g[r + 1]);
        const double a = ((double)m - (double)model->mu[k]) / (double)model->L[k];
        e[r + 1] = 0.5 * std::erfc(-a * 0.70710678118654752440);
      }
    }
    p.edges.assign(edges, edges + p.points + n + 1);
    band_table(p, model, mids, img.data() + p.lay.band);
  } else {
    float4* pts = reinterpret_cast<float4*>(img.data() + p.lay.points);
    for (int64_t t = 0; t < p.points; ++t) {
      const float* g = grid + t * d;
      // half norm |g|^2 / 2: g0*g0, then fused g_c*g_c + t, then the exact halving
      float h = g[0] * g[0];
      for (int c = 1; c < d; ++c) h = std::fmaf(g[c], g[c], h);
      h = 0.5f * h;
      pts[t] = make_float4(g[0], d > 1 ? g[1] : 0.f, d > 2 ? g[2] : 0.f, h);
    }
    if (d == 2) bucket_boxes(p, model, grid, layers);
  }
  hipError_t e = hipMemcpy(workspace, img.data(), p.lay.total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(workspace)");
  p.ws = static_cast<char*>(workspace);
  if (p.buckets > 0) {
    // the bucket rows, from the records just uploaded
    e = qtree::launch_bucket_build(
        reinterpret_cast<const qtree::LayerDev*>(p.ws + p.lay.layers), n + 1, (int)p.buckets,
        reinterpret_cast<const float4*>(p.ws + p.lay.points),
        reinterpret_cast<uint16_t*>(p.ws + p.lay.bk_rows), nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(e, "bucket tables");
  }
  *out = new qtree_plan(std::move(p));
  return QTREE_OK;
}

void qtree_plan_destroy(qtree_plan* plan) { delete plan; }

int32_t qtree_plan_dim(const qtree_plan* p) { return p ? p->d : 0; }
int32_t qtree_plan_layers(const qtree_plan* p) { return p ? p->n : 0; }
int64_t qtree_plan_count_entries(const qtree_plan* p) { return p ? p->entries : 0; }
int64_t qtree_plan_points(const qtree_plan* p) { return p ? p->points : 0; }

static qtree::FwdArgs fwd_args(const qtree_plan* p, uint64_t m0, uint64_t M, uint64_t seed,
                               uint32_t contract, int32_t* counts) {
  qtree::FwdArgs a{};
  a.layers = reinterpret_cast<const qtree::LayerDev*>(p->ws + p->lay.layers);
  a.mids = reinterpret_cast<const float*>(p->ws + p->lay.aux);
  a.guide = reinterpret_cast<const uint16_t*>(p->ws + p->lay.guide);
  a.gt_Kmax = p->d == 1 ? p->gt_Kmax : -1;
  a.gt_Bmax = p->gt_Bmax;
  if (a.gt_Kmax >= 0 && qtree::keys_lds_1d_guide(p->maxP, p->gt_Bmax, p->max_tiles) > 160 * 1024)
    a.gt_Kmax = -1;  // the tables do not fit beside the midpoints: binary search
  a.pts = reinterpret_cast<const float4*>(p->ws + p->lay.points);
  a.pts1 = reinterpret_cast<const float*>(p->ws + p->lay.points);
  a.counts = counts;
  a.m0 = m0;
  a.M = M;
  a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(seed >> 32);
  a.contract = contract;
  a.n = p->n;
  a.d = p->d;
  a.maxP = p->maxP;
  a.maxN = p->maxN;
  a.mids_total = p->mids_total;
  a.keys = reinterpret_cast<uint16_t*>(p->ws + p->lay.keys);
  a.segs = reinterpret_cast<uint32_t*>(p->ws + p->lay.segs);
  a.max_tiles = p->max_tiles;
  a.seg_stride = p->max_tiles + 1;
  a.total_tiles = p->unit_off[p->n];
  a.nd_samples = p->tune_nd_samples;
  a.bucketed = (p->buckets > 0 && p->tune_buckets) ? 1 : 0;
  a.bk_rows = reinterpret_cast<const uint4*>(p->ws + p->lay.bk_rows);
  return a;
}

// Two-pass LAYERWISE counting over [m0, m0 + M) in batches that fit the
// scratch: pass A writes the keys of a batch, pass B folds them into counts.
// The plan's stream and events for overlapped histogram passes.
static hipError_t ensure_aux(const qtree_plan* p, int groups) {
  hipError_t e = hipSuccess;
  if (!p->aux) e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking);
  for (int g = 0; g < groups && e == hipSuccess; ++g) {
    if (!p->fork[g]) e = hipEventCreateWithFlags(&p->fork[g], hipEventDisableTiming);
  }
  if (e == hipSuccess && !p->join) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
  return e;
}

// First layer of group g of `groups`: the first groups - 1 groups get equal
// shares of the layers and the last a share tune_tail percent of theirs (its
// histogram pass is the one no sampling pass overlaps).
static int group_start(const qtree_plan* p, int groups, int g) {
  if (g <= 0) return 0;
  if (g >= groups) return p->n;
  const int64_t w = 100 * (int64_t)(groups - 1) + p->tune_tail;  // total weight
  int k = (int)((int64_t)p->n * 100 * g / w);
  k = std::max(k, g);  // every group keeps at least one layer
  return std::min(k, p->n - (groups - g));
}

// Two-pass forward over sample batches that fit the scratch.  The layers are
// split into `groups`; with more than one, the histogram pass of group g runs
// on the plan's stream while the sampling pass of group g + 1 runs on `s`
// (the passes of different layers touch disjoint scratch), and `s` waits for
// the histograms before the scratch is reused and before returning, so the
// call is complete on `s` like a single-stream one.
static hipError_t two_pass(const qtree_plan* p, qtree::FwdArgs a, bool zero, hipStream_t s,
                           const qtree::CountScratch& sc) {
  const uint64_t end = a.m0 + a.M;
  const uint64_t bs = p->d == 1 ? (uint64_t)sc.chunks * qtree::kChunk - 2
                                : (uint64_t)sc.chunks * qtree::kChunk;
  a.keys = sc.keys;
  a.segs = sc.segs;
  // automatic: four groups hide most of the 1-D histogram pass; for d >= 2
  // two (with the bucketed search that pass is a fifth of the forward, and
  // more launches add tails)
  const int want = p->tune_groups > 0 ? p->tune_groups : (p->d == 1 ? 4 : 2);
  const int groups = std::max(1, std::min(std::min(want, sc.max_groups), p->n));
  if (groups > 1) {
    hipError_t e = ensure_aux(p, groups);
    if (e != hipSuccess) return e;
  }
  bool first = zero;
  for (uint64_t lo = a.m0; lo < end; lo += bs) {
    const uint64_t mb = (end - lo) < bs ? (end - lo) : bs;
    qtree::FwdArgs b = a;
    b.m0 = lo;
    b.M = mb;
    uint64_t chunks;
    if (p->d == 1) {
      const uint64_t blocks = ((lo + mb - 1) >> 1) - (lo >> 1) + 1;
      chunks = (blocks + qtree::kChunk / 2 - 1) / (qtree::kChunk / 2);
    } else {
      chunks = (mb + qtree::kChunk - 1) / qtree::kChunk;
    }
    b.chunks = (int32_t)chunks;
    b.xcd_map = p->tune_xcd_map;
    b.first_batch = first ? 1 : 0;
    hipError_t e = hipSuccess;
    if (groups > 1 && lo > a.m0) e = hipStreamWaitEvent(s, p->join, 0);  // scratch reuse
    for (int g = 0; g < groups && e == hipSuccess; ++g) {
      const int k0 = group_start(p, groups, g);
      const int k1 = group_start(p, groups, g + 1);
      qtree::FwdArgs c = b;
      c.layer0 = k0;
      c.units = (k1 - k0) * b.chunks;
      c.units_per_xcd = (c.units + 7) / 8;
      c.tile0 = p->unit_off[k0];
      c.total_tiles = p->unit_off[k1] - p->unit_off[k0];
      // a split layer's histogram parts add into its count block: clear it
      // first (ordered before the histogram pass by the stream and the fork)
      bool any_split = false;
      for (int k = k0; k < k1; ++k) any_split = any_split || p->split[k] > 1;
      if (b.first_batch && any_split) e = qtree::launch_zero_split(c, k1 - k0, s);
      if (e == hipSuccess) e = qtree::launch_fwd_keys(c, s);
      if (e != hipSuccess) break;
      if (g == groups - 1 && p->trace_keys) e = hipEventRecord(p->trace_keys, s);
      if (e != hipSuccess) break;
      if (groups == 1) {
        e = qtree::launch_count_tiles(c, s);
      } else {
        e = hipEventRecord(p->fork[g], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->aux, p->fork[g], 0);
        if (e == hipSuccess) e = qtree::launch_count_tiles(c, p->aux);
      }
    }
    if (e == hipSuccess && groups > 1) e = hipEventRecord(p->join, p->aux);
    if (e != hipSuccess) return e;
    first = false;
  }
  return groups > 1 ? hipStreamWaitEvent(s, p->join, 0) : hipSuccess;
}

// Split each layer's M samples into chunks; one workgroup per (layer, chunk).
static void plan_units(qtree::FwdArgs& a, const qtree_plan* p) {
  uint64_t target;
  if (p->tune_chunk > 0) {
    target = (uint64_t)p->tune_chunk;
  } else if (p->d == 1) {
    target = 1ull << 16;
  } else {
    // keep the per-workgroup scan work near 2^27 point evaluations
    const uint64_t per_sample = 2ull * (uint64_t)p->maxN + 1;
    target = (1ull << 27) / per_sample;
    if (target < 2048) target = 2048;
  }
  uint64_t chunks = (a.M + target - 1) / target;
  if (chunks < 1) chunks = 1;
  if (chunks > (1u << 20)) chunks = 1u << 20;
  uint64_t len = (a.M + chunks - 1) / chunks;
  len += len & 1;  // even, so a chunk never splits a Philox block needlessly
  if (len == 0) len = 2;
  chunks = (a.M + len - 1) / len;
  if (chunks < 1) chunks = 1;
  a.chunk_len = len;
  a.chunks = (int32_t)chunks;
  a.units = a.n * a.chunks;
  a.units_per_xcd = (a.units + 7) / 8;
  a.xcd_map = p->tune_xcd_map;
}

qtree_status qtree_plan_trace(qtree_plan* plan, void* event_after_keys) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  plan->trace_keys = static_cast<hipEvent_t>(event_after_keys);
  return QTREE_OK;
}

qtree_status qtree_plan_buckets(const qtree_plan* plan, int32_t k, float* lo, float* scale,
                                int32_t* B) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (k < 0 || k > plan->n) return fail(QTREE_EINVAL, "layer index out of range");
  if (!lo || !scale || !B) return fail(QTREE_EINVAL, "NULL output");
  // the host image of the layer record is not kept: read it back
  qtree::LayerDev L{};
  const hipError_t e =
      hipMemcpy(&L, plan->ws + plan->lay.layers + sizeof(qtree::LayerDev) * (size_t)k,
                sizeof(L), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "layer record copy");
  for (int r = 0; r < 2; ++r) {
    lo[r] = L.bk_lo[r];
    scale[r] = L.bk_scale[r];
    B[r] = L.bk_B[r];
  }
  return QTREE_OK;
}

qtree_status qtree_plan_bucket_counts(const qtree_plan* plan, int32_t k, uint16_t* counts) {
  float lo[2], scale[2];
  int32_t B[2];
  const qtree_status st = qtree_plan_buckets(plan, k, lo, scale, B);
  if (st != QTREE_OK) return st;
  if (!counts) return fail(QTREE_EINVAL, "counts is NULL");
  if (B[0] == 0) return QTREE_OK;
  qtree::LayerDev L{};
  hipError_t e = hipMemcpy(&L, plan->ws + plan->lay.layers + sizeof(qtree::LayerDev) * (size_t)k,
                           sizeof(L), hipMemcpyDeviceToHost);
  const size_t nb = (size_t)B[0] * (size_t)B[1];
  std::vector<uint16_t> rows;
  try {
    rows.resize(nb * qtree::kBucketRow);
  } catch (const std::bad_alloc&) {
    return fail(QTREE_ENOMEM, "host copy of the bucket rows");
  }
  if (e == hipSuccess)
    e = hipMemcpy(rows.data(),
                  plan->ws + plan->lay.bk_rows + sizeof(uint16_t) * qtree::kBucketRow * (size_t)L.bk_off,
                  sizeof(uint16_t) * rows.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "bucket rows copy");
  for (size_t t = 0; t < nb; ++t) counts[t] = rows[t * qtree::kBucketRow];  // entry 0: the count
  return QTREE_OK;
}

qtree_status qtree_plan_cell_search(const qtree_plan* plan, int32_t* guide_k,
                                    int32_t* guide_buckets) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  // the choice of fwd_args: d = 1 tables that fit beside the midpoints
  int32_t k = plan->d == 1 ? plan->gt_Kmax : -1;
  if (k >= 0 && qtree::keys_lds_1d_guide(plan->maxP, plan->gt_Bmax, plan->max_tiles) > 160 * 1024)
    k = -1;
  if (guide_k) *guide_k = k;
  if (guide_buckets) *guide_buckets = k >= 0 ? plan->gt_Bmax : 0;
  return QTREE_OK;
}

int64_t qtree_plan_batch_samples(const qtree_plan* p) {
  if (!p || !p->two_pass_ok) return 0;
  return p->d == 1 ? p->batch_chunks * qtree::kChunk - 2 : p->batch_chunks * qtree::kChunk;
}

qtree_status qtree_plan_tune(qtree_plan* plan, int32_t key, int64_t value) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (key == QTREE_TUNE_CHUNK) {
    if (value < 0 || value > (1ll << 31)) return fail(QTREE_EINVAL, "chunk out of range");
    plan->tune_chunk = value;
    return QTREE_OK;
  }
  if (key == QTREE_TUNE_COUNT) {
    if (value < 0 || value > 2) return fail(QTREE_EINVAL, "count mode must be 0, 1 or 2");
    if (value == 2 && !plan->two_pass_shape)
      return fail(QTREE_EUNSUPPORTED, "count blocks too large for two-pass counting");
    plan->tune_count = (int32_t)value;
    return QTREE_OK;
  }
  if (key == QTREE_TUNE_GROUPS) {
    if (value < 0 || value > qtree_plan::kMaxGroups)
      return fail(QTREE_EINVAL, "groups must be in 0..8");
    plan->tune_groups = (int32_t)value;
    return QTREE_OK;
  }
  if (key == QTREE_TUNE_TAIL) {
    if (value < 10 || value > 100) return fail(QTREE_EINVAL, "tail share must be 10..100");
    plan->tune_tail = (int32_t)value;
    return QTREE_OK;
  }
  if (key == QTREE_TUNE_ND_SAMPLES) {
    if (value != 4 && value != 8) return fail(QTREE_EINVAL, "samples per lane must be 4 or 8");
    plan->tune_nd_samples = (int32_t)value;
    return QTREE_OK;
  }
  if (key == QTREE_TUNE_XCD_MAP) {
    if (value != 0 && value != 1) return fail(QTREE_EINVAL, "xcd map must be 0 or 1");
    plan->tune_xcd_map = (int32_t)value;
    return QTREE_OK;
  }
  if (key == QTREE_TUNE_BUCKETS) {
    if (value != 0 && value != 1) return fail(QTREE_EINVAL, "buckets must be 0 or 1");
    plan->tune_buckets = (int32_t)value;
    return QTREE_OK;
  }
  return fail(QTREE_EINVAL, "unknown tuning key");
}

static qtree_status transitions_impl(const qtree_plan* plan, uint64_t m0, uint64_t M,
                                     uint64_t seed, uint32_t contract_id, qtree_mode mode,
                                     int32_t* counts, void* stream, bool zero,
                                     const qtree::CountScratch* scratch = nullptr) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!counts) return fail(QTREE_EINVAL, "counts is NULL");
  if (reinterpret_cast<uintptr_t>(counts) % 16)
    return fail(QTREE_EINVAL, "counts must be 16-byte aligned");
  if (mode != QTREE_LAYERWISE && mode != QTREE_PATHWISE)
    return fail(QTREE_EINVAL, "unknown mode");
  if (M >= (1ull << 31)) return fail(QTREE_EOVERFLOW, "M must be < 2^31");
  if (m0 + M > (1ull << 32)) return fail(QTREE_EOVERFLOW, "m0 + M must be <= 2^32");
  // the two-pass scratch: the plan's workspace, or the caller's
  qtree::CountScratch sc;
  if (scratch) {
    sc = *scratch;
  } else {
    sc.keys = reinterpret_cast<uint16_t*>(plan->ws + plan->lay.keys);
    sc.segs = reinterpret_cast<uint32_t*>(plan->ws + plan->lay.segs);
    sc.chunks = plan->two_pass_ok ? plan->batch_chunks : 0;
    sc.max_groups = qtree_plan::kMaxGroups;
  }
  const bool two_ok = plan->two_pass_shape && sc.chunks > 0;
  const bool two = mode == QTREE_LAYERWISE && M > 0 &&
                   (plan->tune_count == 2 || (plan->tune_count == 0 && two_ok));
  if (two && !two_ok)
    return fail(QTREE_EUNSUPPORTED, "two-pass counting needs scratch this call does not have");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (zero && !two) {
    e = qtree::launch_zero_i32(counts, plan->entries, s);
    if (e != hipSuccess) return hip_fail(e, "zero fill");
  }
  if (M == 0) return QTREE_OK;
  qtree::FwdArgs a = fwd_args(plan, m0, M, seed, contract_id, counts);
  if (mode == QTREE_PATHWISE) {
    e = qtree::launch_fwd_path(a, s);
  } else if (two) {
    e = two_pass(plan, a, zero, s, sc);
  } else {
    plan_units(a, plan);
    e = plan->d == 1 ? qtree::launch_fwd_layer_1d(a, s) : qtree::launch_fwd_layer_nd(a, s);
  }
  if (e != hipSuccess) return hip_fail(e, "forward kernel launch");
  return QTREE_OK;
}

}  // extern "C"

namespace qtree {
// Forward step whose two-pass counting uses `bytes` of caller scratch at
// `base` (keys [n][chunks][kChunk], then segment starts [n][chunks][max
// tiles + 1]) and one layer group (no stream or event of the plan).
qtree_status transitions_on_scratch(const qtree_plan* plan, uint64_t m0, uint64_t M,
                                    uint64_t seed, uint32_t contract_id, qtree_mode mode,
                                    int32_t* counts, void* stream, void* base, size_t bytes) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  CountScratch sc;
  sc.max_groups = 1;
  sc.chunks = 0;
  const bool layerwise_two = mode == QTREE_LAYERWISE && M > 0 && plan->tune_count != 1 &&
                             plan->two_pass_shape;
  if (layerwise_two) {
    const size_t key_chunk = sizeof(uint16_t) * kChunk;
    const size_t seg_chunk = sizeof(uint32_t) * (size_t)(plan->max_tiles + 1);
    const size_t per = (size_t)plan->n * (key_chunk + seg_chunk);
    int64_t c = (int64_t)(bytes / per);
    while (c > 0 && align_up((size_t)plan->n * (size_t)c * key_chunk, 256) +
                            (size_t)plan->n * (size_t)c * seg_chunk > bytes)
      --c;
    if (c < 1)
      return fail(QTREE_EUNSUPPORTED,
                  "one chunk per layer needs " + std::to_string(per) + " bytes of scratch, " +
                      std::to_string(bytes) + " available");
    sc.chunks = c;
    sc.keys = static_cast<uint16_t*>(base);
    sc.segs = reinterpret_cast<uint32_t*>(
        static_cast<char*>(base) + align_up((size_t)plan->n * (size_t)c * key_chunk, 256));
  }
  return transitions_impl(plan, m0, M, seed, contract_id, mode, counts, stream, true, &sc);
}
}  // namespace qtree

extern "C" {

qtree_status qtree_transitions(const qtree_plan* plan, uint64_t m0, uint64_t M, uint64_t seed,
                               uint32_t contract_id, qtree_mode mode, int32_t* counts,
                               void* stream) {
  return transitions_impl(plan, m0, M, seed, contract_id, mode, counts, stream, true);
}

qtree_status qtree_transitions_add(const qtree_plan* plan, uint64_t m0, uint64_t M, uint64_t seed,
                                   uint32_t contract_id, qtree_mode mode, int32_t* counts,
                                   void* stream) {
  return transitions_impl(plan, m0, M, seed, contract_id, mode, counts, stream, false);
}

int64_t qtree_plan_get_tune(const qtree_plan* plan, int32_t key) {
  if (!plan) return -1;
  switch (key) {
    case QTREE_TUNE_CHUNK: return plan->tune_chunk;
    case QTREE_TUNE_XCD_MAP: return plan->tune_xcd_map;
    case QTREE_TUNE_COUNT: return plan->tune_count;
    case QTREE_TUNE_GROUPS: return plan->tune_groups;
    case QTREE_TUNE_ND_SAMPLES: return plan->tune_nd_samples;
    case QTREE_TUNE_TAIL: return plan->tune_tail;
    case QTREE_TUNE_BUCKETS: return plan->tune_buckets;
  }
  return -1;
}

qtree_status qtree_plan_autotune(qtree_plan* plan, uint64_t M, uint64_t seed, int32_t* counts,
                                 void* stream, double* best_ms) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!counts) return fail(QTREE_EINVAL, "counts is NULL");
  if (M < 1 || M >= (1ull << 31)) return fail(QTREE_EOVERFLOW, "M must be in 1 .. 2^31 - 1");
  // candidates: (groups, tail share, samples per lane)
  struct Cand {
    int groups, tail, nds;
  };
  std::vector<Cand> cand;
  if (plan->d == 1) {
    cand.push_back({1, 100, 8});
    for (int g : {2, 4, 6, 8})
      for (int t : {100, 50, 33}) cand.push_back({g, t, 8});
  } else {
    for (int nds : {8, 4})
      for (int g : {1, 2}) cand.push_back({g, 100, nds});
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t keep_g = plan->tune_groups, keep_t = plan->tune_tail,
                keep_s = plan->tune_nd_samples;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = -1.0;
  Cand win = cand[0];
  qtree_status st = QTREE_OK;
  // one warm-up run, then every candidate kReps times (its fastest run counts)
  constexpr int kReps = 3;
  for (size_t i = 0; i <= cand.size() * kReps && e == hipSuccess && st == QTREE_OK; ++i) {
    const Cand c = cand[i == 0 ? 0 : (i - 1) / kReps];
    plan->tune_groups = c.groups;
    plan->tune_tail = c.tail;
    plan->tune_nd_samples = c.nds;
    e = hipEventRecord(e0, s);
    if (e != hipSuccess) break;
    st = transitions_impl(plan, 0, M, seed, 0, QTREE_LAYERWISE, counts, stream, true);
    if (st != QTREE_OK) break;
    e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && i > 0 && (best < 0.0 || ms < best)) {
      best = ms;
      win = c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != QTREE_OK || e != hipSuccess) {
    plan->tune_groups = keep_g;
    plan->tune_tail = keep_t;
    plan->tune_nd_samples = keep_s;
    return st != QTREE_OK ? st : hip_fail(e, "autotune timing");
  }
  plan->tune_groups = win.groups;
  plan->tune_tail = win.tail;
  plan->tune_nd_samples = win.nds;
  if (best_ms) *best_ms = best;
  return QTREE_OK;
}

// Samples of row i of layer k (the rule of the device kernel).
static uint64_t strat_row(const qtree_plan* plan, int k, int i, uint64_t M, int alloc) {
  if (alloc == 0) return M;
  const double* e = plan->edges.data() + plan->pt_off[k] + k;
  const long long r = (long long)std::rint((double)M * (e[i + 1] - e[i]));
  return r > 1 ? (uint64_t)r : 1ull;
}

static qtree_status strat_args(const qtree_plan* plan, uint64_t M, int32_t alloc, uint64_t seed,
                               uint32_t contract_id, qtree::StratArgs& a) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (plan->d != 1) return fail(QTREE_EUNSUPPORTED, "stratified sampling is for d = 1");
  if (alloc != 0 && alloc != 1) return fail(QTREE_EINVAL, "alloc must be 0 or 1");
  if (M < 1 || M >= (1ull << 31)) return fail(QTREE_EOVERFLOW, "M must be in 1 .. 2^31 - 1");
  for (int k = 0; k < plan->n; ++k) {
    const float L = plan->marg_L[k];
    if (plan->N[k] > 1 && !(L > 0.0f && std::isfinite(L)))
      return fail(QTREE_EINVAL, "stratified sampling needs L_k > 0 on layers with N_k > 1");
  }
  if (plan->maxP > 8192) return fail(QTREE_EUNSUPPORTED, "N above 8192");
  if (qtree::strat_lds_bytes(plan->maxP, plan->maxN) > 160 * 1024)
    return fail(QTREE_EUNSUPPORTED, "count rows do not fit in LDS");
  a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
  a.mids = reinterpret_cast<const float*>(plan->ws + plan->lay.aux);
  a.guide = reinterpret_cast<const uint16_t*>(plan->ws + plan->lay.guide);
  a.gt_Kmax = plan->gt_Kmax;
  a.gt_Bmax = plan->gt_Bmax;
  a.edges = reinterpret_cast<const double*>(plan->ws + plan->lay.edges);
  a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(seed >> 32);
  a.contract = contract_id;
  a.M = M;
  a.alloc = alloc;
  a.n = plan->n;
  a.maxP = plan->maxP;
  a.maxN = plan->maxN;
  return QTREE_OK;
}

// Work list of the stratified counts: every tile of kStratRows rows of every
// layer, cut into segments of at most kStratSegment samples.
static std::vector<qtree::StratUnit> strat_units(const qtree_plan* plan, uint64_t M, int alloc,
                                                 bool* any_split) {
  std::vector<qtree::StratUnit> u;
  *any_split = false;
  for (int k = 0; k < plan->n; ++k) {
    for (int i0 = 0; i0 < plan->N[k]; i0 += qtree::kStratRows) {
      uint64_t total = 0;
      for (int i = i0; i < std::min(i0 + qtree::kStratRows, (int)plan->N[k]); ++i)
        total += strat_row(plan, k, i, M, alloc);
      const uint64_t segs = (total + qtree::kStratSegment - 1) / qtree::kStratSegment;
      if (segs > 1) *any_split = true;
      for (uint64_t g = 0; g < segs; ++g) {
        qtree::StratUnit x{};
        x.k = k;
        x.i0 = i0;
        x.split = segs > 1 ? 1 : 0;
        x.s0 = g * qtree::kStratSegment;
        x.s1 = std::min(total, (g + 1) * qtree::kStratSegment);
        u.push_back(x);
      }
    }
  }
  return u;
}

size_t qtree_strat_workspace_size(const qtree_plan* plan, uint64_t M, int32_t alloc) {
  qtree::StratArgs a{};
  if (strat_args(plan, M, alloc, 0, 0, a) != QTREE_OK) return 0;
  bool split = false;
  return sizeof(qtree::StratUnit) * std::max<size_t>(1, strat_units(plan, M, alloc, &split).size());
}

qtree_status qtree_transitions_stratified(const qtree_plan* plan, uint64_t M, int32_t alloc,
                                          uint64_t seed, uint32_t contract_id, int32_t* counts,
                                          void* workspace, size_t workspace_bytes,
                                          void* stream) {
  qtree::StratArgs a{};
  qtree_status st = strat_args(plan, M, alloc, seed, contract_id, a);
  if (st != QTREE_OK) return st;
  if (!counts || !workspace) return fail(QTREE_EINVAL, "counts or workspace is NULL");
  bool split = false;
  const std::vector<qtree::StratUnit> units = strat_units(plan, M, alloc, &split);
  if (units.size() >= (1u << 31)) return fail(QTREE_EOVERFLOW, "too many work units");
  if (workspace_bytes < sizeof(qtree::StratUnit) * units.size())
    return fail(QTREE_ENOMEM, "workspace smaller than qtree_strat_workspace_size");
  a.counts = counts;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* dev_units = static_cast<qtree::StratUnit*>(workspace);
  // the copy from pageable memory is staged before the call returns
  hipError_t e = hipMemcpyAsync(dev_units, units.data(), sizeof(qtree::StratUnit) * units.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess && split) e = qtree::launch_zero_i32(counts, plan->entries, s);
  if (e == hipSuccess) e = qtree::launch_strat(a, dev_units, (int)units.size(), s);
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "stratified launch");
}

qtree_status qtree_strat_band(const qtree_plan* plan, int64_t* values, int64_t* row_off,
                              int32_t* row_lo) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (plan->d != 1) return fail(QTREE_EUNSUPPORTED, "banded counts are for d = 1");
  const int64_t R = plan->pt_off[plan->n];
  if (values) *values = plan->band_off[(size_t)R];
  if (row_off) std::memcpy(row_off, plan->band_off.data(), sizeof(int64_t) * (size_t)(R + 1));
  if (row_lo) std::memcpy(row_lo, plan->band_lo.data(), sizeof(int32_t) * (size_t)R);
  return QTREE_OK;
}

qtree_status qtree_transitions_stratified_banded(const qtree_plan* plan, uint64_t M,
                                                 int32_t alloc, uint64_t seed,
                                                 uint32_t contract_id, int32_t* band,
                                                 uint32_t* overflow, void* workspace,
                                                 size_t workspace_bytes, void* stream) {
  qtree::StratArgs a{};
  qtree_status st = strat_args(plan, M, alloc, seed, contract_id, a);
  if (st != QTREE_OK) return st;
  if (!band || !overflow || !workspace)
    return fail(QTREE_EINVAL, "band, overflow or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(band) % 4 || reinterpret_cast<uintptr_t>(overflow) % 4)
    return fail(QTREE_EINVAL, "band and overflow must be 4-byte aligned");
  bool split = false;
  const std::vector<qtree::StratUnit> units = strat_units(plan, M, alloc, &split);
  if (units.size() >= (1u << 31)) return fail(QTREE_EOVERFLOW, "too many work units");
  if (workspace_bytes < sizeof(qtree::StratUnit) * units.size())
    return fail(QTREE_ENOMEM, "workspace smaller than qtree_strat_workspace_size");
  const int64_t R = plan->pt_off[plan->n];
  a.counts = band;
  a.band_off = reinterpret_cast<const int64_t*>(plan->ws + plan->lay.band);
  a.band_lo = reinterpret_cast<const int32_t*>(plan->ws + plan->lay.band +
                                               sizeof(int64_t) * (size_t)(R + 1));
  a.overflow = overflow;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* dev_units = static_cast<qtree::StratUnit*>(workspace);
  hipError_t e = hipMemcpyAsync(dev_units, units.data(), sizeof(qtree::StratUnit) * units.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = qtree::launch_zero_i32(reinterpret_cast<int32_t*>(overflow), 1, s);
  if (e == hipSuccess && split)
    e = qtree::launch_zero_i32(band, plan->band_off[(size_t)R], s);
  if (e == hipSuccess) e = qtree::launch_strat(a, dev_units, (int)units.size(), s);
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "stratified launch");
}

int64_t qtree_strat_row(const qtree_plan* plan, int32_t k, int32_t i, uint64_t M, int32_t alloc) {
  if (!plan || plan->d != 1 || k < 0 || k >= plan->n || i < 0 || i >= plan->N[k]) return -1;
  if ((alloc != 0 && alloc != 1) || M < 1 || M >= (1ull << 31)) return -1;
  return (int64_t)strat_row(plan, k, i, M, alloc);
}

qtree_status qtree_strat_samples(const qtree_plan* plan, int32_t k, int32_t i, uint64_t M,
                                 int32_t alloc, uint64_t t0, int64_t count, uint64_t seed,
                                 uint32_t contract_id, float* x, float* y, void* stream) {
  qtree::StratArgs a{};
  qtree_status st = strat_args(plan, M, alloc, seed, contract_id, a);
  if (st != QTREE_OK) return st;
  if (k < 0 || k >= plan->n) return fail(QTREE_EINVAL, "layer index out of range");
  if (i < 0 || i >= plan->N[k]) return fail(QTREE_EINVAL, "row index out of range");
  if (count < 0) return fail(QTREE_EINVAL, "count must be >= 0");
  if (t0 + (uint64_t)count > strat_row(plan, k, i, M, alloc))
    return fail(QTREE_EINVAL, "samples beyond the row's sample count");
  if (count == 0) return QTREE_OK;
  if (!x || !y) return fail(QTREE_EINVAL, "NULL array");
  const hipError_t e =
      qtree::launch_strat_samples(a, k, i, t0, count, x, y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "stratified samples launch");
}

static qtree_status bdp_impl(const qtree_plan* plan, const int32_t* counts, const double* phi,
                             int32_t n_pay, double* V, double* V0_host, void* stream,
                             bool banded);

qtree_status qtree_bdp(const qtree_plan* plan, const int32_t* counts, const double* phi,
                       int32_t n_pay, double* V, double* V0_host, void* stream) {
  return bdp_impl(plan, counts, phi, n_pay, V, V0_host, stream, false);
}

qtree_status qtree_bdp_banded(const qtree_plan* plan, const int32_t* band, const double* phi,
                              int32_t n_pay, double* V, double* V0_host, void* stream) {
  if (plan && plan->d != 1) return fail(QTREE_EUNSUPPORTED, "banded counts are for d = 1");
  return bdp_impl(plan, band, phi, n_pay, V, V0_host, stream, true);
}

static qtree_status bdp_impl(const qtree_plan* plan, const int32_t* counts, const double* phi,
                             int32_t n_pay, double* V, double* V0_host, void* stream,
                             bool banded) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!counts || !phi || !V) return fail(QTREE_EINVAL, "counts, phi and V must be non-NULL");
  if (n_pay < 1) return fail(QTREE_EINVAL, "n_pay must be >= 1");
  if (n_pay > (1 << 20)) return fail(QTREE_EINVAL, "n_pay must be <= 2^20");
  hipStream_t s = static_cast<hipStream_t>(stream);
  qtree::BdpArgs a{};
  a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
  a.counts = counts;
  a.phi = phi;
  a.V = V;
  a.P = plan->points;
  a.n_pay = n_pay;
  const int n = plan->n;
  if (banded) {
    a.band_off = reinterpret_cast<const int64_t*>(plan->ws + plan->lay.band);
    a.band_lo = reinterpret_cast<const int32_t*>(plan->ws + plan->lay.band +
                                                 sizeof(int64_t) * (size_t)(plan->pt_off[n] + 1));
  }
  hipError_t e = qtree::launch_copy_last_layer(a, plan->pt_off[n], plan->N[n], s);
  if (e != hipSuccess) return hip_fail(e, "bdp launch");
  for (int k = n - 1; k >= 0; --k) {
    e = qtree::launch_bdp_layer(a, k, plan->N[k], plan->N[k + 1], plan->pt_off[k],
                                plan->pt_off[k + 1], plan->cnt_off[k], s);
    if (e != hipSuccess) return hip_fail(e, "bdp launch");
  }
  if (V0_host) {
    e = hipMemcpy2DAsync(V0_host, sizeof(double), V, sizeof(double) * (size_t)plan->points,
                         sizeof(double), (size_t)n_pay, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "V0 copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  }
  return QTREE_OK;
}

qtree_status qtree_payoff_batch(const qtree_plan* plan, int32_t n_pay, const int32_t* kind,
                                const double* S0, const double* K, const double* r,
                                const double* Tm, const double* sigma, const double* mix,
                                double* phi, void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (n_pay < 0) return fail(QTREE_EINVAL, "n_pay must be >= 0");
  if (n_pay == 0) return QTREE_OK;
  if (!kind || !S0 || !K || !r || !Tm || !sigma || !phi)
    return fail(QTREE_EINVAL, "NULL array");
  for (int q = 0; q < n_pay; ++q) {
    if (kind[q] < 0 || kind[q] > 3) return fail(QTREE_EINVAL, "kind must be in 0..3");
    if (!(Tm[q] > 0.0) || !std::isfinite(Tm[q]) || !std::isfinite(S0[q]) ||
        !std::isfinite(K[q]) || !std::isfinite(r[q]))
      return fail(QTREE_EINVAL, "contract parameters must be finite, Tm > 0");
    for (int c = 0; c < plan->d; ++c)
      if (!std::isfinite(sigma[(size_t)q * plan->d + c]))
        return fail(QTREE_EINVAL, "sigma must be finite");
    if (mix)
      for (int c = 0; c < plan->d * plan->d; ++c)
        if (!std::isfinite(mix[(size_t)q * plan->d * plan->d + c]))
          return fail(QTREE_EINVAL, "mix must be finite");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int q0 = 0; q0 < n_pay; q0 += qtree::kPayoffGroup) {
    qtree::PayoffArgs a{};
    a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
    a.pts1 = reinterpret_cast<const float*>(plan->ws + plan->lay.points);
    a.pts = reinterpret_cast<const float4*>(plan->ws + plan->lay.points);
    a.phi = phi + (size_t)q0 * plan->points;
    a.P = plan->points;
    a.n = plan->n;
    a.d = plan->d;
    a.maxN = plan->maxN;
    a.count = (n_pay - q0) < qtree::kPayoffGroup ? (n_pay - q0) : qtree::kPayoffGroup;
    for (int q = 0; q < a.count; ++q) {
      qtree::Contract& C = a.c[q];
      C.kind = kind[q0 + q];
      C.S0 = S0[q0 + q];
      C.K = K[q0 + q];
      C.r = r[q0 + q];
      C.Tm = Tm[q0 + q];
      for (int c = 0; c < plan->d; ++c) C.sigma[c] = sigma[(size_t)(q0 + q) * plan->d + c];
      C.has_mix = mix ? 1 : 0;
      const int dd = plan->d * plan->d;
      for (int c = 0; c < dd; ++c) C.mix[c] = mix ? mix[(size_t)(q0 + q) * dd + c] : 0.0;
    }
    hipError_t e = qtree::launch_payoff(a, st);
    if (e != hipSuccess) return hip_fail(e, "payoff launch");
  }
  return QTREE_OK;
}

// Layout of the transition-weight workspace: layer offsets, row bands, weights.
struct PiLayout {
  size_t off, band, pi, total;
  int64_t rows, weights;
};
static PiLayout pi_layout(const qtree_plan* p) {
  PiLayout l{};
  l.rows = p->pt_off[p->n];
  l.weights = 0;
  for (int k = 0; k < p->n; ++k) l.weights += (int64_t)p->N[k] * ((p->N[k + 1] + 3) & ~3);
  l.off = 0;
  l.band = align_up(sizeof(int64_t) * (size_t)p->n, 256);
  l.pi = align_up(l.band + sizeof(int2) * (size_t)l.rows, 256);
  l.total = l.pi + sizeof(double) * (size_t)l.weights;
  return l;
}

qtree_status qtree_pi_workspace_size(const qtree_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(QTREE_EINVAL, "plan and bytes must be non-NULL");
  *bytes = pi_layout(plan).total;
  return QTREE_OK;
}

qtree_status qtree_pi(const qtree_plan* plan, const int32_t* counts, void* pi, size_t pi_bytes,
                      void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!counts || !pi) return fail(QTREE_EINVAL, "counts and pi must be non-NULL");
  if (reinterpret_cast<uintptr_t>(pi) % 256) return fail(QTREE_EINVAL, "pi must be 256-byte aligned");
  const PiLayout l = pi_layout(plan);
  if (pi_bytes < l.total)
    return fail(QTREE_ENOMEM, "pi needs " + std::to_string(l.total) + " bytes");
  char* base = static_cast<char*>(pi);
  qtree::PiArgs a{};
  a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
  a.counts = counts;
  a.pi_off = reinterpret_cast<const int64_t*>(base + l.off);
  a.band = reinterpret_cast<int2*>(base + l.band);
  a.pi = reinterpret_cast<double*>(base + l.pi);
  a.rows = l.rows;
  a.n = plan->n;
  hipError_t e = qtree::launch_pi(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "pi launch");
}

qtree_status qtree_bdp_many(const qtree_plan* plan, const void* pi, size_t pi_bytes, int64_t n_q,
                            const qtree_payoff_spec* specs, double* V0, void* stream) {
  static_assert(sizeof(qtree_payoff_spec) == sizeof(qtree::Contract),
                "qtree_payoff_spec must match the device contract record");
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!pi) return fail(QTREE_EINVAL, "pi is NULL");
  if (n_q < 0) return fail(QTREE_EINVAL, "n_q must be >= 0");
  if (n_q == 0) return QTREE_OK;
  if (!specs || !V0) return fail(QTREE_EINVAL, "specs and V0 must be non-NULL");
  if (reinterpret_cast<uintptr_t>(specs) % 8 || reinterpret_cast<uintptr_t>(V0) % 8)
    return fail(QTREE_EINVAL, "specs and V0 must be 8-byte aligned");
  const PiLayout l = pi_layout(plan);
  if (pi_bytes < l.total)
    return fail(QTREE_ENOMEM, "pi needs " + std::to_string(l.total) + " bytes");
  if (qtree::bdp_many_maxr(plan->maxN) < 0)
    return fail(QTREE_EUNSUPPORTED, "qtree_bdp_many takes layers of at most 256 points");
  const char* base = static_cast<const char*>(pi);
  qtree::ManyArgs a{};
  a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
  a.pts1 = reinterpret_cast<const float*>(plan->ws + plan->lay.points);
  a.pts = reinterpret_cast<const float4*>(plan->ws + plan->lay.points);
  a.pi_off = reinterpret_cast<const int64_t*>(base + l.off);
  a.band = reinterpret_cast<const int2*>(base + l.band);
  a.pi = reinterpret_cast<const double*>(base + l.pi);
  a.specs = reinterpret_cast<const qtree::Contract*>(specs);
  a.V0 = V0;
  a.nq = n_q;
  a.n = plan->n;
  a.d = plan->d;
  a.max_n = plan->maxN;
  a.np_max = (plan->maxN + 3) & ~3;
  hipError_t e = qtree::launch_bdp_many(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "bdp_many launch");
}

qtree_status qtree_bdp_many_trees(int32_t n_trees, const qtree_plan* const* plans,
                                  const void* const* pi, const size_t* pi_bytes,
                                  const int64_t* q_begin, const qtree_payoff_spec* specs,
                                  double* V0, void* workspace, size_t workspace_bytes,
                                  void* stream) {
  static_assert(sizeof(qtree::ManyTree) == 80, "the header states 80 bytes per tree record");
  if (n_trees < 0) return fail(QTREE_EINVAL, "n_trees must be >= 0");
  if (n_trees == 0) return QTREE_OK;
  if (!plans || !pi || !pi_bytes || !q_begin)
    return fail(QTREE_EINVAL, "plans, pi, pi_bytes and q_begin must be non-NULL");
  if (q_begin[0] < 0) return fail(QTREE_EINVAL, "q_begin[0] must be >= 0");
  int d = 0, max_n = 0;
  int64_t blocks = 0;
  std::vector<int> order((size_t)n_trees);
  for (int t = 0; t < n_trees; ++t) {
    const qtree_plan* p = plans[t];
    if (!p || !pi[t]) return fail(QTREE_EINVAL, "plan or pi " + std::to_string(t) + " is NULL");
    if (t == 0) d = p->d;
    if (p->d != d) return fail(QTREE_EINVAL, "every tree must have the same dimension");
    if (reinterpret_cast<uintptr_t>(pi[t]) % 256) return fail(QTREE_EINVAL, "pi must be 256-byte aligned");
    if (pi_bytes[t] < pi_layout(p).total)
      return fail(QTREE_ENOMEM, "pi " + std::to_string(t) + " is smaller than qtree_pi_workspace_size");
    if (q_begin[t + 1] < q_begin[t]) return fail(QTREE_EINVAL, "q_begin must be nondecreasing");
    max_n = std::max(max_n, p->maxN);
    blocks += (q_begin[t + 1] - q_begin[t] + 63) / 64;
    order[(size_t)t] = t;
  }
  if (q_begin[n_trees] > q_begin[0] && (!specs || !V0))
    return fail(QTREE_EINVAL, "specs and V0 must be non-NULL");
  if (reinterpret_cast<uintptr_t>(specs) % 8 || reinterpret_cast<uintptr_t>(V0) % 8)
    return fail(QTREE_EINVAL, "specs and V0 must be 8-byte aligned");
  if (qtree::bdp_many_maxr(max_n) < 0)
    return fail(QTREE_EUNSUPPORTED, "qtree_bdp_many takes layers of at most 256 points");
  if (blocks >= (1ll << 31)) return fail(QTREE_EOVERFLOW, "too many contracts");
  if (!workspace || workspace_bytes < sizeof(qtree::ManyTree) * (size_t)n_trees)
    return fail(QTREE_ENOMEM, "workspace must hold " + std::to_string(n_trees) + " tree records");
  if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(QTREE_EINVAL, "workspace must be 16-byte aligned");
  if (blocks == 0) return QTREE_OK;
  // trees with the most layers (the longest workgroups) first
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return plans[x]->n > plans[y]->n; });
  std::vector<qtree::ManyTree> tab((size_t)n_trees);
  int32_t blk = 0;
  for (int r = 0; r < n_trees; ++r) {
    const int t = order[(size_t)r];
    const qtree_plan* p = plans[t];
    const PiLayout l = pi_layout(p);
    const char* base = static_cast<const char*>(pi[t]);
    qtree::ManyTree& T = tab[(size_t)r];
    T.layers = reinterpret_cast<const qtree::LayerDev*>(p->ws + p->lay.layers);
    T.pts1 = reinterpret_cast<const float*>(p->ws + p->lay.points);
    T.pts = reinterpret_cast<const float4*>(p->ws + p->lay.points);
    T.pi_off = reinterpret_cast<const int64_t*>(base + l.off);
    T.band = reinterpret_cast<const int2*>(base + l.band);
    T.pi = reinterpret_cast<const double*>(base + l.pi);
    T.q0 = q_begin[t];
    T.nq = q_begin[t + 1] - q_begin[t];
    T.blk0 = blk;
    T.n = p->n;
    blk += (int32_t)((T.nq + 63) / 64);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(workspace, tab.data(), sizeof(qtree::ManyTree) * tab.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "tree table copy");
  qtree::ManyArgs a{};
  a.specs = reinterpret_cast<const qtree::Contract*>(specs);
  a.V0 = V0;
  a.d = d;
  a.max_n = max_n;
  a.np_max = (max_n + 3) & ~3;
  a.trees = static_cast<const qtree::ManyTree*>(workspace);
  a.n_trees = n_trees;
  a.blocks = (int32_t)blocks;
  e = qtree::launch_bdp_many(a, s);
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "bdp_many launch");
}

qtree_status qtree_payoff(const qtree_plan* plan, int32_t kind, double S0, double K, double r,
                          double Tm, const double* sigma, const double* mix, double* phi,
                          void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!sigma) return fail(QTREE_EINVAL, "sigma is NULL");
  return qtree_payoff_batch(plan, 1, &kind, &S0, &K, &r, &Tm, sigma, mix, phi, stream);
}

qtree_status qtree_payoff_forward(const qtree_plan* plan, double S0, double K, double r,
                                  double Tm, const double* sigma, const double* mix, double* v,
                                  void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!sigma || !v) return fail(QTREE_EINVAL, "sigma and v must be non-NULL");
  if (!(Tm > 0.0) || !std::isfinite(Tm) || !std::isfinite(S0) || !std::isfinite(K) ||
      !std::isfinite(r))
    return fail(QTREE_EINVAL, "contract parameters must be finite, Tm > 0");
  const int d = plan->d;
  for (int c = 0; c < d; ++c)
    if (!std::isfinite(sigma[c])) return fail(QTREE_EINVAL, "sigma must be finite");
  if (mix)
    for (int c = 0; c < d * d; ++c)
      if (!std::isfinite(mix[c])) return fail(QTREE_EINVAL, "mix must be finite");
  qtree::ForwardArgs a{};
  a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
  a.pts1 = reinterpret_cast<const float*>(plan->ws + plan->lay.points);
  a.pts = reinterpret_cast<const float4*>(plan->ws + plan->lay.points);
  a.v = v;
  a.n = plan->n;
  a.d = d;
  a.maxN = plan->maxN;
  a.S0 = S0;
  a.K = K;
  a.r = r;
  a.Tm = Tm;
  for (int b = 0; b < d; ++b) {  // w = mix' sigma, summed over a in order
    a.w[b] = 0.0;
    for (int c = 0; c < d; ++c) a.w[b] += sigma[c] * (mix ? mix[c * d + b] : (c == b ? 1.0 : 0.0));
  }
  const hipError_t e = qtree::launch_forward_payoff(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "forward payoff launch");
}

qtree_status qtree_swing(const qtree_plan* plan, const int32_t* counts, const double* v,
                         int32_t Qmin, int32_t Qmax, double* P, double* P0_host, void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (!counts || !v || !P) return fail(QTREE_EINVAL, "counts, v and P must be non-NULL");
  if (Qmin < 0 || Qmin > Qmax || Qmax > plan->n)
    return fail(QTREE_EINVAL, "need 0 <= Qmin <= Qmax <= n");
  if (Qmax > qtree::kSwingMaxQ) return fail(QTREE_EUNSUPPORTED, "Qmax above 2046");
  qtree::SwingArgs a{};
  a.layers = reinterpret_cast<const qtree::LayerDev*>(plan->ws + plan->lay.layers);
  a.counts = counts;
  a.v = v;
  a.P = P;
  a.Pts = plan->points;
  a.n = plan->n;
  a.Qmin = Qmin;
  a.Qmax = Qmax;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = qtree::launch_swing(a, plan->N.data(), s);
  if (e != hipSuccess) return hip_fail(e, "swing launch");
  if (P0_host) {
    e = hipMemcpyAsync(P0_host, P, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "swing P0 copy");
  }
  return QTREE_OK;
}

qtree_status qtree_pi_quarter_disc(uint64_t seed, uint32_t rep0, int32_t reps, uint64_t npts,
                                   uint64_t* inside, void* stream) {
  if (!inside) return fail(QTREE_EINVAL, "inside is NULL");
  if (reps < 1 || reps > 65535) return fail(QTREE_EINVAL, "reps must be in 1..65535");
  if (npts == 0 || (npts & 1) || npts > (1ull << 33))
    return fail(QTREE_EINVAL, "npts must be even, in 2..2^33");
  const hipError_t e = qtree::launch_pi_quarter_disc(
      (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), rep0, reps, npts / 2,
      reinterpret_cast<unsigned long long*>(inside), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "pi launch");
}

qtree_status qtree_box_muller(const uint32_t* ra, const uint32_t* rb, int64_t count, float* z0,
                              float* z1, void* stream) {
  if (count < 0) return fail(QTREE_EINVAL, "count must be >= 0");
  if (count == 0) return QTREE_OK;
  if (!ra || !rb || !z0 || !z1) return fail(QTREE_EINVAL, "NULL array");
  hipError_t e = qtree::launch_box_muller(ra, rb, count, z0, z1, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "box_muller launch");
}

qtree_status qtree_layer_samples(const qtree_plan* plan, int32_t k, uint64_t m0, int64_t count,
                                 uint64_t seed, uint32_t contract_id, float* x, float* y,
                                 void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (k < 0 || k >= plan->n) return fail(QTREE_EINVAL, "layer index out of range");
  if (count < 0) return fail(QTREE_EINVAL, "count must be >= 0");
  if (m0 + (uint64_t)count > (1ull << 32)) return fail(QTREE_EOVERFLOW, "m0 + count > 2^32");
  if (count == 0) return QTREE_OK;
  if (!x || !y) return fail(QTREE_EINVAL, "NULL array");
  qtree::FwdArgs a = fwd_args(plan, m0, (uint64_t)count, seed, contract_id, nullptr);
  hipError_t e = qtree::launch_layer_samples(a, k, count, x, y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "layer_samples launch");
}

qtree_status qtree_cells(const qtree_plan* plan, int32_t k, const float* x, int64_t count,
                         int32_t* cell, void* stream) {
  if (!plan) return fail(QTREE_EINVAL, "plan is NULL");
  if (k < 0 || k > plan->n) return fail(QTREE_EINVAL, "layer index out of range");
  if (count < 0) return fail(QTREE_EINVAL, "count must be >= 0");
  if (count == 0) return QTREE_OK;
  if (!x || !cell) return fail(QTREE_EINVAL, "NULL array");
  qtree::FwdArgs a = fwd_args(plan, 0, 0, 0, 0, nullptr);
  hipError_t e = qtree::launch_cells(a, k, x, count, cell, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "cells launch");
}

}  // extern "C"
