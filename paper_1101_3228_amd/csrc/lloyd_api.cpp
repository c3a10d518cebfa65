// C-ABI of the device grid optimizer (randomized Lloyd iteration for the
// quadratic quantization error, Sec. 2, eq. Qerr).  Contract in
// include/qtree.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "qtree.h"
#include "qtree_internal.hpp"
#include "qtree_plan.hpp"

using qtree::set_error;

namespace {

constexpr int kMaxN1 = 8192;   // d = 1
constexpr int kMaxNd = 2048;   // d = 2, 3
// |z| <= sqrt(-2 ln 2^-24) < 5.77 for the Box-Muller normals, so a sample
// coordinate is at most 5.77 x the absolute row sum of L.  Coordinates and
// start points up to 64 keep the integer cell sums (M < 2^31 samples of
// 64 x 2^24) and the squared distances (3 (64 + 64)^2 2^16 each) below 2^63.
constexpr double kZMax = 5.77;
constexpr double kCoordMax = 64.0;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct LloydLayout {
  int Npad, P, logP;
  size_t recs, mids, cnt, sum, acc, part, total;
};
constexpr int kExtra = 3;  // partial-table words per row beyond sums and counts

LloydLayout layout(int d, int N) {
  LloydLayout l{};
  l.Npad = (N + qtree::kScanTile - 1) / qtree::kScanTile * qtree::kScanTile;
  l.P = 1;
  l.logP = 0;
  while (l.P < N) {
    l.P <<= 1;
    ++l.logP;
  }
  size_t off = 0;
  l.recs = off;
  off = align_up(off + (d == 1 ? 0 : sizeof(float4) * (size_t)l.Npad), 256);
  l.mids = off;
  off = align_up(off + (d == 1 ? sizeof(float) * (size_t)l.P : 0), 256);
  l.cnt = off;
  off = align_up(off + sizeof(unsigned int) * (size_t)N, 256);
  l.sum = off;
  off = align_up(off + sizeof(unsigned long long) * (size_t)N * d, 256);
  l.acc = off;  // distortion, admissible, inadmissible, running inadmissible total
  off = align_up(off + 4 * sizeof(unsigned long long), 256);
  l.part = off;
  off = align_up(off + sizeof(unsigned long long) * qtree::kLloydMaxBlocks *
                           ((size_t)N * d + (size_t)N + kExtra),
                 256);
  l.total = off;
  return l;
}

// Device arguments of a step over workspace `ws` laid out by `l`.
qtree::LloydArgs args_of(int d, int N, const LloydLayout& l, float* grid, void* workspace) {
  char* ws = static_cast<char*>(workspace);
  qtree::LloydArgs a{};
  a.d = d;
  a.N = N;
  a.Npad = l.Npad;
  a.P = l.P;
  a.logP = l.logP;
  a.grid = grid;
  a.recs = reinterpret_cast<float4*>(ws + l.recs);
  a.mids = reinterpret_cast<float*>(ws + l.mids);
  a.cnt = reinterpret_cast<unsigned int*>(ws + l.cnt);
  a.sum = reinterpret_cast<unsigned long long*>(ws + l.sum);
  auto* acc = reinterpret_cast<unsigned long long*>(ws + l.acc);
  a.dist = acc;
  a.used = acc + 1;
  a.rej = acc + 2;
  a.rej_total = acc + 3;
  a.part = reinterpret_cast<unsigned long long*>(ws + l.part);
  a.E = N * d + N + kExtra;
  a.gamma = 1.0;
  return a;
}

// Two accumulation workgroups per CU (at most kLloydMaxBlocks), fewer when
// the samples of a step are few.
int accum_blocks(int d, uint64_t M, int cus) {
  const uint64_t per_block = 256ull * (d == 1 ? 1 : 8);  // samples per workgroup round
  const uint64_t want = (M + per_block - 1) / per_block;
  const uint64_t cap = std::min<uint64_t>(2ull * (uint64_t)cus, qtree::kLloydMaxBlocks);
  return (int)std::max<uint64_t>(1, want < cap ? want : cap);
}

qtree_status device_cus(int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess)
    return set_error(QTREE_EDEVICE, std::string("device query: ") + hipGetErrorString(e));
  return QTREE_OK;
}

qtree_status check_grid0(int32_t d, int32_t N, const float* grid0) {
  for (int64_t i = 0; i < (int64_t)N * d; ++i) {
    if (!std::isfinite(grid0[i])) return set_error(QTREE_EINVAL, "non-finite start grid");
    if (std::fabs((double)grid0[i]) > kCoordMax)
      return set_error(QTREE_EOVERFLOW, "start grid coordinates must be within [-64, 64]");
  }
  if (d == 1)
    for (int32_t i = 0; i + 1 < N; ++i)
      if (!(grid0[i] < grid0[i + 1]))
        return set_error(QTREE_EINVAL, "1-D start grid must be strictly increasing");
  return QTREE_OK;
}

qtree_status check_shape(int32_t d, int32_t N) {
  if (d < 1 || d > 3) return set_error(QTREE_EINVAL, "d must be 1, 2 or 3");
  if (N < 1) return set_error(QTREE_EINVAL, "N must be >= 1");
  if (N > (d == 1 ? kMaxN1 : kMaxNd))
    return set_error(QTREE_EUNSUPPORTED, "N above the grid optimizer's limit (8192 for d = 1, "
                                         "2048 for d = 2, 3)");
  return QTREE_OK;
}

}  // namespace

extern "C" {

size_t qtree_lloyd_workspace_size(int32_t d, int32_t N) {
  if (check_shape(d, N) != QTREE_OK) return 0;
  return layout(d, N).total;
}

qtree_status qtree_lloyd(int32_t d, int32_t N, const float* L, const float* grid0, float* grid,
                         uint64_t M, int32_t steps, uint64_t seed, int32_t fresh,
                         double* distortion, void* workspace, size_t workspace_bytes,
                         void* stream) {
  qtree_status st = check_shape(d, N);
  if (st != QTREE_OK) return st;
  if (!L || !grid0 || !grid || !workspace) return set_error(QTREE_EINVAL, "NULL argument");
  if (M < 1 || M >= (1ull << 31)) return set_error(QTREE_EOVERFLOW, "M must be in 1 .. 2^31 - 1");
  if (steps < 1) return set_error(QTREE_EINVAL, "steps must be >= 1");
  const LloydLayout l = layout(d, N);
  if (workspace_bytes < l.total) return set_error(QTREE_ENOMEM, "workspace too small");
  for (int r = 0; r < d; ++r) {
    double row = 0.0;
    for (int c = 0; c < d; ++c) {
      if (!std::isfinite(L[r * d + c])) return set_error(QTREE_EINVAL, "non-finite L");
      row += std::fabs((double)L[r * d + c]);
    }
    if (kZMax * row > kCoordMax)
      return set_error(QTREE_EOVERFLOW, "L too large: sample coordinates may exceed 64");
  }
  if ((st = check_grid0(d, N, grid0)) != QTREE_OK) return st;
  const size_t lds = qtree::lloyd_lds_bytes(d, N, l.Npad, l.P);
  if (lds > 160 * 1024) return set_error(QTREE_EUNSUPPORTED, "grid does not fit in LDS");

  int cus = 0;
  if ((st = device_cus(&cus)) != QTREE_OK) return st;
  hipError_t e;
  hipStream_t s = static_cast<hipStream_t>(stream);
  qtree::LloydArgs a = args_of(d, N, l, grid, workspace);
  std::memcpy(a.L, L, sizeof(float) * d * d);
  a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(seed >> 32);
  a.M = M;
  a.distortion = distortion;
  e = hipMemcpyAsync(grid, grid0, sizeof(float) * (size_t)N * d, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("start grid copy: ") +
                                                           hipGetErrorString(e));
  e = qtree::launch_lloyd_prepare(a, s);
  // two workgroups per CU (at most kLloydMaxBlocks), fewer when the samples
  // of a step are few
  const int blocks = accum_blocks(d, M, cus);
  for (int32_t it = 0; it < steps && e == hipSuccess; ++it) {
    a.it = it;
    a.it_ctr = fresh ? (uint32_t)it : 0u;
    e = qtree::launch_lloyd_step(a, blocks, s);
  }
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("lloyd launch: ") +
                                                           hipGetErrorString(e));
  return QTREE_OK;
}

qtree_status qtree_lloyd_samples(int32_t d, int32_t N, const float* grid0, float* grid,
                                 const float* x, uint64_t M, uint64_t batch, int32_t steps,
                                 double gamma, double* distortion, int64_t* rejected,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  qtree_status st = check_shape(d, N);
  if (st != QTREE_OK) return st;
  if (!grid0 || !grid || !x || !workspace) return set_error(QTREE_EINVAL, "NULL argument");
  if (M < 1) return set_error(QTREE_EINVAL, "the sample set is empty");
  if (M > (1ull << 40)) return set_error(QTREE_EOVERFLOW, "at most 2^40 samples in the set");
  if (batch < 1 || batch >= (1ull << 31))
    return set_error(QTREE_EOVERFLOW, "batch must be in 1 .. 2^31 - 1");
  if (steps < 1) return set_error(QTREE_EINVAL, "steps must be >= 1");
  if (!(gamma > 0.0 && gamma <= 1.0)) return set_error(QTREE_EINVAL, "gamma must be in (0, 1]");
  const LloydLayout l = layout(d, N);
  if (workspace_bytes < l.total) return set_error(QTREE_ENOMEM, "workspace too small");
  if ((st = check_grid0(d, N, grid0)) != QTREE_OK) return st;
  const size_t lds = qtree::lloyd_lds_bytes(d, N, l.Npad, l.P);
  if (lds > 160 * 1024) return set_error(QTREE_EUNSUPPORTED, "grid does not fit in LDS");
  int cus = 0;
  if ((st = device_cus(&cus)) != QTREE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  qtree::LloydArgs a = args_of(d, N, l, grid, workspace);
  a.xs = x;
  a.Ms = M;
  a.M = batch;
  a.gamma = gamma;
  a.distortion = distortion;
  a.rejected = reinterpret_cast<long long*>(rejected);
  hipError_t e =
      hipMemcpyAsync(grid, grid0, sizeof(float) * (size_t)N * d, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("start grid copy: ") +
                                                           hipGetErrorString(e));
  e = qtree::launch_lloyd_prepare(a, s);
  const int blocks = accum_blocks(d, batch, cus);
  for (int32_t it = 0; it < steps && e == hipSuccess; ++it) {
    a.it = it;
    a.start = ((uint64_t)it * batch) % M;  // t batch < 2^62
    e = qtree::launch_lloyd_step(a, blocks, s);
  }
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("lloyd launch: ") +
                                                           hipGetErrorString(e));
  return QTREE_OK;
}

qtree_status qtree_sample_moments(int32_t d, const float* x, uint64_t M, int64_t* sums,
                                  void* stream) {
  if (d < 1 || d > 3) return set_error(QTREE_EINVAL, "d must be 1, 2 or 3");
  if (!sums || (M > 0 && !x)) return set_error(QTREE_EINVAL, "NULL argument");
  if (M > (1ull << 31)) return set_error(QTREE_EOVERFLOW, "at most 2^31 samples");
  if (reinterpret_cast<uintptr_t>(sums) % 8) return set_error(QTREE_EINVAL, "sums must be 8-byte aligned");
  const hipError_t e = qtree::launch_sample_moments(d, x, M, reinterpret_cast<long long*>(sums),
                                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return set_error(QTREE_EDEVICE, std::string("moments launch: ") + hipGetErrorString(e));
  return QTREE_OK;
}

qtree_status qtree_moment_grid(int32_t d, const int64_t* sums, const float* base, int32_t N,
                               float* grid, double* moments, void* stream) {
  if (d < 1 || d > 3) return set_error(QTREE_EINVAL, "d must be 1, 2 or 3");
  if (N < 1) return set_error(QTREE_EINVAL, "N must be >= 1");
  if (!sums || !base || !grid) return set_error(QTREE_EINVAL, "NULL argument");
  const hipError_t e =
      qtree::launch_moment_grid(d, reinterpret_cast<const long long*>(sums), base, N, grid,
                                moments, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return set_error(QTREE_EDEVICE, std::string("moment grid launch: ") + hipGetErrorString(e));
  return QTREE_OK;
}

}  // extern "C"
