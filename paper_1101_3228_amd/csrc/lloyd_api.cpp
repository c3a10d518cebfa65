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
  size_t recs, mids, cnt, sum, dist, part, total;
};

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
  l.dist = off;
  off = align_up(off + sizeof(unsigned long long), 256);
  l.part = off;
  off = align_up(off + sizeof(unsigned long long) * qtree::kLloydMaxBlocks *
                           ((size_t)N * d + (size_t)N + 1),
                 256);
  l.total = off;
  return l;
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
  for (int64_t i = 0; i < (int64_t)N * d; ++i) {
    if (!std::isfinite(grid0[i])) return set_error(QTREE_EINVAL, "non-finite start grid");
    if (std::fabs((double)grid0[i]) > kCoordMax)
      return set_error(QTREE_EOVERFLOW, "start grid coordinates must be within [-64, 64]");
  }
  if (d == 1)
    for (int32_t i = 0; i + 1 < N; ++i)
      if (!(grid0[i] < grid0[i + 1]))
        return set_error(QTREE_EINVAL, "1-D start grid must be strictly increasing");
  const size_t lds = qtree::lloyd_lds_bytes(d, N, l.Npad, l.P);
  if (lds > 160 * 1024) return set_error(QTREE_EUNSUPPORTED, "grid does not fit in LDS");

  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("device query: ") +
                                                           hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  qtree::LloydArgs a{};
  a.d = d;
  a.N = N;
  a.Npad = l.Npad;
  a.P = l.P;
  a.logP = l.logP;
  std::memcpy(a.L, L, sizeof(float) * d * d);
  a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(seed >> 32);
  a.M = M;
  a.grid = grid;
  a.recs = reinterpret_cast<float4*>(ws + l.recs);
  a.mids = reinterpret_cast<float*>(ws + l.mids);
  a.cnt = reinterpret_cast<unsigned int*>(ws + l.cnt);
  a.sum = reinterpret_cast<unsigned long long*>(ws + l.sum);
  a.dist = reinterpret_cast<unsigned long long*>(ws + l.dist);
  a.distortion = distortion;
  a.part = reinterpret_cast<unsigned long long*>(ws + l.part);
  a.E = N * d + N + 1;
  e = hipMemcpyAsync(grid, grid0, sizeof(float) * (size_t)N * d, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("start grid copy: ") +
                                                           hipGetErrorString(e));
  e = qtree::launch_lloyd_prepare(a, s);
  // two workgroups per CU (at most kLloydMaxBlocks), fewer when the samples
  // of a step are few
  const uint64_t per_block = 256ull * (d == 1 ? 1 : 8);  // samples per workgroup round
  const uint64_t want = (M + per_block - 1) / per_block;
  const uint64_t cap = std::min<uint64_t>(2ull * cus, qtree::kLloydMaxBlocks);
  const int blocks = (int)(want < cap ? want : cap);
  for (int32_t it = 0; it < steps && e == hipSuccess; ++it) {
    a.it = it;
    a.it_ctr = fresh ? (uint32_t)it : 0u;
    e = qtree::launch_lloyd_step(a, blocks, s);
  }
  if (e != hipSuccess) return set_error(QTREE_EDEVICE, std::string("lloyd launch: ") +
                                                           hipGetErrorString(e));
  return QTREE_OK;
}

}  // extern "C"
