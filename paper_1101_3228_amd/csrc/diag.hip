// Per-sample diagnostic kernels.  They call the very device functions the
// forward kernels use (Philox, Box-Muller, the AR(1) sample, the cell
// searches), so the tests can compare each intermediate result with the
// oracle instead of only the aggregated counts.
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"
#include "qtree_search.hpp"

namespace qtree {

namespace {
constexpr int kBlock = 256;
}

__global__ void box_muller_kernel(const uint32_t* ra, const uint32_t* rb, int64_t count,
                                  float* z0, float* z1) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  float a, b;
  box_muller(ra[i], rb[i], a, b);
  z0[i] = a;
  z1[i] = b;
}

template <int D>
__global__ void layer_samples_kernel(FwdArgs a, int k, int64_t count, float* x, float* y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const uint64_t m = a.m0 + (uint64_t)i;
  float z[D], e[D], xs[D], ys[D];
  layer_normals<D>(a.key0, a.key1, a.contract, k, m, z, e);
  layer_pair<D>(a.layers[k], z, e, xs, ys);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x[i * D + c] = xs[c];
    y[i * D + c] = ys[c];
  }
}

// d = 1: the binary search over the layer's sorted midpoints (the cell the
// forward's guide or breadth-first search returns).
__global__ void cells_1d_kernel(FwdArgs a, int k, const float* x, int64_t count, int32_t* cell) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const LayerDev& L = a.layers[k];
  cell[i] = cell_1d(a.mids + L.aux_off, L.logP, x[i]);
}

// d >= 2: the forward's scan.  The layer's records staged in LDS, padded to
// whole kScanTile-record tiles with records whose key is +inf; kCellsS points
// per lane share every record read (argmin_scan_tiled, tiles of kScanTile).
constexpr int kCellsS = 8;
// With bucket tables (d = 2, BK): each point's bucket list, as the
// forward's bucketed search.
template <int D, bool BK = false>
__global__ __launch_bounds__(kBlock) void cells_kernel(FwdArgs a, int k, const float* x,
                                                       int64_t count, int32_t* cell) {
  extern __shared__ float4 recs[];
  const LayerDev& L = a.layers[k];
  const int N = L.N;
  const int Npad = (N + kScanTile - 1) / kScanTile * kScanTile;
  float2* xy = reinterpret_cast<float2*>(recs);  // the bucketed search's (x, y) pairs
  if constexpr (BK && D == 2) {
    for (int r = threadIdx.x; r <= N; r += kBlock) {  // and the pad pair at N
      const float4 g = r < N ? a.pts[L.pt_off + r] : make_float4(0.f, 0.f, 0.f, 0.f);
      xy[r] = r < N ? make_float2(g.x, g.y) : make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
  } else {
    const float4 pad = make_float4(0.f, 0.f, 0.f, __builtin_huge_valf());
    for (int r = threadIdx.x; r < Npad; r += kBlock) recs[r] = r < N ? a.pts[L.pt_off + r] : pad;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBlock * kCellsS + threadIdx.x;
  float q[kCellsS][D];
  int idx[kCellsS];
#pragma unroll
  for (int s = 0; s < kCellsS; ++s) {
    const int64_t i = base + (int64_t)s * kBlock;
    const int64_t ii = i < count ? i : count - 1;  // the tail repeats the last point
#pragma unroll
    for (int c = 0; c < D; ++c) q[s][c] = x[ii * D + c];
  }
  if constexpr (BK && D == 2) {
    int slot[kCellsS];
    uint4 w[kCellsS];
    bucket_rows<kCellsS>(L, a.bk_rows, q, slot, w);
    bucket_argmin<kCellsS>(xy, N, a.bk_rows, q, slot, w, idx);
  } else {
    argmin_scan_tiled<D, kCellsS, kScanTile>(recs, Npad, q, idx);
  }
#pragma unroll
  for (int s = 0; s < kCellsS; ++s) {
    const int64_t i = base + (int64_t)s * kBlock;
    if (i < count) cell[i] = idx[s];
  }
}

// Quarter-disc experiment of the generator comparison (Sec. 3, Table rngs):
// point h of Philox block i of repetition rep (counter (i, rep, 0, 3)) is
// (U, V) = (r_{2h} >> 8, r_{2h+1} >> 8) 2^-24, inside when U^2 + V^2 <= 2^48
// (integers, exact).  Blocks of a repetition are dealt over the grid's x
// dimension; every workgroup adds its count to inside[rep] once.
__global__ __launch_bounds__(kBlock) void pi_quarter_disc_kernel(uint32_t key0, uint32_t key1,
                                                                 uint32_t rep0, uint64_t blocks,
                                                                 unsigned long long* inside) {
  __shared__ unsigned long long part[kBlock / 64];
  const uint32_t rep = rep0 + blockIdx.y;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint64_t n = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < blocks; i += stride) {
    const U4 r = philox4x32_10(U4{(uint32_t)i, rep, 0u, 3u}, key0, key1);
    const uint64_t u0 = r.x >> 8, v0 = r.y >> 8, u1 = r.z >> 8, v1 = r.w >> 8;
    n += (u0 * u0 + v0 * v0 <= (1ull << 48)) ? 1u : 0u;
    n += (u1 * u1 + v1 * v1 <= (1ull << 48)) ? 1u : 0u;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += part[w];
    atomicAdd(&inside[blockIdx.y], t);
  }
}

hipError_t launch_pi_quarter_disc(uint32_t key0, uint32_t key1, uint32_t rep0, int reps,
                                  uint64_t blocks, unsigned long long* inside, hipStream_t s) {
  const uint64_t want = (blocks + kBlock - 1) / kBlock;
  const unsigned gx = (unsigned)(want < 2048 ? (want < 1 ? 1 : want) : 2048);
  hipLaunchKernelGGL(pi_quarter_disc_kernel, dim3(gx, (unsigned)reps), dim3(kBlock), 0, s, key0,
                     key1, rep0, blocks, inside);
  return hipGetLastError();
}

hipError_t launch_box_muller(const uint32_t* ra, const uint32_t* rb, int64_t count, float* z0,
                             float* z1, hipStream_t s) {
  const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(box_muller_kernel, dim3(blocks), dim3(kBlock), 0, s, ra, rb, count, z0, z1);
  return hipGetLastError();
}

hipError_t launch_layer_samples(const FwdArgs& a, int k, int64_t count, float* x, float* y,
                                hipStream_t s) {
  const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
  if (a.d == 1)
    hipLaunchKernelGGL((layer_samples_kernel<1>), dim3(blocks), dim3(kBlock), 0, s, a, k, count, x, y);
  else if (a.d == 2)
    hipLaunchKernelGGL((layer_samples_kernel<2>), dim3(blocks), dim3(kBlock), 0, s, a, k, count, x, y);
  else
    hipLaunchKernelGGL((layer_samples_kernel<3>), dim3(blocks), dim3(kBlock), 0, s, a, k, count, x, y);
  return hipGetLastError();
}

hipError_t launch_cells(const FwdArgs& a, int k, const float* x, int64_t count, int32_t* cell,
                        hipStream_t s) {
  if (a.d == 1) {
    const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(cells_1d_kernel, dim3(blocks), dim3(kBlock), 0, s, a, k, x, count, cell);
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)((count + kBlock * kCellsS - 1) / (kBlock * kCellsS));
  const size_t lds = sizeof(float4) * (size_t)((a.maxN + kScanTile - 1) / kScanTile * kScanTile);
  const bool bk = a.d == 2 && a.bucketed;
  const void* fn = bk ? reinterpret_cast<const void*>(cells_kernel<2, true>)
                 : a.d == 2 ? reinterpret_cast<const void*>(cells_kernel<2>)
                            : reinterpret_cast<const void*>(cells_kernel<3>);
  hipError_t e = lds <= 65536 ? hipSuccess
                              : hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    (int)lds);
  if (e != hipSuccess) return e;
  if (bk)
    hipLaunchKernelGGL((cells_kernel<2, true>), dim3(blocks), dim3(kBlock), lds, s, a, k, x, count,
                       cell);
  else if (a.d == 2)
    hipLaunchKernelGGL((cells_kernel<2>), dim3(blocks), dim3(kBlock), lds, s, a, k, x, count, cell);
  else
    hipLaunchKernelGGL((cells_kernel<3>), dim3(blocks), dim3(kBlock), lds, s, a, k, x, count, cell);
  return hipGetLastError();
}

}  // namespace qtree
