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

template <int D>
__global__ void cells_kernel(FwdArgs a, int k, const float* x, int64_t count, int32_t* cell) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const LayerDev& L = a.layers[k];
  if (D == 1) {
    cell[i] = cell_1d(a.mids + L.aux_off, L.logP, x[i]);
  } else {
    float q[1][D];
#pragma unroll
    for (int c = 0; c < D; ++c) q[0][c] = x[i * D + c];
    int j;
    argmin_scan<D, 1>(a.pts + L.pt_off, L.N, q, &j);
    cell[i] = j;
  }
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
  const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
  if (a.d == 1)
    hipLaunchKernelGGL((cells_kernel<1>), dim3(blocks), dim3(kBlock), 0, s, a, k, x, count, cell);
  else if (a.d == 2)
    hipLaunchKernelGGL((cells_kernel<2>), dim3(blocks), dim3(kBlock), 0, s, a, k, x, count, cell);
  else
    hipLaunchKernelGGL((cells_kernel<3>), dim3(blocks), dim3(kBlock), 0, s, a, k, x, count, cell);
  return hipGetLastError();
}

}  // namespace qtree
