// Stratified time-layer counts for d = 1 (not in the paper; a variance
// reduction of Algorithm III's estimate).  Layer k's samples of X_k are
// drawn cell by cell from the marginal N(mu_k, L_k^2) conditioned on the
// cell, by inversion of the normal distribution function between the cell's
// edge probabilities; X_{k+1} follows by the AR(1) step and its cell is
// searched as in the forward.  Row i gets M samples (equal allocation) or
// max(1, rint(M p_i)) (proportional allocation, p_i the cell's probability),
// so row i of counts[k] sums to its sample count by construction.
//
// Rows are taken kStratRows at a time (a tile); a tile with more than
// kStratSegment samples is shared by several workgroups (host-built work
// list).  A workgroup keeps its tile's counts in LDS (rows x N_{k+1} words,
// times S sub-counters taken by lane mod S: the samples of a wave share a row
// and mostly fall in a few cells, and same-word LDS atomics of one wave
// serialize) while its lanes walk the samples, then writes the rows with
// plain stores, zeros included, or, for a shared tile, adds its nonzero
// counts onto the zeroed rows with atomics.  No sort and no histogram pass.
// A banded output keeps of each row only the columns its samples can reach
// (a band the plan computes from the cell, the AR(1) step and the largest
// Box-Muller normal), packed row after row.
// X_{k+1}'s cell comes from the layer's guide table (cell_1d_guide) when the
// plan has tables, else from the breadth-first search.
//
// Sample t of row i of layer k, as in the arithmetic specification:
// Philox counter (t, k, contract, 4 + 256 i); u = (k52 + 1/2) 2^-52 with
// k52 = (r0 >> 12) 2^32 + r1; p = e_i + u (e_{i+1} - e_i), kept inside
// [2^-1074, 1 - 2^-53]; z = Phi^-1(p) by
// Wichura's algorithm AS 241 (FP64; ln by the atanh series); X_k =
// fma(L_k, (float)z, mu_k); eps = the first Box-Muller normal of (r2, r3);
// X_{k+1} = fma(T_k, eps, fma(A_k, X_k, b_k)).
#include "qtree_internal.hpp"
#include "qtree_rng.hpp"
#include "qtree_search.hpp"

namespace qtree {

namespace {

constexpr int kBlock = 256;

// ln x for finite x > 0: x = 2^e f, f in [1, 2) from the bits (subnormals
// scaled by 2^54), folded into [sqrt(1/2), sqrt(2)) by an exact halving;
// ln f = 2 s sum_{k=0..11} s^(2k) / (2k + 1), s = (f - 1) / (f + 1), by
// fused Horner steps in s^2; ln x = fma(e, ln 2, ln f).
__device__ __forceinline__ double ln64(double x) {
  uint64_t bits = (uint64_t)__double_as_longlong(x);
  int e = 0;
  if (((bits >> 52) & 0x7FF) == 0) {
    x = x * 0x1p54;
    bits = (uint64_t)__double_as_longlong(x);
    e = -54;
  }
  e += (int)((bits >> 52) & 0x7FF) - 1023;
  double f = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) |
                                              0x3FF0000000000000ull));
  if (f > 1.4142135623730951) {
    f = 0.5 * f;
    e += 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double P = 1.0 / 23.0;
#pragma unroll
  for (int k = 10; k >= 0; --k) P = fma(P, s2, 1.0 / (double)(2 * k + 1));
  return fma((double)e, 0.6931471805599453, (2.0 * s) * P);
}

// c[0] + c[1] r + ... + c[7] r^7, Horner with separate multiply and add.
__device__ __forceinline__ double poly7(const double (&c)[8], double r) {
  double v = c[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) v = v * r + c[k];
  return v;
}

// Standard normal quantile, Wichura (1988), algorithm AS 241 (PPND16).
__device__ __forceinline__ double normal_quantile(double p) {
  constexpr double A[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
                           1.9715909503065514427e+3, 1.3731693765509461125e+4,
                           4.5921953931549871457e+4, 6.7265770927008700853e+4,
                           3.3430575583588128105e+4, 2.5090809287301226727e+3};
  constexpr double B[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
                           5.3941960214247511077e+3, 2.1213794301586595867e+4,
                           3.9307895800092710610e+4, 2.8729085735721942674e+4,
                           5.2264952788528545610e+3};
  constexpr double C[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
                           5.76949722146069140550e0, 3.64784832476320460504e0,
                           1.27045825245236838258e0, 2.41780725177450611770e-1,
                           2.27238449892691845833e-2, 7.74545014278341407640e-4};
  constexpr double D[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
                           6.89767334985100004550e-1, 1.48103976427480074590e-1,
                           1.51986665636164571966e-2, 5.47593808499534494600e-4,
                           1.05075007164441684324e-9};
  constexpr double E[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
                           1.78482653991729133580e0, 2.96560571828504891230e-1,
                           2.65321895265761230930e-2, 1.24266094738807843860e-3,
                           2.71155556874348757815e-5, 2.01033439929228813265e-7};
  constexpr double F[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
                           1.48753612908506148525e-2, 7.86869131145613259100e-4,
                           1.84631831751005468180e-5, 1.42151175831644588870e-7,
                           2.04426310338993978564e-15};
  if (!(p > 0.0)) return -__builtin_huge_val();
  if (!(p < 1.0)) return __builtin_huge_val();
  const double q = p - 0.5;
  if (fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    return q * poly7(A, r) / poly7(B, r);
  }
  double r = q < 0.0 ? p : 1.0 - p;
  r = sqrt(-ln64(r));
  double x;
  if (r <= 5.0) {
    r = r - 1.6;
    x = poly7(C, r) / poly7(D, r);
  } else {
    r = r - 5.0;
    x = poly7(E, r) / poly7(F, r);
  }
  return q < 0.0 ? -x : x;
}

// Samples of row i (e: the layer's edge probabilities).
__device__ __forceinline__ uint64_t strat_row(const StratArgs& a, const double* e, int i) {
  if (a.alloc == 0) return a.M;
  const long long r = (long long)__builtin_rint((double)a.M * (e[i + 1] - e[i]));
  return r > 1 ? (uint64_t)r : 1ull;
}

// (X_k, X_{k+1}) of sample t of row i of layer k.
__device__ __forceinline__ void strat_pair(const StratArgs& a, const LayerDev& L, int k, int i,
                                           uint64_t t, float& x, float& y) {
  const U4 r = philox4x32_10(U4{(uint32_t)t, (uint32_t)k, a.contract, 4u + 256u * (uint32_t)i},
                             a.key0, a.key1);
  const double* e = a.edges + L.edge_off;
  const double k52 = (double)(r.x >> 12) * 4294967296.0 + (double)r.y;
  const double u = (k52 + 0.5) * 0x1p-52;
  const double step = u * (e[i + 1] - e[i]);
  double p = e[i] + step;
  // p rounds to 0 or 1 only in cells beyond ~8 standard deviations; the
  // nearest representable probabilities keep every sample finite
  if (!(p < 1.0)) p = 0x1.fffffffffffffp-1;
  if (!(p > 0.0)) p = 0x1p-1074;
  const double z = normal_quantile(p);
  float eps, unused;
  box_muller(r.z, r.w, eps, unused);
  x = fmaf(L.L[0], (float)z, L.mu[0]);
  y = fmaf(L.T[0], eps, fmaf(L.A[0], x, L.b[0]));
}

// Stores a tile's rows (cnt: [rows][N1][S] sub-counters in LDS): the whole
// rows with plain stores (zeros included), or, for a tile shared by several
// workgroups, its nonzero counts added onto the zeroed rows; with a banded
// output only the columns of each row's band, counting the rest in
// *overflow (no sample reaches them when the band is right).
template <int S>
__device__ __forceinline__ void store_tile(const StratArgs& a, const StratUnit& U,
                                           const LayerDev& L0, const uint32_t* cnt) {
  const int i0 = U.i0, N1 = L0.N1;
  const int rows = L0.N - i0 < kStratRows ? L0.N - i0 : kStratRows;
  if (a.band_off) {
    __shared__ int64_t boff[kStratRows];
    __shared__ int32_t blo[kStratRows], bw[kStratRows];
    if ((int)threadIdx.x < rows) {
      const int64_t r = (int64_t)L0.pt_off + i0 + threadIdx.x;
      boff[threadIdx.x] = a.band_off[r];
      bw[threadIdx.x] = (int32_t)(a.band_off[r + 1] - a.band_off[r]);
      blo[threadIdx.x] = a.band_lo[r];
    }
    __syncthreads();
    uint32_t lost = 0u;
    for (int i = threadIdx.x; i < rows * N1; i += kBlock) {
      uint32_t v = 0u;
#pragma unroll
      for (int q = 0; q < S; ++q) v += cnt[i * S + q];
      const int row = i / N1;
      const uint32_t w = (uint32_t)(i - row * N1 - blo[row]);
      if (w < (uint32_t)bw[row]) {
        int32_t* dst = a.counts + boff[row] + w;
        if (U.split) {
          if (v) atomicAdd(dst, (int32_t)v);
        } else {
          *dst = (int32_t)v;
        }
      } else {
        lost += v;
      }
    }
    if (lost) atomicAdd(a.overflow, lost);
    return;
  }
  int32_t* out = a.counts + L0.cnt_off + (int64_t)i0 * N1;
  for (int i = threadIdx.x; i < rows * N1; i += kBlock) {
    uint32_t v = 0u;
#pragma unroll
    for (int q = 0; q < S; ++q) v += cnt[i * S + q];
    if (U.split) {
      if (v) atomicAdd(&out[i], (int32_t)v);
    } else {
      out[i] = (int32_t)v;
    }
  }
}

}  // namespace

// Workgroup b takes unit b of the work list.
template <int LOGP>
__global__ __launch_bounds__(kBlock) void strat_kernel(StratArgs a, const StratUnit* units) {
  extern __shared__ float lds[];
  const StratUnit U = units[blockIdx.x];
  const int k = U.k;
  const LayerDev& L0 = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  const int i0 = U.i0;
  const int N1 = L0.N1;
  constexpr int P = 1 << LOGP;
  float* tree = lds;                                              // [P] breadth-first
  uint32_t* cnt = reinterpret_cast<uint32_t*>(lds + P);           // [kStratRows][N1]
  const float inf = __builtin_huge_valf();
  for (int i = threadIdx.x; i < P; i += kBlock) {
    const int src = i > 0 ? bfs_source<LOGP>(i) : 0;
    tree[i] = (i > 0 && src < L1.P) ? a.mids[L1.aux_off + src] : inf;
  }
  for (int i = threadIdx.x; i < kStratRows * N1; i += kBlock) cnt[i] = 0u;
  __syncthreads();

  // first sample of each of the rows in the workgroup's index space
  const double* e = a.edges + L0.edge_off;
  uint64_t pre[kStratRows + 1];
  pre[0] = 0;
#pragma unroll
  for (int r = 0; r < kStratRows; ++r)
    pre[r + 1] = pre[r] + (i0 + r < L0.N ? strat_row(a, e, i0 + r) : 0ull);
  for (uint64_t s = U.s0 + threadIdx.x; s < U.s1; s += kBlock) {
    int row = 0;
#pragma unroll
    for (int r = 1; r < kStratRows; ++r) row += s >= pre[r] ? 1 : 0;
    float x, y;
    strat_pair(a, L0, k, i0 + row, s - pre[row], x, y);
    const int j = cell_1d_bfs<LOGP>(tree, y);
    atomicAdd(&cnt[row * N1 + j], 1u);
  }
  __syncthreads();
  store_tile<1>(a, U, L0, cnt);
}

// The same with layer k+1's guide table: its sorted midpoints (+inf beyond
// its P, to maxP + kGuideKMax entries), its table, then the counts
// [kStratRows][N1][S].
// Launch bounds of four workgroups per CU hold the kernel to 128 VGPRs, four
// waves per SIMD, without spills (145 VGPRs, three waves, unbounded: 6 %
// slower).
template <int GK, int S>
__global__ __launch_bounds__(kBlock, 4) void strat_kernel_guide(StratArgs a,
                                                             const StratUnit* units) {
  extern __shared__ float lds[];
  const StratUnit U = units[blockIdx.x];
  const int k = U.k;
  const LayerDev& L0 = a.layers[k];
  const LayerDev& L1 = a.layers[k + 1];
  const int i0 = U.i0;
  const int N1 = L0.N1;
  const int PM = a.maxP + kGuideKMax;
  float* mk1 = lds;
  uint16_t* tk1 = reinterpret_cast<uint16_t*>(lds + PM);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(lds + PM + (a.gt_Bmax + 1) / 2);
  const float inf = __builtin_huge_valf();
  for (int i = threadIdx.x; i < PM; i += kBlock) mk1[i] = i < L1.P ? a.mids[L1.aux_off + i] : inf;
  for (int i = threadIdx.x; i < L1.gt_B; i += kBlock) tk1[i] = a.guide[L1.gt_off + i];
  for (int i = threadIdx.x; i < kStratRows * N1 * S; i += kBlock) cnt[i] = 0u;
  __syncthreads();
  const float s1 = L1.gt_scale, h1 = L1.gt_shift, bm1 = (float)(L1.gt_B - 1);
  const double* e = a.edges + L0.edge_off;
  uint64_t pre[kStratRows + 1];
  pre[0] = 0;
#pragma unroll
  for (int r = 0; r < kStratRows; ++r)
    pre[r + 1] = pre[r] + (i0 + r < L0.N ? strat_row(a, e, i0 + r) : 0ull);
  const uint32_t sub = threadIdx.x & (S - 1);
  for (uint64_t s = U.s0 + threadIdx.x; s < U.s1; s += kBlock) {
    int row = 0;
#pragma unroll
    for (int r = 1; r < kStratRows; ++r) row += s >= pre[r] ? 1 : 0;
    float x, y;
    strat_pair(a, L0, k, i0 + row, s - pre[row], x, y);
    const int j = cell_1d_guide<GK>(mk1, tk1, s1, h1, bm1, y);
    atomicAdd(&cnt[(uint32_t)(row * N1 + j) * S + sub], 1u);
  }
  __syncthreads();
  store_tile<S>(a, U, L0, cnt);
}

__global__ void strat_samples_kernel(StratArgs a, int k, int i, uint64_t t0, int64_t count,
                                     float* x, float* y) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= count) return;
  float xv, yv;
  strat_pair(a, a.layers[k], k, i, t0 + (uint64_t)t, xv, yv);
  x[t] = xv;
  y[t] = yv;
}

size_t strat_lds_bytes(int maxP, int maxN) {
  return sizeof(float) * (size_t)maxP + sizeof(uint32_t) * (size_t)kStratRows * (size_t)maxN;
}

namespace {
size_t strat_lds_guide(const StratArgs& a, int S) {
  return sizeof(float) * ((size_t)a.maxP + kGuideKMax + ((size_t)a.gt_Bmax + 1) / 2) +
         sizeof(uint32_t) * (size_t)kStratRows * (size_t)a.maxN * (size_t)S;
}

template <int GK, int S>
hipError_t launch_strat_guide(const StratArgs& a, const StratUnit* units, int n_units,
                              size_t lds, hipStream_t s) {
  hipError_t e = lds <= 65536 ? hipSuccess
                              : hipFuncSetAttribute(
                                    reinterpret_cast<const void*>(strat_kernel_guide<GK, S>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((strat_kernel_guide<GK, S>), dim3((unsigned)n_units), dim3(kBlock), lds, s,
                     a, units);
  return hipGetLastError();
}

template <int GK>
hipError_t launch_strat_guide_k(const StratArgs& a, const StratUnit* units, int n_units,
                                hipStream_t s) {
  // four sub-counters while the counts stay within 64 KiB (more would cost
  // occupancy), else one
  const size_t lds4 = strat_lds_guide(a, 4);
  if (lds4 <= 65536) return launch_strat_guide<GK, 4>(a, units, n_units, lds4, s);
  return launch_strat_guide<GK, 1>(a, units, n_units, strat_lds_guide(a, 1), s);
}
}  // namespace

hipError_t launch_strat(const StratArgs& a, const StratUnit* units, int n_units, hipStream_t s) {
  const dim3 grid((unsigned)n_units);
  if (a.gt_Kmax >= 0 && a.gt_Kmax <= kGuideKMax && strat_lds_guide(a, 1) <= 160 * 1024) {
    switch (a.gt_Kmax) {
      case 0:
      case 1: return launch_strat_guide_k<1>(a, units, n_units, s);
      case 2: return launch_strat_guide_k<2>(a, units, n_units, s);
      case 3: return launch_strat_guide_k<3>(a, units, n_units, s);
      default: return launch_strat_guide_k<4>(a, units, n_units, s);
    }
  }
  const size_t lds = strat_lds_bytes(a.maxP, a.maxN);
  hipError_t e = hipErrorInvalidValue;
  switch (a.maxP) {
#define QTREE_STRAT(LG)                                                                     \
  case 1 << LG:                                                                             \
    e = lds <= 65536 ? hipSuccess                                                           \
                     : hipFuncSetAttribute(reinterpret_cast<const void*>(strat_kernel<LG>), \
                                           hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                           (int)lds);                                       \
    if (e == hipSuccess)                                                                    \
      hipLaunchKernelGGL(strat_kernel<LG>, grid, dim3(kBlock), lds, s, a, units);             \
    break;
    QTREE_STRAT(1) QTREE_STRAT(2) QTREE_STRAT(3) QTREE_STRAT(4) QTREE_STRAT(5) QTREE_STRAT(6)
    QTREE_STRAT(7) QTREE_STRAT(8) QTREE_STRAT(9) QTREE_STRAT(10) QTREE_STRAT(11)
    QTREE_STRAT(12) QTREE_STRAT(13)
#undef QTREE_STRAT
    default:
      break;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_strat_samples(const StratArgs& a, int k, int i, uint64_t t0, int64_t count,
                                float* x, float* y, hipStream_t s) {
  const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(strat_samples_kernel, dim3(blocks), dim3(kBlock), 0, s, a, k, i, t0, count,
                     x, y);
  return hipGetLastError();
}

}  // namespace qtree
