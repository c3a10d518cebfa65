// Pricing-surrogate kernels for gfx950: fused forward (inference and
// training), fused back-propagation of the activation gradients, the weight
// gradients of the two 256x256 layers as an MFMA reduction over the batch,
// the remaining sums, and Adam with the refresh of the BF16 weight copies.
//
// MFMA mapping.  A wave owns 32 samples.  A 256x256 layer is computed as
// Z^T = W H^T with the weights as the A operand (rows = output units) and
// the activations as the B operand (columns = samples), 8 output blocks x
// 16 K-steps of v_mfma_f32_32x32x16_bf16.  Lane l holds accumulator r of
// output block jb for unit 32 jb + 8 (r / 4) + 4 (l / 32) + r % 4 and sample
// l % 32.  The K order inside a dot product is free, so K-step t is defined
// to take, for lane half h and element e, the unit
//     unit(t, h, e) = 32 (t / 2) + 16 (t % 2) + 8 (e / 4) + 4 h + e % 4,
// which is exactly accumulator r = 8 (t % 2) + e of block t / 2 of the lane:
// a layer's output, once activated, is the next layer's B operand without
// leaving the registers.  The weights are stored pre-permuted to match
// (fragment (ib, t) of lane l = W[32 ib + l % 32][unit(t, l / 32, e)],
// e = 0..7, 16 contiguous bytes per lane).
//
// Layer 1 (6 inputs) is one K-step per output block as well: the 16 K-slots
// hold the normalised inputs as two BF16 terms, (u_hi[0..5], u_lo[0..5], 0 x4)
// for lane halves h = 0 (slots 0..7) and h = 1 (slots 8..15), against
// (W1[i][0..5], W1[i][0..5], 0 x4); the accumulators start from the biases.
#include <hip/hip_runtime.h>

#include "qtree_mlp_internal.hpp"

namespace qtree {
namespace mlp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

__device__ __forceinline__ float dsilu(float z) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  return s * fmaf(z, 1.0f - s, 1.0f);
}

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float bf16_float(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// Position of W1[i][c] in the layer-1 fragments: K-slot c (hi term) and
// K-slot 6 + c (lo term); slot s lives in lane half s / 8, element s % 8.
__host__ __device__ __forceinline__ int frag1_index(int i, int slot) {
  return (((i >> 5) * 64) + 32 * (slot >> 3) + (i & 31)) * 8 + (slot & 7);
}

// Index of W[i][k] in the fragment layout described at the top.
__host__ __device__ __forceinline__ int frag_index(int i, int k) {
  const int t = 2 * (k >> 5) + ((k >> 4) & 1);
  const int rem = k & 15;
  const int e = 4 * (rem >> 3) + (rem & 3);
  const int lane = 32 * ((rem >> 2) & 1) + (i & 31);
  return (((i >> 5) * 16 + t) * 64 + lane) * 8 + e;
}

// The 16 accumulators of output block jb (already activated) as the B
// operands of K-steps 2 jb and 2 jb + 1, in TERMS BF16 parts.
template <int TERMS>
__device__ __forceinline__ void to_operand(const float (&v)[16], bf16x8 (&op)[TERMS][16],
                                           int jb) {
  bf16x8 a0, a1, b0, b1;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 p = (__bf16)v[e];
    const __bf16 q = (__bf16)v[8 + e];
    a0[e] = p;
    a1[e] = q;
    if (TERMS == 2) {
      b0[e] = (__bf16)(v[e] - (float)p);
      b1[e] = (__bf16)(v[8 + e] - (float)q);
    }
  }
  op[0][2 * jb] = a0;
  op[0][2 * jb + 1] = a1;
  if (TERMS == 2) {
    op[TERMS - 1][2 * jb] = b0;
    op[TERMS - 1][2 * jb + 1] = b1;
  }
}

__device__ __forceinline__ int unit_of(int jb, int r, int h) {
  return 32 * jb + 8 * (r >> 2) + 4 * h + (r & 3);
}

// acc[ib] = bias + sum over the 16 K-steps of fragment(ib, t) x op[.][t]
// (bias: per-unit LDS array, or NULL for zero).
template <int TERMS>
__device__ __forceinline__ void mfma_layer(const uint16_t* __restrict__ frags,
                                           const bf16x8 (&op)[TERMS][16], int lane,
                                           const float* bias, f32x16 (&acc)[8]) {
  const bf16x8* wf = reinterpret_cast<const bf16x8*>(frags);
  const int h = lane >> 5;
#pragma unroll
  for (int ib = 0; ib < 8; ++ib) {
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[ib][r] = bias ? bias[unit_of(ib, r, h)] : 0.0f;
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
#pragma unroll
    for (int ib = 0; ib < 8; ++ib) {
      const bf16x8 a = wf[(ib * 16 + t) * 64 + lane];
      acc[ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, op[0][t], acc[ib], 0, 0, 0);
      if (TERMS == 2)
        acc[ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, op[TERMS - 1][t], acc[ib], 0, 0, 0);
    }
  }
}

// Offset of accumulator r of block jb of a lane inside its wave's tile of a
// per-unit training array (the wave's base is wave * 8192).
__device__ __forceinline__ int tile_off(int jb, int r) { return (jb * 16 + r) * 64; }
constexpr int kWaveTile = 8 * 16 * 64;

// Tile-layout offset of (unit, sample s) (for kernels that walk units).
__device__ __forceinline__ int64_t tile_index(int unit, int64_t s) {
  const int u = unit & 31;
  const int r = 4 * (u >> 3) + (u & 3);
  const int h = (u >> 2) & 1;
  return (s >> 5) * kWaveTile + ((unit >> 5) * 16 + r) * 64 + 32 * h + (s & 31);
}

// Black-Scholes European put per unit strike on (S0/K, sigma, r, T).
__device__ __forceinline__ float bs_put(float s, float sig, float r, float T) {
  const float v = sig * sqrtf(T);
  const float d1 = (logf(s) + (r + 0.5f * sig * sig) * T) / v;
  const float d2 = d1 - v;
  return expf(-r * T) * 0.5f * erfcf(d2 * 0.70710678f) - s * 0.5f * erfcf(d1 * 0.70710678f);
}

struct FwdIO {
  const float* x;
  int64_t B;
  float* y;
  uint8_t* in_range;
};

// Forward pass of 32 samples per wave.  TRAIN: rows come from the training
// set through idx, pre-activations and layer inputs are kept for the
// backward pass, and the loss gradient dL/dy replaces y.
template <int TERMS, bool TRAIN>
__global__ __launch_bounds__(kBlock) void mlp_forward(Weights W, FwdIO io, Train T) {
  __shared__ float sb[3][kHid];
  __shared__ float sw4[kHid];
  for (int i = threadIdx.x; i < kHid; i += kBlock) {
    sb[0][i] = W.master[kOffB1 + i];
    sb[1][i] = W.master[kOffB2 + i];
    sb[2][i] = W.master[kOffB3 + i];
    sw4[i] = bf16_float(W.w4[i]);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t s = wave * kWaveRows + (lane & 31);
  const int64_t B = TRAIN ? T.B : io.B;
  const bool live = s < B;
  const int64_t tb = wave * kWaveTile + lane;  // this lane's place in a training tile

  int64_t row = s;
  if (TRAIN && live && T.idx) row = T.idx[s];
  const float* xs = TRAIN ? T.x : io.x;
  float u[kIn], raw[4];
  bool inside = true;
#pragma unroll
  for (int c = 0; c < kIn; ++c) {
    const float xv = live ? xs[row * kIn + c] : W.lo[c];
    if (c < 4) raw[c] = xv;
    inside = inside && xv >= W.lo[c] && xv <= W.hi[c];
    u[c] = live ? fmaf(xv - W.lo[c], W.scale[c], W.shift[c]) : 0.0f;
  }
  if (TRAIN && h == 0) {
#pragma unroll
    for (int c = 0; c < kIn; ++c) T.u[s * 8 + c] = u[c];
  }

  bf16x8 op[TERMS][16];
  f32x16 acc[8];
  {
    // layer 1 (MFMA): z1 = b1 + W1 (u_hi + u_lo), one K-step per block
    float q[16];
#pragma unroll
    for (int c = 0; c < kIn; ++c) {
      const __bf16 a = (__bf16)u[c];
      q[c] = (float)a;
      q[kIn + c] = (float)(__bf16)(u[c] - (float)a);
    }
#pragma unroll
    for (int c = 2 * kIn; c < 16; ++c) q[c] = 0.0f;
    bf16x8 ub;
#pragma unroll
    for (int e = 0; e < 8; ++e) ub[e] = (__bf16)(h ? q[8 + e] : q[e]);
    const bf16x8* w1f = reinterpret_cast<const bf16x8*>(W.w1);
#pragma unroll
    for (int ib = 0; ib < 8; ++ib) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[ib][r] = sb[0][unit_of(ib, r, h)];
      acc[ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1f[ib * 64 + lane], ub, acc[ib], 0, 0, 0);
    }
  }
#pragma unroll
  for (int jb = 0; jb < 8; ++jb) {
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float z = acc[jb][r];
      v[r] = silu(z);
      if (TRAIN) {
        T.z1[tb + tile_off(jb, r)] = z;
        T.h1[tb + tile_off(jb, r)] = bf16_bits(v[r]);
      }
    }
    to_operand<TERMS>(v, op, jb);
  }
  // layer 2 (MFMA)
  mfma_layer<TERMS>(W.w2f, op, lane, nullptr, acc);
#pragma unroll
  for (int jb = 0; jb < 8; ++jb) {
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float z = acc[jb][r] + sb[1][unit_of(jb, r, h)];
      v[r] = silu(z);
      if (TRAIN) {
        T.z2[tb + tile_off(jb, r)] = z;
        T.h2[tb + tile_off(jb, r)] = bf16_bits(v[r]);
      }
    }
    to_operand<TERMS>(v, op, jb);
  }
  // layer 3 (MFMA) and the head
  mfma_layer<TERMS>(W.w3f, op, lane, nullptr, acc);
  float part = 0.0f;
#pragma unroll
  for (int jb = 0; jb < 8; ++jb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int unit = unit_of(jb, r, h);
      const float z = acc[jb][r] + sb[2][unit];
      if (TRAIN) T.z3[tb + tile_off(jb, r)] = z;
      part = fmaf(sw4[unit], silu(z), part);
    }
  }
  part += __shfl_xor(part, 32);
  float y = W.out_scale * (part + W.master[kOffB4]);
  if (W.baseline && live && inside) y += bs_put(raw[0], raw[1], raw[2], raw[3]);

  if (!TRAIN) {
    if (h == 0 && live) {
      io.y[s] = y;
      if (io.in_range) io.in_range[s] = inside ? 1 : 0;
    }
    return;
  }
  float lc = 0.0f;
  if (h == 0) {
    float g = 0.0f;
    if (live) {
      const float wv = T.w ? T.w[row] : 1.0f;
      const float res = y - T.t[row];
      g = 2.0f * wv * res * T.inv_b;
      lc = wv * res * res * T.inv_b;
    }
    T.dy[s] = g;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) lc += __shfl_xor(lc, m);
  if (lane == 0) T.lossp[wave] = lc;
}

// Back-propagation of dL/dy to dz3, dz2, dz1 for 32 samples per wave, the
// transposed weights as the A operand (same register layout as forward).
__global__ __launch_bounds__(kBlock) void mlp_backward(Weights W, Train T) {
  __shared__ float sw4[kHid];
  for (int i = threadIdx.x; i < kHid; i += kBlock) sw4[i] = bf16_float(W.w4[i]);
  __syncthreads();
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t s = wave * kWaveRows + (lane & 31);
  const int64_t tb = wave * kWaveTile + lane;
  const float gy = W.out_scale * T.dy[s];

  bf16x8 op[1][16];
  f32x16 acc[8];
#pragma unroll
  for (int jb = 0; jb < 8; ++jb) {
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int unit = unit_of(jb, r, h);
      const float dz = sw4[unit] * gy * dsilu(T.z3[tb + tile_off(jb, r)]);
      T.dz3[tb + tile_off(jb, r)] = dz;
      v[r] = dz;
    }
    to_operand<1>(v, op, jb);
  }
  mfma_layer<1>(W.w3t, op, lane, nullptr, acc);  // dh2 = W3^T dz3
#pragma unroll
  for (int jb = 0; jb < 8; ++jb) {
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float dz = acc[jb][r] * dsilu(T.z2[tb + tile_off(jb, r)]);
      T.dz2[tb + tile_off(jb, r)] = dz;
      v[r] = dz;
    }
    to_operand<1>(v, op, jb);
  }
  mfma_layer<1>(W.w2t, op, lane, nullptr, acc);  // dh1 = W2^T dz2
#pragma unroll
  for (int jb = 0; jb < 8; ++jb) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
      T.dz1[tb + tile_off(jb, r)] = acc[jb][r] * dsilu(T.z1[tb + tile_off(jb, r)]);
  }
}

// Partial weight gradients dW[i][k] = sum_s dz[i][s] h[k][s] of layers 2
// and 3 over one chunk of kChunk samples: one 32x32 tile per wave, the
// samples as the K dimension.
__global__ __launch_bounds__(kBlock) void mlp_wgrad(Train T) {
  const int nchunks = (int)(T.Bp / kChunk);
  const int job = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int q = job % nchunks;
  const int tile = (job / nchunks) & 63;
  const int L = job / (nchunks * 64);
  if (L >= 2) return;
  const int ib = tile >> 3, kb = tile & 7;
  const int lane = threadIdx.x & 63, h = lane >> 5, row = lane & 31;
  const float* dz = L ? T.dz3 : T.dz2;
  const uint16_t* hh = L ? T.h2 : T.h1;
  f32x16 acc = f32x16{};
  for (int s0 = q * kChunk; s0 < (q + 1) * kChunk; s0 += 16) {
    // 8 consecutive samples of one unit are contiguous in the tile layout
    const int64_t sa = s0 + 8 * h;
    const float4 p0 = *reinterpret_cast<const float4*>(dz + tile_index(32 * ib + row, sa));
    const float4 p1 = *reinterpret_cast<const float4*>(dz + tile_index(32 * ib + row, sa) + 4);
    bf16x8 a;
    a[0] = (__bf16)p0.x;
    a[1] = (__bf16)p0.y;
    a[2] = (__bf16)p0.z;
    a[3] = (__bf16)p0.w;
    a[4] = (__bf16)p1.x;
    a[5] = (__bf16)p1.y;
    a[6] = (__bf16)p1.z;
    a[7] = (__bf16)p1.w;
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(hh + tile_index(32 * kb + row, sa));
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  float* out = T.part + ((size_t)(L * nchunks + q) << 16);
#pragma unroll
  for (int r = 0; r < 16; ++r)
    out[(32 * ib + 8 * (r >> 2) + 4 * h + (r & 3)) * kHid + 32 * kb + row] = acc[r];
}

__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.0f;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) t += red[w];
  return t;
}

// Gradient sums in a fixed order: blocks [0, 512) add the partials of dW2
// and dW3; block 512 + u sums unit u's dW1 row, db1, db2, db3 and dw4 over
// the batch; the last block db4 and the loss.
__global__ __launch_bounds__(kBlock) void mlp_reduce(Weights W, Train T, float* grad,
                                                     float* loss) {
  __shared__ float red[kBlock / 64];
  const int nchunks = (int)(T.Bp / kChunk);
  const int b = blockIdx.x;
  if (b < 512) {
    const int e = b * kBlock + threadIdx.x;
    const int L = e >> 16, at = e & 0xFFFF;
    float sum = 0.0f;
    for (int q = 0; q < nchunks; ++q) sum += T.part[((size_t)(L * nchunks + q) << 16) + at];
    grad[(L ? kOffW3 : kOffW2) + at] = sum;
    return;
  }
  const int64_t Bp = T.Bp;
  if (b < 512 + kHid) {
    const int unit = b - 512;
    float a[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) a[i] = 0.0f;
    for (int64_t s = threadIdx.x; s < Bp; s += kBlock) {
      const int64_t at = tile_index(unit, s);
      const float d1 = T.dz1[at];
#pragma unroll
      for (int c = 0; c < kIn; ++c) a[c] = fmaf(d1, T.u[s * 8 + c], a[c]);
      a[6] += d1;
      a[7] += T.dz2[at];
      a[8] += T.dz3[at];
      a[9] = fmaf(T.dy[s], silu(T.z3[at]), a[9]);
    }
    float tot[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) tot[i] = block_sum(a[i], red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < kIn; ++c) grad[kOffW1 + unit * kIn + c] = tot[c];
      grad[kOffB1 + unit] = tot[6];
      grad[kOffB2 + unit] = tot[7];
      grad[kOffB3 + unit] = tot[8];
      grad[kOffW4 + unit] = W.out_scale * tot[9];
    }
    return;
  }
  float gy = 0.0f, l = 0.0f;
  for (int64_t s = threadIdx.x; s < Bp; s += kBlock) gy += T.dy[s];
  for (int64_t w = threadIdx.x; w < Bp / kWaveRows; w += kBlock) l += T.lossp[w];
  gy = block_sum(gy, red);
  l = block_sum(l, red);
  if (threadIdx.x == 0) {
    grad[kOffB4] = W.out_scale * gy;
    if (loss) *loss = l;
  }
}

// Adam on the FP32 master parameters (when a.update), then every matrix
// weight's BF16 copy, in the forward and the transposed fragment layouts.
__global__ __launch_bounds__(kBlock) void mlp_adam(AdamArgs a) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= kParams) return;
  float v = a.master[p];
  if (a.update) {
    const float g = a.grad[p];
    const float m = fmaf(a.beta1, a.mom[p], (1.0f - a.beta1) * g);
    const float q = fmaf(a.beta2, a.vel[p], (1.0f - a.beta2) * g * g);
    a.mom[p] = m;
    a.vel[p] = q;
    v -= a.lr * (m * a.c1) / (sqrtf(q * a.c2) + a.eps);
    a.master[p] = v;
  }
  const uint16_t bits = bf16_bits(v);
  if (p < kOffB1) {
    const int i = p / kIn, c = p % kIn;
    a.w1[frag1_index(i, c)] = bits;
    a.w1[frag1_index(i, kIn + c)] = bits;
    if (c == 0)
      for (int z = 2 * kIn; z < 16; ++z) a.w1[frag1_index(i, z)] = 0;
  } else if (p >= kOffW2 && p < kOffB2) {
    const int i = (p - kOffW2) >> 8, k = (p - kOffW2) & 255;
    a.w2f[frag_index(i, k)] = bits;
    a.w2t[frag_index(k, i)] = bits;
  } else if (p >= kOffW3 && p < kOffB3) {
    const int i = (p - kOffW3) >> 8, k = (p - kOffW3) & 255;
    a.w3f[frag_index(i, k)] = bits;
    a.w3t[frag_index(k, i)] = bits;
  } else if (p >= kOffW4 && p < kOffB4) {
    a.w4[p - kOffW4] = bits;
  }
}

// ------------------------------------------------------------- launchers

hipError_t launch_forward(const Weights& W, int terms, const float* x, int64_t B, float* y,
                          uint8_t* in_range, hipStream_t s) {
  FwdIO io{x, B, y, in_range};
  Train T{};
  const dim3 grid((unsigned)((B + kBlockRows - 1) / kBlockRows));
  if (terms == 2)
    hipLaunchKernelGGL((mlp_forward<2, false>), grid, dim3(kBlock), 0, s, W, io, T);
  else
    hipLaunchKernelGGL((mlp_forward<1, false>), grid, dim3(kBlock), 0, s, W, io, T);
  return hipGetLastError();
}

hipError_t launch_train_grad(const Weights& W, int terms, const Train& T, float* grad,
                             float* loss, hipStream_t s) {
  FwdIO io{};
  const dim3 rows((unsigned)(T.Bp / kBlockRows));
  if (terms == 2)
    hipLaunchKernelGGL((mlp_forward<2, true>), rows, dim3(kBlock), 0, s, W, io, T);
  else
    hipLaunchKernelGGL((mlp_forward<1, true>), rows, dim3(kBlock), 0, s, W, io, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_backward, rows, dim3(kBlock), 0, s, W, T);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int jobs = 2 * 64 * (int)(T.Bp / kChunk);
  hipLaunchKernelGGL(mlp_wgrad, dim3((unsigned)(jobs / (kBlock / 64))), dim3(kBlock), 0, s, T);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_reduce, dim3(512 + kHid + 1), dim3(kBlock), 0, s, W, T, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam, dim3((kParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace mlp
}  // namespace qtree
