// Device layout of the pricing surrogate (6-256-256-256-1 perceptron).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtree {
namespace mlp {

constexpr int kIn = 6;
constexpr int kHid = 256;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid;
constexpr int kOffB4 = kOffW4 + kHid;
constexpr int kParams = kOffB4 + 1;  // 133 633
constexpr int kBlock = 256;          // 4 waves
constexpr int kWaveRows = 32;        // samples per wave (one MFMA column block)
constexpr int kBlockRows = kBlock / 64 * kWaveRows;
constexpr int kChunk = 256;          // samples per weight-gradient partial; training rows pad to it

// Network as the kernels read it.  Matrix weights are BF16 (raw bits);
// w1f holds W1 as the A operand of one K-step (see mlp.hip), w2f / w3f hold
// W2, W3 as MFMA A-operand fragments, w2t / w3t the same for the transposes.
struct Weights {
  const float* master;  // FP32 packed parameters (biases are read from here)
  const uint16_t* w1;   // [8][64][8] fragments of W1
  const uint16_t* w4;   // [256]
  const uint16_t* w2f;
  const uint16_t* w3f;
  const uint16_t* w2t;
  const uint16_t* w3t;
  float lo[kIn], hi[kIn], scale[kIn], shift[kIn];
  float out_scale;
  int baseline;  // 1: add the Black-Scholes European put per unit strike
};

// Training batch and its buffers.  Rows are padded to Bp (a multiple of
// kChunk).  Per-unit arrays (z, h, dz) are stored in the accumulator tile
// layout of the kernels: element (unit, sample s) at
//   ((s / 32) * 8 + unit / 32) * 1024 + r * 64 + 32 h + s % 32
// with u = unit % 32, h = (u / 4) % 2, r = 4 (u / 8) + u % 4, so that a wave
// addresses its 32 samples with constant offsets and the 32 samples of one
// unit are contiguous.
struct Train {
  const float* x;      // [rows][6] training set
  const float* t;      // [rows]
  const float* w;      // [rows] or NULL (ones)
  const int32_t* idx;  // [B] rows of this batch, or NULL (0..B-1)
  int64_t B, Bp;
  float inv_b;
  float* z1;
  float* z2;
  float* z3;
  uint16_t* h1;        // BF16 inputs of layers 2 and 3 (hi term)
  uint16_t* h2;
  float* dz1;
  float* dz2;
  float* dz3;
  float* u;            // [Bp][8] normalised inputs
  float* dy;           // [Bp]
  float* lossp;        // [Bp / 32]
  float* part;         // [2][Bp / kChunk][256][256] weight-gradient partials
};

struct AdamArgs {
  float* master;
  float* mom;
  float* vel;
  const float* grad;
  uint16_t* w1;
  uint16_t* w4;
  uint16_t* w2f;
  uint16_t* w3f;
  uint16_t* w2t;
  uint16_t* w3t;
  float lr, beta1, beta2, eps, c1, c2;  // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
  int update;                           // 0: only refresh the BF16 copies
};

hipError_t launch_forward(const Weights& W, int terms, const float* x, int64_t B, float* y,
                          uint8_t* in_range, hipStream_t s);
hipError_t launch_train_grad(const Weights& W, int terms, const Train& T, float* grad,
                             float* loss, hipStream_t s);
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);

}  // namespace mlp
}  // namespace qtree
