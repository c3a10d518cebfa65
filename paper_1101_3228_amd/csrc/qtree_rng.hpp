// Device-side random numbers and Gaussian transform for the forward kernels.
//
// The paper draws its innovations from drand48 / MRG32k3a / XORWOW streams
// (Sec. 3, "Random number generation"); here every sample is a pure function
// of a counter, so no generator state exists and any thread can produce any
// sample: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) followed by the
// Box-Muller transform.  ln, sin and cos are evaluated by fixed sequences of
// IEEE FP32 operations (explicit fmaf, correctly rounded sqrt, no hardware
// approximations) so that the result is a bit-reproducible function of the
// counter.  Build with -ffp-contract=off.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtree {

struct U4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10: ten rounds of two 32x32->64 products; the key advances by
// the Weyl increments 0x9E3779B9, 0xBB67AE85 between rounds.
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// A wave-uniform 32-bit value (held in a scalar register) copied into a
// vector register.  On gfx950 a vector instruction with a scalar-register
// operand issues at half the rate of one whose operands are all vector
// registers, inline constants or literals, so a uniform value that feeds
// many vector operations is copied once.  Only for values that are uniform
// across the wave (kernel arguments and what is computed from them).
__device__ __forceinline__ uint32_t vgpr_copy(uint32_t s) {
  uint32_t v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

__device__ __forceinline__ float vgpr_copy(float s) {
  return __uint_as_float(vgpr_copy(__float_as_uint(s)));
}

// The same Philox4x32-10 for a wave-uniform key: the key is copied into
// vector registers and advanced there, so that all four xors of a round take
// vector operands (same function, same result).
__device__ __forceinline__ U4 philox4x32_10_vk(U4 c, uint32_t k0, uint32_t k1) {
  return philox4x32_10(c, vgpr_copy(k0), vgpr_copy(k1));
}

// ln(K 2^-24) for K in [1, 2^24].  K = 2^e f with f folded into [2/3, 4/3)
// by an exact halving; ln(1+t) for t = f - 1 (exact) is the Mercator series
// through t^14 by Horner; ln 2 = LN2_HI + LN2_LO with e*LN2_HI exact.
__device__ __forceinline__ float ln_u24(uint32_t K) {
  const float F = (float)K;
  const uint32_t bits = __float_as_uint(F);
  int e = (int)(bits >> 23) - 127;
  uint32_t mb = (bits & 0x007FFFFFu) | 0x3F800000u;
  if (mb >= 0x3FAAAAABu) {
    mb -= 0x00800000u;
    e += 1;
  }
  const float t = __uint_as_float(mb) - 1.0f;
  // (-1)^(n+1)/n rounded to FP32, n = 14 .. 2
  float P = -0x1.24924ap-4f;
  P = fmaf(P, t, 0x1.3b13b2p-4f);
  P = fmaf(P, t, -0x1.555556p-4f);
  P = fmaf(P, t, 0x1.745d18p-4f);
  P = fmaf(P, t, -0x1.99999ap-4f);
  P = fmaf(P, t, 0x1.c71c72p-4f);
  P = fmaf(P, t, -0x1p-3f);
  P = fmaf(P, t, 0x1.24924ap-3f);
  P = fmaf(P, t, -0x1.555556p-3f);
  P = fmaf(P, t, 0x1.99999ap-3f);
  P = fmaf(P, t, -0x1p-2f);
  P = fmaf(P, t, 0x1.555556p-2f);
  P = fmaf(P, t, -0x1p-1f);
  const float w = t * t;
  const float r = fmaf(w, P, t);
  const float ee = (float)(e - 24);
  const float s = fmaf(ee, 0x1.7f7d1cp-20f, r);  // LN2_LO
  return fmaf(ee, 0x1.62e4p-1f, s);              // LN2_HI = floor(ln2 2^16) 2^-16
}

// sin and cos of 2 pi J 2^-24, J in [0, 2^24): quadrant and reflection in
// integer arithmetic, Taylor series of sin(pi y/2) (to y^9) and
// cos(pi y/2) (to y^10) on y in [0, 1/2].
__device__ __forceinline__ void sincos_2pi_u24(uint32_t J, float& sn, float& cs) {
  const uint32_t q = J >> 22;
  uint32_t r = J & 0x003FFFFFu;
  const bool swap = r > 0x00200000u;
  r = swap ? 0x00400000u - r : r;
  const float y = (float)r * 0x1p-22f;
  const float w = y * y;
  float ps = fmaf(0x1.507834p-13f, w, -0x1.32d2ccp-8f);
  ps = fmaf(ps, w, 0x1.466bc6p-4f);
  ps = fmaf(ps, w, -0x1.4abbcep-1f);
  ps = fmaf(ps, w, 0x1.921fb6p+0f);
  const float sy = ps * y;
  float pc = fmaf(-0x1.a6d1f2p-16f, w, 0x1.e1f506p-11f);
  pc = fmaf(pc, w, -0x1.55d3c8p-6f);
  pc = fmaf(pc, w, 0x1.03c1f0p-2f);
  pc = fmaf(pc, w, -0x1.3bd3ccp+0f);
  const float cy = fmaf(pc, w, 1.0f);
  const float sp = swap ? cy : sy;
  const float cp = swap ? sy : cy;
  // rotate by q quarter turns: (s, c) -> (c, -s) per quarter
  const float a = (q & 1u) ? cp : sp;
  const float b = (q & 1u) ? sp : cp;
  const uint32_t sgn_s = (q & 2u) ? 0x80000000u : 0u;
  const uint32_t sgn_c = ((q + 1u) & 2u) ? 0x80000000u : 0u;
  sn = __uint_as_float(__float_as_uint(a) ^ sgn_s);
  cs = __uint_as_float(__float_as_uint(b) ^ sgn_c);
}

// Correctly rounded square root of a in {+0, -0} u [2^-24, 64] (the
// Box-Muller radius argument; -0 when u_a = 1).  r = the hardware estimate (within one ulp), rd its
// predecessor (r (1 - 2^-24) rounds to it for every normal r), ru = the
// successor of rd's successor; the residuals rd r - a and ru r - a, each
// one rounded fma, decide between the three candidates (the neighbour test
// of the IEEE square root): rd when rd r >= a, ru when ru r < a, else r.
// An exact zero residual is +0, so each decision is the residual's sign bit
// and the result is bits(rd) + [rd r < a] + [ru r < a].  On this domain no
// residual underflows, so no input scaling is needed; a = +-0 gives
// r = rd = +-0 (the hardware square root keeps the sign of zero), both
// residuals +0 and the result +-0.
__device__ __forceinline__ float sqrt_rn_radius(float a) {
  const float r = __builtin_amdgcn_sqrtf(a);
  const float rd = r * 0x1.fffffep-1f;
  const uint32_t rb = __float_as_uint(rd);
  const float ru = __uint_as_float(rb + 2u);
  const uint32_t ed = __float_as_uint(fmaf(rd, r, -a));
  const uint32_t eu = __float_as_uint(fmaf(ru, r, -a));
  return __uint_as_float(rb + (ed >> 31) + (eu >> 31));
}

// Box-Muller: rho = sqrt(-2 ln u_a), u_a = ((ra >> 8) + 1) 2^-24 in (0, 1];
// angle 2 pi u_b, u_b = (rb >> 8) 2^-24.  z0 = rho cos, z1 = rho sin.
__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, float& z0, float& z1) {
  const float l = ln_u24((ra >> 8) + 1u);
  const float rho = sqrt_rn_radius(-2.0f * l);
  float s, c;
  sincos_2pi_u24(rb >> 8, s, c);
  z0 = rho * c;
  z1 = rho * s;
}

}  // namespace qtree
