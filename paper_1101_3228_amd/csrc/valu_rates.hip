// Calibration program for the ALU rooflines: sustained issue rate of single
// VALU opcodes (and a few pairs) on the GPU it runs on, in lane-operations per
// clock per CU at the 2.4 GHz peak engine clock.
//
// Each kernel runs 8 independent register chains per lane of one opcode (inline
// asm on registers only, no memory access inside the loop), 256 threads per
// workgroup, 32 workgroups per CU (8 waves per SIMD), and writes one word per
// thread at the end.  The best of 3 launches is reported.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kIters = 2048;
constexpr int kThreads = 256;

#define CHAINS(S) S(0) S(1) S(2) S(3) S(4) S(5) S(6) S(7)

// One kernel per opcode: `STEP(J)` issues the instruction(s) on chain J.
#define RATE_KERNEL(NAME, STEP)                                                              \
  __global__ __launch_bounds__(kThreads) void NAME(uint32_t* out, uint32_t b, uint32_t c) {  \
    uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4,           \
             a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;                                          \
    uint32_t e0 = 3 * a0, e1 = 3 * a1, e2 = 3 * a2, e3 = 3 * a3, e4 = 3 * a4, e5 = 3 * a5,    \
             e6 = 3 * a6, e7 = 3 * a7;                                                        \
    uint64_t d0 = a0, d1 = a1, d2 = a2, d3 = a3, d4 = a4, d5 = a5, d6 = a6, d7 = a7;         \
    uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0, m6 = 0, m7 = 0;                 \
    for (int i = 0; i < kIters; ++i) {                                                       \
      CHAINS(STEP)                                                                           \
    }                                                                                        \
    const uint64_t w = d0 ^ d1 ^ d2 ^ d3 ^ d4 ^ d5 ^ d6 ^ d7 ^ m0 ^ m1 ^ m2 ^ m3 ^ m4 ^ m5 ^  \
                       m6 ^ m7;                                                              \
    out[blockIdx.x * kThreads + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^ e0 ^  \
                                               e1 ^ e2 ^ e3 ^ e4 ^ e5 ^ e6 ^ e7 ^ (uint32_t)w; \
  }

// fp32 arithmetic, all operands in VGPRs / inline constants / literals
#define S_FMA(J) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a##J) : "v"(b), "v"(c));
#define S_FMAAK(J) asm volatile("v_fmaak_f32 %0, %0, %1, 0x3e9a209b" : "+v"(a##J) : "v"(b));
#define S_ADDF(J) asm volatile("v_add_f32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_MULF(J) asm volatile("v_mul_f32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
// the same with one SGPR operand
#define S_FMA_S(J) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a##J) : "s"(b), "v"(c));
// integer and bitwise
#define S_ADDU(J) asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_XOR(J) asm volatile("v_xor_b32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_AND(J) asm volatile("v_and_b32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_LSHR(J) asm volatile("v_lshrrev_b32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_LSHL(J) asm volatile("v_lshlrev_b32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_ADD3(J) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a##J) : "v"(b), "v"(c));
#define S_MULHI(J) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a##J) : "v"(b));
#define S_MAD64(J) \
  asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(d##J) : "v"(b), "v"(c) : "vcc");
// compare, select, min
#define S_MINF(J) asm volatile("v_min_f32_e32 %0, %1, %0" : "+v"(a##J) : "v"(b));
#define S_CMP(J) asm volatile("v_cmp_lt_f32_e64 %0, %1, %2" : "=s"(m##J) : "v"(a##J), "v"(b));
#define S_CND(J) \
  asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a##J) : "v"(b), "s"(0x5555ull));
#define S_CVT(J) asm volatile("v_cvt_f32_u32_e32 %0, %0" : "+v"(a##J));
// transcendental
#define S_EXP(J) asm volatile("v_exp_f32_e32 %0, %0" : "+v"(a##J));
#define S_SQRT(J) asm volatile("v_sqrt_f32_e32 %0, %0" : "+v"(a##J));
// fp64
#define S_FMA64(J) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(d##J) : "v"(d0));
// pairs: a half-rate op next to a full-rate op
#define S_MIN_ADD(J) \
  asm volatile("v_min_f32_e32 %0, %2, %0\n\tv_add_f32_e32 %1, %2, %1" : "+v"(a##J), "+v"(e##J) : "v"(b));
#define S_MAD64_XOR(J)                                                                   \
  asm volatile("v_mad_u64_u32 %0, vcc, %2, %3, 0\n\tv_xor_b32_e32 %1, %3, %1"           \
               : "+v"(d##J), "+v"(a##J) : "v"(b), "v"(c) : "vcc");
#define S_CMP_CND(J)                                                                     \
  asm volatile("v_cmp_lt_f32_e64 %1, %0, %2\n\tv_cndmask_b32_e64 %0, %0, %2, %1"        \
               : "+v"(a##J), "=s"(m##J) : "v"(b));

RATE_KERNEL(k_fma, S_FMA)
RATE_KERNEL(k_fmaak, S_FMAAK)
RATE_KERNEL(k_addf, S_ADDF)
RATE_KERNEL(k_mulf, S_MULF)
RATE_KERNEL(k_fma_s, S_FMA_S)
RATE_KERNEL(k_addu, S_ADDU)
RATE_KERNEL(k_xor, S_XOR)
RATE_KERNEL(k_and, S_AND)
RATE_KERNEL(k_lshr, S_LSHR)
RATE_KERNEL(k_lshl, S_LSHL)
RATE_KERNEL(k_add3, S_ADD3)
RATE_KERNEL(k_mulhi, S_MULHI)
RATE_KERNEL(k_mad64, S_MAD64)
RATE_KERNEL(k_minf, S_MINF)
RATE_KERNEL(k_cmp, S_CMP)
RATE_KERNEL(k_cnd, S_CND)
RATE_KERNEL(k_cvt, S_CVT)
RATE_KERNEL(k_exp, S_EXP)
RATE_KERNEL(k_sqrt, S_SQRT)
RATE_KERNEL(k_fma64, S_FMA64)
RATE_KERNEL(k_min_add, S_MIN_ADD)
RATE_KERNEL(k_mad64_xor, S_MAD64_XOR)
RATE_KERNEL(k_cmp_cnd, S_CMP_CND)

typedef void (*Kernel)(uint32_t*, uint32_t, uint32_t);

struct Entry {
  const char* name;
  Kernel k;
  int per_step;  // instructions per chain step
};

}  // namespace

int main() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    fprintf(stderr, "no HIP device\n");
    return 1;
  }
  const int blocks = cus * 32;
  uint32_t* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kThreads * sizeof(uint32_t)) != hipSuccess) return 1;
  const Entry table[] = {
      {"v_fma_f32 (VGPR operands)", k_fma, 1},  {"v_fmaak_f32 (literal)", k_fmaak, 1},
      {"v_add_f32", k_addf, 1},                 {"v_mul_f32", k_mulf, 1},
      {"v_fma_f32 (one SGPR operand)", k_fma_s, 1},
      {"v_add_u32", k_addu, 1},                 {"v_xor_b32", k_xor, 1},
      {"v_and_b32", k_and, 1},                  {"v_lshrrev_b32", k_lshr, 1},
      {"v_lshlrev_b32", k_lshl, 1},             {"v_add3_u32", k_add3, 1},
      {"v_mul_hi_u32", k_mulhi, 1},             {"v_mad_u64_u32", k_mad64, 1},
      {"v_min_f32", k_minf, 1},                 {"v_cmp_lt_f32 (to SGPR)", k_cmp, 1},
      {"v_cndmask_b32 (SGPR mask)", k_cnd, 1},  {"v_cvt_f32_u32", k_cvt, 1},
      {"v_exp_f32", k_exp, 1},                  {"v_sqrt_f32", k_sqrt, 1},
      {"v_fma_f64", k_fma64, 1},                {"v_min_f32 + v_add_f32", k_min_add, 2},
      {"v_mad_u64_u32 + v_xor_b32", k_mad64_xor, 2},
      {"v_cmp_lt_f32 + v_cndmask_b32", k_cmp_cnd, 2},
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  printf("| Opcode(s) | lane-instructions / clock / CU |\n|---|---|\n");
  for (const Entry& t : table) {
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, 0) != hipSuccess) return 1;
      hipLaunchKernelGGL(t.k, dim3(blocks), dim3(kThreads), 0, 0, out, 3u, 5u);
      if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
      if (ms < best) best = ms;
    }
    const double lane_instr = (double)blocks * kThreads * kIters * 8 * t.per_step;
    printf("| %s | %.1f |\n", t.name, lane_instr / (best * 1e-3) / (cus * 2.4e9));
  }
  const hipError_t err = hipGetLastError();
  (void)hipFree(out);
  if (err != hipSuccess) {
    fprintf(stderr, "%s\n", hipGetErrorString(err));
    return 1;
  }
  return 0;
}
