// Forward step whose two-pass counting scratch is a fixed device array of
// the library instead of device memory the caller grants, for callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc).  Contract in include/qtree.h.
//
// The array is a file-scope __device__ symbol.  In host code its name is a
// host-side stand-in, not a device address, so the first call on a device
// (with that device current) asks the runtime for the array's address on
// that device and keeps it; every later use -- the kernels' key and segment
// pointers -- takes that address.  Each device holds its own copy of the
// array until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "qtree.h"
#include "qtree_internal.hpp"
#include "qtree_plan.hpp"

namespace {

constexpr size_t kFixedScratchBytes = size_t(64) << 20;  // QTREE_FIXED_SCRATCH_BYTES
constexpr int kMaxDevices = 64;

static_assert(kFixedScratchBytes == (size_t)QTREE_FIXED_SCRATCH_BYTES,
              "the header states the size of the fixed scratch");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once per device).
qtree_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return qtree::set_error(QTREE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return qtree::set_error(QTREE_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return qtree::set_error(QTREE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                 hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return QTREE_OK;
}

}  // namespace

extern "C" {

qtree_status qtree_transitions_fixed_scratch(const qtree_plan* plan, uint64_t m0, uint64_t M,
                                             uint64_t seed, uint32_t contract_id,
                                             qtree_mode mode, int32_t* counts, void* stream) {
  if (!plan) return qtree::set_error(QTREE_EINVAL, "plan is NULL");
  void* base = nullptr;
  const qtree_status st = scratch_on_current_device(&base);
  if (st != QTREE_OK) return st;
  return qtree::transitions_on_scratch(plan, m0, M, seed, contract_id, mode, counts, stream, base,
                                       kFixedScratchBytes);
}

}  // extern "C"
