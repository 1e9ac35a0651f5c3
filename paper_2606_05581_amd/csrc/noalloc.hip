// Fixed device workspace of msk_estimate_dtn_noalloc, for callers that
// cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc). The array lives in the code
// object, so every device the library runs on holds its own copy from module
// load until the process ends. Host code never names the array itself (its
// host-side symbol is only a stand-in): the device address of each copy is
// looked up once per device, with that device current, and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "msk_internal.h"

namespace msk {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return g_err[device];
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_ptr[device] = e == hipSuccess ? p : nullptr;
  g_err[device] = e;
  g_done[device] = true;
  return e;
}

void* noalloc_scratch(int device, hipError_t* err) {
  if (device < 0 || device >= kMaxDevices) {
    if (err) *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (err) *err = g_done[device] ? g_err[device] : hipErrorNotInitialized;
  return g_ptr[device];
}

}  // namespace msk
