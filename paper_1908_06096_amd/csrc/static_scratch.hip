// Transforms for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// Fourier workspace comes from a fixed array in the library's device memory
// instead of a caller-supplied buffer.
//
// The array is a file-scope device variable, so every GPU the library runs
// on holds its own copy (kScratchBytes) from the moment the code object is
// loaded until the process ends.  Its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and kept; the
// host-side name `scratch` is only a stand-in and is never passed to a
// kernel or a copy.
//
// No kernel here needs the scratch to start at zero: every Fourier row a
// stage reads has been written earlier in the same call (padding fields
// beyond F are read by the analysis product but only feed outputs that are
// never stored), so nothing is cleared between calls.
#include <mutex>

#include "sht_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)SHT_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on
// the first call on that device).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int sht_transform_static(sht_plan_t plan, int direction, const void* in, void* out, void* hip_stream) {
  if (!plan || !in || !out) return SHT_EINVAL;
  if (direction != SHT_DIR_INVERSE && direction != SHT_DIR_DIRECT) return SHT_EINVAL;
  if (sht_workspace_size(plan) > kScratchBytes) return SHT_ESCRATCH;
  void* ws = nullptr;
  const hipError_t e = scratch_address(&ws);
  if (e != hipSuccess) return shtmi::hip_status(e);
  return direction == SHT_DIR_INVERSE ? sht_inverse(plan, in, out, ws, hip_stream)
                                      : sht_direct(plan, in, out, ws, hip_stream);
}
