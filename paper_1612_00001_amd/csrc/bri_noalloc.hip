// invert_block_noalloc: invert_block with its workspace in a file-scope
// device array, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The array `scratch` below is the workspace: slots, permutations, tile
// scratch, the status word and the step descriptors of one call.  In host
// code its name is only a host-side stand-in, so the device address is
// looked up with hipGetSymbolAddress, once per device (with that device
// current, on the first call made there), and only that address is used:
// the kernels take it as their workspace argument.  Every GPU the library
// runs on holds its own copy of the array until the process ends.  All calls
// on one GPU share it and it keeps the last call's contents, so calls that
// overlap in time on one GPU race; the kernels clear what must start at zero
// (the status word) themselves.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bri.h"

namespace bri {
// invert_block into the given scratch, staging its descriptors without
// allocating (bri_api.cpp).
int invert_block_scratch(const void* M, int64_t n, int64_t ldm, int k, int i, int j, void* out, int64_t ldo,
                         const bri_opts* o, void* scratch, size_t scratch_bytes);
}  // namespace bri

namespace {

constexpr size_t kScratchBytes = BRI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once).
int scratch_address(void** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BRI_ERR_HIP;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BRI_ERR_HIP;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return BRI_OK;
}

}  // namespace

extern "C" {

size_t bri_noalloc_scratch_bytes(void) { return kScratchBytes; }

int invert_block_noalloc(const void* M, int64_t n, int64_t ldm, int k, int i, int j, void* out, int64_t ldo,
                         const bri_opts* o) {
  if (!o) return -9;
  if (o->precision != BRI_F64 && o->precision != BRI_F32) return BRI_ERR_UNSUPPORTED;
  void* ptr = nullptr;
  const int rc = scratch_address(&ptr);
  if (rc != BRI_OK) return rc;
  return bri::invert_block_scratch(M, n, ldm, k, i, j, out, ldo, o, ptr, kScratchBytes);
}

}  // extern "C"
