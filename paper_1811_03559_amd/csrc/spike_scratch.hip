// Allocation-free factorisation: spike_factor with the library's own
// device scratch array as the workspace, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ object, so every GPU the library runs
// on holds one copy (kScratchBytes) from module load until the process ends.
// Host code never uses the array's name as an address: its device address
// is taken once per device with hipGetSymbolAddress, with that device
// current, and kept per device.  Every call on one GPU shares that GPU's
// array: a later call overwrites the factorisation of an earlier one, and
// calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/spike.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (resolved on the first
// call on the device), or an error code.
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return SPIKE_ERR_HIP - (int)e;
  if (dev < 0 || dev >= kMaxDevices) return SPIKE_ERR_HIP - (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return SPIKE_ERR_HIP - (int)e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return 0;
}

}  // namespace

extern "C" {

size_t spike_scratch_capacity(void) { return kScratchBytes; }

int spike_factor_scratch(int64_t n, int32_t kl, int32_t ku, const double* dAB, int64_t ldab,
                         const spike_opts* opts, hipStream_t stream, spike_handle* out) {
  if (n < 0) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  if (dAB == nullptr && n > 0) return -4;
  if (ldab < (int64_t)kl + ku + 1) return -5;
  size_t need = 0;
  if (spike_workspace_size(n, kl, ku, opts, &need) != 0) return -6;
  if (need > kScratchBytes) return -7;
  if (out == nullptr) return -8;
  void* ws = nullptr;
  if (int e = scratch_ptr(&ws)) return e;
  return spike_factor(n, kl, ku, dAB, ldab, opts, ws, kScratchBytes, stream, out);
}

}  // extern "C"
