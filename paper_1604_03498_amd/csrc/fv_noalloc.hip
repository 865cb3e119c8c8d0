// fv_encode_noalloc: the single-frame encode for callers that cannot allocate device memory.
// Every intermediate lives in one fixed array per GPU, `scratch`, which is part of this
// library's code object: the runtime places it on each GPU when the code object is loaded
// there and it stays until the process ends.  In host code the array's name stands for a
// host-side shadow, never for the device memory: the device address is looked up with
// hipGetSymbolAddress once per device (with that device current) and only that address is
// handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fv.h"
#include "fv_internal.h"

static __device__ __align__(256) char scratch[FV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (a fixed table)

// The device address of `scratch` on `device`, which is current.
int scratch_on(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) return FV_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fv::device_error(e);
    if (!p) return fv::device_error(hipErrorInvalidSymbol);
    g_ptr[device] = static_cast<char*>(p);
  }
  *out = g_ptr[device];
  return FV_OK;
}

}  // namespace

extern "C" int fv_encode_noalloc(const fv_gmm* gmm, const float* X, int64_t N, float* out,
                                 int precision, unsigned flags, void* hip_stream) {
  if (!gmm) return FV_E_INVAL;
  if ((flags & (FV_X_DEVICE | FV_OUT_DEVICE)) != (FV_X_DEVICE | FV_OUT_DEVICE)) return FV_E_INVAL;
  int device = 0;
  if (fv_gmm_info(gmm, nullptr, nullptr, &device) != FV_OK) return FV_E_INVAL;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != device) {
    const int rc = fv::set_device(device);
    if (rc) return rc;
  }
  char* ptr = nullptr;
  int rc = scratch_on(device, &ptr);
  if (rc == FV_OK)
    rc = fv::encode_on_scratch(gmm, X, N, out, precision, flags, hip_stream, ptr,
                               FV_NOALLOC_SCRATCH_BYTES);
  if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  return rc;
}
