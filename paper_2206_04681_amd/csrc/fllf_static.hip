// fourier_llf_run_static: the filter of one job with the workspace taken from a
// fixed device array of this library instead of the caller (for callers that
// cannot allocate device memory: code under stream capture, tight serving
// loops).  The array lives in the code object, so every GPU the library runs on
// holds its own copy of it from the first use until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fllf_internal.h"

// The workspace of every call on a device.  Only its address as returned by
// hipGetSymbolAddress (kept per device below) is ever handed to a kernel or a
// runtime call: in host code the name stands for a host-side shadow.
static __device__ __align__(256) unsigned char scratch[FLLF_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices];   // device address of `scratch` on each device (null: not looked up yet)

// The device address of the array on `device` (looked up once per device,
// with that device current).
fllf_status scratch_on(fllf_ctx *ctx, int device, void **out) {
  if (device < 0 || device >= kMaxDevices)
    return fllf::ctx_fail(ctx, FLLF_EUNSUPPORTED, "run_static: device %d beyond the %d the library tracks", device,
                          kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    hipError_t e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fllf::ctx_fail(ctx, FLLF_EDEVICE, "run_static: address of the static workspace on device %d: %s",
                            device, hipGetErrorString(e));
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return FLLF_OK;
}

}  // namespace

extern "C" fllf_status fourier_llf_run_static(fllf_ctx *ctx, const fllf_job *job, void *hip_stream) {
  if (!ctx || !job) return fllf::ctx_fail(ctx, FLLF_EINVAL, "run_static: ctx and job must be non-NULL");
  void *ws = nullptr;
  const fllf_status st = scratch_on(ctx, fllf::ctx_device(ctx), &ws);
  if (st != FLLF_OK) return st;
  return fllf::run_single(ctx, "run_static", *job, ws, FLLF_STATIC_WORKSPACE_BYTES, (hipStream_t)hip_stream);
}
