// akf_noalloc.hip -- akf_mh_step_noalloc: one auxiliary Kalman MH step whose
// scratch memory is a fixed device array of the library instead of a caller
// workspace, for callers that cannot allocate device memory (code under graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The step itself is akf_mh_step's (same kernels, same launch sequence); only
// the workspace pointer differs.  Every device keeps its own copy of the array
// at its own address, found once per device with hipGetSymbolAddress and kept
// in g_addr.  The array's name is a host-side stand-in and is never passed to
// a kernel or a copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/akf.h"
#include "akf_layout.h"

namespace {

__device__ __align__(256) unsigned char scratch[AKF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices];  // device address of `scratch` per device, once found

// The device address of this device's scratch array.  `dev` must be current.
akf_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return akf::fail(AKF_ERR_UNSUPPORTED, "akf_mh_step_noalloc: device %d beyond the %d supported",
                     dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return akf::fail(AKF_ERR_HIP, "akf_mh_step_noalloc: hipGetSymbolAddress of the scratch "
                       "array on device %d: %s", dev, hipGetErrorString(e));
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return AKF_OK;
}

}  // namespace

extern "C" {

akf_status akf_mh_step_noalloc(const akf_model* model, const double* y, const double* x_in,
                               double delta, int32_t order, const double* xi, const double* unif,
                               double* x_out, double* log_ratio, int32_t* accepted,
                               double* logZ_fwd, double* logZ_rev, int32_t* status, int32_t block,
                               void* stream) {
  // size check first: an invalid model sizes to 0 and akf_mh_step reports why
  const size_t need = akf_mh_workspace_bytes(model, order, block);
  if (need > (size_t)AKF_NOALLOC_SCRATCH_BYTES)
    return akf::fail(AKF_ERR_SHAPE, "akf_mh_step_noalloc: this problem needs %zu bytes of scratch "
                     "memory, more than the %zu bytes the library holds per device; use "
                     "akf_mh_step with a workspace", need, (size_t)AKF_NOALLOC_SCRATCH_BYTES);
  int cur = -1, sdev = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess)
    return akf::fail(AKF_ERR_HIP, "akf_mh_step_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  e = hipStreamGetDevice((hipStream_t)stream, &sdev);
  if (e != hipSuccess)
    return akf::fail(AKF_ERR_HIP, "akf_mh_step_noalloc: hipStreamGetDevice: %s",
                     hipGetErrorString(e));
  if (sdev != cur)
    return akf::fail(AKF_ERR_INVALID, "akf_mh_step_noalloc: the stream belongs to device %d but "
                     "device %d is current; make the stream's device current", sdev, cur);
  void* ws = nullptr;
  akf_status s = scratch_address(cur, &ws);
  if (s != AKF_OK) return s;
  return akf_mh_step(model, y, x_in, delta, order, xi, unif, x_out, log_ratio, accepted, logZ_fwd,
                     logZ_rev, status, ws, (size_t)AKF_NOALLOC_SCRATCH_BYTES, block, stream);
}

}  // extern "C"
