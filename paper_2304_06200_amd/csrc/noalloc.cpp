// hg_eval_noalloc: hg_eval on memory the library owns from load time, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The device workspace is `scratch`, a fixed array of device memory defined
// here (the code object's zero-initialised data: one copy per device, held
// until the process ends).  In host code the name `scratch` is a host-side
// stand-in, not a device address; its device address is looked up once per
// device with hipGetSymbolAddress (hg_create calls noalloc_setup with the
// device current) and only that address reaches kernels or copies.  The host
// staging is a fixed host array per device.  Calls that overlap on one device
// share both and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hg_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kHostStageBytes = (size_t)2 << 20;
constexpr int kDevices = 16;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_dev[kDevices];
alignas(256) char g_host_stage[kDevices][kHostStageBytes];

hg_status nfail(hg_status s, const std::string& msg) {
  hg::set_error(msg);
  return s;
}

}  // namespace

namespace hg {

hg_status noalloc_setup(int device) {
  if (device < 0 || device >= kDevices)
    return nfail(HG_ERR_UNSUPPORTED, "device ordinal " + std::to_string(device) +
                                         " beyond the no-allocation scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch_dev[device]) return HG_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess)
    return nfail(HG_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  if (!ptr) return nfail(HG_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_dev[device] = ptr;
  return HG_OK;
}

}  // namespace hg

extern "C" {

hg_status hg_eval_noalloc(hg_problem* p, const hg_eval_desc* d, hg_result* results, double* grad,
                          void* stream) {
  try {
    if (!p || !p->ctx) return nfail(HG_ERR_INVALID_ARG, "NULL problem");
    if (d && (d->flags & HG_FLAG_TIMING))
      return nfail(HG_ERR_INVALID_ARG, "hg_eval_noalloc: HG_FLAG_TIMING needs events (use hg_eval)");
    const int dev = p->ctx->device;
    void* ws = nullptr;
    if (dev >= 0 && dev < kDevices) {
      std::lock_guard<std::mutex> lk(g_mu);
      ws = g_scratch_dev[dev];
    }
    if (!ws) return nfail(HG_ERR_DEVICE, "no scratch address for device " + std::to_string(dev));
    return hg::eval_on_buffers(p, d, results, grad, (hipStream_t)stream, ws, kScratchBytes,
                               g_host_stage[dev], kHostStageBytes, false);
  } catch (const std::bad_alloc&) {  // error messages are the only host allocations here
    return nfail(HG_ERR_OUT_OF_MEMORY, "hg_eval_noalloc: host allocation failed");
  } catch (...) {
    return nfail(HG_ERR_DEVICE, "hg_eval_noalloc: unexpected exception");
  }
}

hg_status hg_eval_noalloc_limits(size_t* scratch_bytes, size_t* host_stage_bytes) {
  if (scratch_bytes) *scratch_bytes = kScratchBytes;
  if (host_stage_bytes) *host_stage_bytes = kHostStageBytes;
  return HG_OK;
}

}  // extern "C"
