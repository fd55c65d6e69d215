// noalloc.hip -- the training step of a two-stage chain for callers that
// cannot allocate device memory (code under stream capture, serving loops,
// harnesses that forbid hipMalloc).
//
// rsm_run_chain_train keeps the per-workgroup weight-gradient partial rows in
// the stream's grow-only library workspace, which it allocates on first use.
// This variant keeps them in a fixed array of device memory defined here
// instead and never allocates.  The array's device address differs per GPU
// (each device holds its own copy of the module's globals), so it is looked
// up with hipGetSymbolAddress once per device, on that device's first call,
// and the looked-up address is what the kernels receive: the array's name in
// host code is only a host-side stand-in, not a device address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rsm_internal.h"

namespace {

// Partial rows of the fused training step: at most 256 x 8 workgroups, each
// writing one row of at most 32 floats (the weight gradients of two stages
// of at most 16 taps): 2048 x 32 x 4 bytes = 256 KiB.
constexpr size_t kScratchBytes = size_t(256) << 10;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
rsm_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rsm::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return rsm::fail(RSM_E_UNSUPPORTED, "device ordinal " + std::to_string(dev) + " is beyond the " +
                                            std::to_string(kMaxDevices) + " devices the fixed scratch table covers");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return rsm::hip_fail(e, "hipGetSymbolAddress (fixed scratch buffer)");
    if (!p) return rsm::fail(RSM_E_HIP, "hipGetSymbolAddress returned a null address for the scratch buffer");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RSM_OK;
}

}  // namespace

extern "C" {

rsm_status rsm_run_chain_train_noalloc(const rsm_stage* stages, int32_t n_stages, const void* d_in,
                                       const void* d_w, void* d_out, void* d_gx, void* const* d_gc,
                                       uint32_t flags, void* hip_stream) {
  try {
    void* p = nullptr;
    const rsm_status s = scratch_address(&p);
    if (s != RSM_OK) return s;
    return rsm::chain_train_step(stages, n_stages, d_in, d_w, d_out, d_gx, d_gc, flags, hip_stream,
                                 static_cast<float*>(p), kScratchBytes);
  } catch (...) {
    return rsm::fail(RSM_E_INVALID, "internal error (exception)");
  }
}

}  // extern "C"
