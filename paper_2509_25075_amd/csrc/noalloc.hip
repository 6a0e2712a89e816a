// qs_adjoint_backward_noalloc: the adjoint of the register/LDS engine with
// its per-block gradient partial sums in a library-owned device array
// instead of a caller workspace, for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid
// allocation). Nothing here allocates: the array is a file-scope device
// global, and the call runs only shapes whose plans an earlier allocating
// call already cached.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qs_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // QS_NOALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;

// One copy per GPU, alive until the process ends. Host code never uses this
// name as an address: it takes each device's address from
// hipGetSymbolAddress, once per device, with that device current.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call made on that device.
int scratch_ptr(void** out) {
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return QS_ERR_LAUNCH;
  if (device < 0 || device >= kMaxDevices) return QS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return QS_ERR_LAUNCH;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return QS_OK;
}

}  // namespace

static_assert(kScratchBytes == QS_NOALLOC_SCRATCH_BYTES, "header and library disagree");

extern "C" int qs_adjoint_backward_noalloc(const qs_circuit* c, int dtype, int64_t B,
                                           const void* params, const void* feats,
                                           const void* state, const double* dexpz,
                                           const void* dstate, double* grad_params,
                                           double* grad_feats, const int32_t* ckpt_gates,
                                           int32_t n_ckpt, const void* ckpt, int flags,
                                           void* stream) {
  void* ws = nullptr;
  const int rc = scratch_ptr(&ws);
  if (rc != QS_OK) return rc;
  return qs::adjoint_backward_impl(c, dtype, B, params, feats, state, dexpz, dstate,
                                   grad_params, grad_feats, ckpt_gates, n_ckpt, ckpt, ws,
                                   kScratchBytes, flags, stream, true);
}
