// Entry points of the register engine: direction and element-type dispatch
// (the instantiations live in sv_c64_fwd.hip, sv_c64_adj.hip, sv_c128.hip
// and sv_prog.hip, which share sv_engine.h).
#include <hip/hip_runtime.h>

#include "qs_internal.h"

namespace qs {

int sv_c64_forward(const SvLaunch& L);
int sv_c64_adjoint(const SvLaunch& L);
int sv_c128_forward(const SvLaunch& L);
int sv_c128_adjoint(const SvLaunch& L);

namespace {

__global__ void zero_i32(int* p) { *p = 0; }

// (dtype, r, direction) -> the block-size bound of the instantiation. The
// bounds are chosen so that no instantiation spills registers to scratch.
int max_threads(int dtype, int r, bool adjoint) {
  if (dtype == QS_C64) {
    if (r <= 3) return 1024;
    if (r == 4) return adjoint ? 512 : 1024;
    return r == 5 ? 512 : 0;
  }
  if (r <= 3) return 1024;
  return r == 4 ? 512 : 0;
}

}  // namespace

int launch_zero_i32(int* p, void* stream) {
  hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, static_cast<hipStream_t>(stream), p);
  return hipGetLastError() == hipSuccess ? QS_OK : QS_ERR_LAUNCH;
}

int launch_sv_forward(int dtype, const SvLaunch& L) {
  return dtype == QS_C64 ? sv_c64_forward(L) : sv_c128_forward(L);
}
int launch_sv_adjoint(int dtype, const SvLaunch& L) {
  return dtype == QS_C64 ? sv_c64_adjoint(L) : sv_c128_adjoint(L);
}

// Largest block size each (dtype, r, direction) instantiation is compiled for.
int sv_max_threads(int dtype, int r, int adjoint) { return max_threads(dtype, r, adjoint != 0); }

}  // namespace qs
