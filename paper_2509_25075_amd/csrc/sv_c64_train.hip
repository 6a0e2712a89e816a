// complex64 training-step instantiations of the register engine: forward,
// readout, MSE loss and adjoint in one launch (register tiles 2^4 and 2^5,
// whole-amplitude staging).
#include "sv_engine.h"

namespace qs {
namespace {
template <int LR>
int launch_sel(const SvLaunch& L) {
  const bool shared = L.p->n_fu == L.p->n_blocks;
  if (L.p->ryrz)
    return shared ? launch_one<float, LR, 512, true, true, false, true, true>(L)
                  : launch_one<float, LR, 512, true, false, false, true, true>(L);
  return shared ? launch_one<float, LR, 512, true, true, false, false, true>(L)
                : launch_one<float, LR, 512, true, false, false, false, true>(L);
}
}  // namespace

bool sv_train_supported(int dtype, const SvShape& shape) {
  return dtype == QS_C64 && shape.half == 0 && (shape.r == 4 || shape.r == 5) &&
         shape.block_threads <= 512;
}

int launch_sv_train(int dtype, const SvLaunch& L) {
  if (!sv_train_supported(dtype, L.shape)) return QS_ERR_UNSUPPORTED;
  return L.shape.r == 4 ? launch_sel<4>(L) : launch_sel<5>(L);
}

}  // namespace qs
