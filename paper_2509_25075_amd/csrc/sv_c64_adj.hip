// complex64 adjoint instantiations of the register engine.
#include "sv_engine.h"

namespace qs {
namespace {
// The specialisation for the plan (shared angles only) and the launch's LDS
// staging mode.
template <int LR, int MAXT>
int launch_sel(const SvLaunch& L, bool shared) {
  // Plans whose every block is RY then RZ take the gate-at-a-time pass
  // (register tiles 2^4 and 2^5, the ones such plans are tuned to).
  if constexpr (LR >= 4) {
    if (L.p->ryrz) {
      if (L.shape.half)
        return shared ? launch_one<float, LR, MAXT, true, true, true, true>(L)
                      : launch_one<float, LR, MAXT, true, false, true, true>(L);
      return shared ? launch_one<float, LR, MAXT, true, true, false, true>(L)
                    : launch_one<float, LR, MAXT, true, false, false, true>(L);
    }
  }
  if (L.shape.half)
    return shared ? launch_one<float, LR, MAXT, true, true, true>(L)
                  : launch_one<float, LR, MAXT, true, false, true>(L);
  return shared ? launch_one<float, LR, MAXT, true, true, false>(L)
                : launch_one<float, LR, MAXT, true, false, false>(L);
}
}  // namespace

int sv_c64_adjoint(const SvLaunch& L) {
  // Plans whose blocks all have shared angles run without the per-sample
  // block code.
  const bool shared = L.p->n_fu == L.p->n_blocks;
  switch (L.shape.r) {
    case 1: return launch_sel<1, 1024>(L, shared);
    case 2: return launch_sel<2, 1024>(L, shared);
    case 3: return launch_sel<3, 1024>(L, shared);
    case 4: return launch_sel<4, 512>(L, shared);
    case 5: return launch_sel<5, 512>(L, shared);
    default: return QS_ERR_UNSUPPORTED;
  }
}

}  // namespace qs
