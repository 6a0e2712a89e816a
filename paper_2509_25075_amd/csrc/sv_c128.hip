// complex128 instantiations of the register engine (both directions).
#include "sv_engine.h"

namespace qs {
namespace {
// The specialisation for the plan: shared angles only (fused matrices and
// generator frames from LDS, no per-sample block code) or not.
template <int LR, int MAXT, bool ADJ>
int launch_sel(const SvLaunch& L) {
  const bool shared = L.p->n_fu == L.p->n_blocks;
  // Plans whose every block is RY then RZ: the adjoint's gate-at-a-time pass
  // (register tile 2^4).
  if constexpr (ADJ && LR == 4) {
    if (L.p->ryrz)
      return shared ? launch_one<double, LR, MAXT, ADJ, true, false, true>(L)
                    : launch_one<double, LR, MAXT, ADJ, false, false, true>(L);
  }
  return shared ? launch_one<double, LR, MAXT, ADJ, true>(L)
                : launch_one<double, LR, MAXT, ADJ, false>(L);
}
}  // namespace

int sv_c128_forward(const SvLaunch& L) {
  switch (L.shape.r) {
    case 1: return launch_sel<1, 1024, false>(L);
    case 2: return launch_sel<2, 1024, false>(L);
    case 3: return launch_sel<3, 1024, false>(L);
    case 4: return launch_sel<4, 512, false>(L);
    default: return QS_ERR_UNSUPPORTED;
  }
}

int sv_c128_adjoint(const SvLaunch& L) {
  switch (L.shape.r) {
    case 1: return launch_sel<1, 1024, true>(L);
    case 2: return launch_sel<2, 1024, true>(L);
    case 3: return launch_sel<3, 1024, true>(L);
    case 4: return launch_sel<4, 512, true>(L);
    default: return QS_ERR_UNSUPPORTED;
  }
}

}  // namespace qs
