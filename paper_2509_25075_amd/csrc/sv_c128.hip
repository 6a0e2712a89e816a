// complex128 instantiations of the register engine (both directions).
#include "sv_engine.h"

namespace qs {

int sv_c128_forward(const SvLaunch& L) {
  switch (L.shape.r) {
    case 1: return launch_one<double, 1, 1024, false>(L);
    case 2: return launch_one<double, 2, 1024, false>(L);
    case 3: return launch_one<double, 3, 1024, false>(L);
    case 4: return launch_one<double, 4, 512, false>(L);
    default: return QS_ERR_UNSUPPORTED;
  }
}

int sv_c128_adjoint(const SvLaunch& L) {
  switch (L.shape.r) {
    case 1: return launch_one<double, 1, 1024, true>(L);
    case 2: return launch_one<double, 2, 1024, true>(L);
    case 3: return launch_one<double, 3, 1024, true>(L);
    case 4: return launch_one<double, 4, 512, true>(L);
    default: return QS_ERR_UNSUPPORTED;
  }
}

}  // namespace qs
