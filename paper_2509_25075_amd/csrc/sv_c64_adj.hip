// complex64 adjoint instantiations of the register engine.
#include "sv_engine.h"

namespace qs {

int sv_c64_adjoint(const SvLaunch& L) {
  switch (L.shape.r) {
    case 1: return launch_one<float, 1, 1024, true>(L);
    case 2: return launch_one<float, 2, 1024, true>(L);
    case 3: return launch_one<float, 3, 1024, true>(L);
    case 4: return launch_one<float, 4, 512, true>(L);
    case 5: return launch_one<float, 5, 512, true>(L);
    default: return QS_ERR_UNSUPPORTED;
  }
}

}  // namespace qs
