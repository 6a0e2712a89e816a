// Persistent uneven-batch instantiations of the register engine.
#include "sv_engine.h"

namespace qs {

// `half`: the LDS stages one state component at a time (for programs whose
// largest class does not fit otherwise).
int launch_program(int dtype, const ProgLaunch& L, bool adjoint) {
  if (L.block != 512) return QS_ERR_UNSUPPORTED;
  if (dtype == QS_C64) {
    if (L.r == 5)
      return L.half ? launch_prog<float, 5, 512, true>(L, adjoint)
                    : launch_prog<float, 5, 512, false>(L, adjoint);
    if (L.r == 4)
      return L.half ? launch_prog<float, 4, 512, true>(L, adjoint)
                    : launch_prog<float, 4, 512, false>(L, adjoint);
    return QS_ERR_UNSUPPORTED;
  }
  if (L.r == 4)
    return L.half ? launch_prog<double, 4, 512, true>(L, adjoint)
                  : launch_prog<double, 4, 512, false>(L, adjoint);
  return QS_ERR_UNSUPPORTED;
}

}  // namespace qs
