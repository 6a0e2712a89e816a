// complex64 forward instantiations of the register engine.
#include "sv_engine.h"

namespace qs {

int sv_c64_forward(const SvLaunch& L) {
  // Plans whose blocks all have shared angles run without the per-sample
  // block code.
  const bool shared = L.p->n_fu == L.p->n_blocks;
  switch (L.shape.r) {
    case 1: return shared ? launch_one<float, 1, 1024, false, true>(L)
                     : launch_one<float, 1, 1024, false, false>(L);
    case 2: return shared ? launch_one<float, 2, 1024, false, true>(L)
                     : launch_one<float, 2, 1024, false, false>(L);
    case 3: return shared ? launch_one<float, 3, 1024, false, true>(L)
                     : launch_one<float, 3, 1024, false, false>(L);
    case 4: return shared ? launch_one<float, 4, 1024, false, true>(L)
                     : launch_one<float, 4, 1024, false, false>(L);
    case 5: return shared ? launch_one<float, 5, 512, false, true>(L)
                     : launch_one<float, 5, 512, false, false>(L);
    default: return QS_ERR_UNSUPPORTED;
  }
}

}  // namespace qs
