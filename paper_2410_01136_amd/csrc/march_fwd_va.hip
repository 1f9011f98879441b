// Forward march with a gridded CR spectral index (see fwd_lane).
#include "march_fwd_impl.h"

namespace sm {

hipError_t launch_forward_va(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, float* maps, double* phi_end,
                             double* em_end, hipStream_t st) {
  return launch_forward_t<false, kSpecGridAlpha>(g, fa, ea, fp, S, maps, phi_end, em_end, st);
}

}  // namespace sm
