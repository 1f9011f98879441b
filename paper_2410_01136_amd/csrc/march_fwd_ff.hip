// Forward march with free-free emission and absorption (see fwd_lane).
#include "march_fwd_impl.h"

namespace sm {

hipError_t launch_forward_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, float* maps, double* phi_end,
                             double* em_end, hipStream_t st) {
  return launch_forward_t<true, kSpecPower>(g, fa, ea, fp, S, maps, phi_end, em_end, st);
}

}  // namespace sm
