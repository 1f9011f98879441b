// Forward march with a broken power-law CR spectrum and free-free (see fwd_lane).
#include "march_fwd_impl.h"

namespace sm {

hipError_t launch_forward_bp_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                const FieldPack& fp, int S, float* maps, double* phi_end,
                                double* em_end, hipStream_t st) {
  return launch_forward_t<true, kSpecBroken>(g, fa, ea, fp, S, maps, phi_end, em_end, st);
}

}  // namespace sm
