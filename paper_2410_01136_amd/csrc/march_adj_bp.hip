// Reverse march with a broken power-law CR spectrum (see adj_lane).
#include "march_adj_impl.h"

namespace sm {

hipError_t launch_adjoint_bp(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                             const double* em_end, double* partials, double* dtheta, float* gbn,
                             float* gc, hipStream_t st) {
  return launch_adjoint_t<false, kSpecBroken>(g, fa, ea, fp, S, dmaps, phi_end, em_end, partials,
                                              dtheta, gbn, gc, st);
}

}  // namespace sm
