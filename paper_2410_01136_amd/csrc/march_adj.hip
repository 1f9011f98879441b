// Reverse pass of the sightline march.
//
// For L = sum(dmaps * maps) the kernel walks every sightline backwards.  The
// Faraday sum at each midpoint is rebuilt from the total stored by the forward
// pass (subtracting the recomputed increments), so no per-step state is kept;
// fields and emissivities are recomputed per step.  The cotangent of a
// Faraday increment is the suffix sum of the phase cotangents behind it (the
// transpose of the prefix sum of Eq. rm), taken with a wavefront suffix scan
// inside a chunk and an FP64 carry across chunks.
//
// Outputs: theta-gradients reduced per block in FP64 (fixed order, no atomics)
// and finished by a second kernel; grid gradients scattered with FP32 atomic
// adds onto the 8 corner nodes of each step's cell.
#include "march_adj_impl.h"

namespace sm {

hipError_t launch_adjoint(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                          const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                          const double* em_end, double* partials, double* dtheta, float* gbn,
                          float* gc, hipStream_t st) {
  if (fp.grid.alpha != nullptr)
    return fp.ff ? launch_adjoint_va_ff(g, fa, ea, fp, S, dmaps, phi_end, em_end, partials, dtheta,
                                        gbn, gc, st)
                 : launch_adjoint_va(g, fa, ea, fp, S, dmaps, phi_end, nullptr, partials, dtheta,
                                     gbn, gc, st);
  if (fp.spec == kSpecBroken)
    return fp.ff ? launch_adjoint_bp_ff(g, fa, ea, fp, S, dmaps, phi_end, em_end, partials, dtheta,
                                        gbn, gc, st)
                 : launch_adjoint_bp(g, fa, ea, fp, S, dmaps, phi_end, nullptr, partials, dtheta,
                                     gbn, gc, st);
  if (fp.ff)
    return launch_adjoint_ff(g, fa, ea, fp, S, dmaps, phi_end, em_end, partials, dtheta, gbn, gc,
                             st);
  return launch_adjoint_t<false, kSpecPower>(g, fa, ea, fp, S, dmaps, phi_end, nullptr, partials,
                                        dtheta, gbn, gc, st);
}

}  // namespace sm
