// Forward sightline march (Sec. 2.3, Eqs. ji, jp, rm, chi, int).
//
// Work decomposition: a sightline is handled by S consecutive lanes of a
// wavefront (S = 1, 4, 16 or 64).  Lanes of a group take consecutive steps of
// the same sightline in chunks of S; the Faraday sum of Eq. rm is carried in
// FP64 from chunk to chunk and combined inside a chunk with a wavefront prefix
// scan.  Sightlines are enumerated in HEALPix NESTED order, so one wavefront
// covers a compact sky patch and its rays sample neighbouring grid cells; the
// result is written at the RING index.
#include "march_fwd_impl.h"

namespace sm {

hipError_t launch_forward(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                          const FieldPack& fp, int S, float* maps, double* phi_end,
                          double* em_end, hipStream_t st) {
  if (fp.grid.alpha != nullptr)
    return fp.ff ? launch_forward_va_ff(g, fa, ea, fp, S, maps, phi_end, em_end, st)
                 : launch_forward_va(g, fa, ea, fp, S, maps, phi_end, nullptr, st);
  if (fp.spec == kSpecBroken)
    return fp.ff ? launch_forward_bp_ff(g, fa, ea, fp, S, maps, phi_end, em_end, st)
                 : launch_forward_bp(g, fa, ea, fp, S, maps, phi_end, nullptr, st);
  if (fp.ff) return launch_forward_ff(g, fa, ea, fp, S, maps, phi_end, em_end, st);
  return launch_forward_t<false, kSpecPower>(g, fa, ea, fp, S, maps, phi_end, nullptr, st);
}

}  // namespace sm
