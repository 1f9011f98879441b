// Coordinate-MLP field surrogate (placeholder until the MFMA kernel lands).
#include "../../include/synmarch.h"

extern "C" {

size_t syn_mlp_packed_bytes(void) { return 0; }

syn_status syn_mlp_pack(const float* fourier, const float* w_in, const float* b_in,
                        const float* w_h, const float* b_h, const float* w_out,
                        const float* b_out, void* packed_host) {
  (void)fourier; (void)w_in; (void)b_in; (void)w_h; (void)b_h; (void)w_out; (void)b_out;
  (void)packed_host;
  return SYN_EUNSUPPORTED;
}

}  // extern "C"
