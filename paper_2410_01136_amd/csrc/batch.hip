// Many MODEL16 parameter sets in one persistent launch (placeholder until the
// persistent kernels land).
#include <stdlib.h>

#include "../../include/synmarch.h"

struct syn_batch {
  int dummy;
};

extern "C" {

syn_status syn_batch_create(const syn_batch_desc* desc, syn_batch** plan) {
  (void)desc;
  if (plan) *plan = nullptr;
  return SYN_EUNSUPPORTED;
}

int64_t syn_batch_total_pixels(const syn_batch* plan) {
  (void)plan;
  return 0;
}

int64_t syn_batch_offset(const syn_batch* plan, int32_t set) {
  (void)plan;
  (void)set;
  return -1;
}

syn_status syn_batch_run(syn_batch* plan, const float* target, const double* inv_sigma2,
                         float* maps, float* dmaps, double* chi2, double* dtheta,
                         hipStream_t stream) {
  (void)plan; (void)target; (void)inv_sigma2; (void)maps; (void)dmaps; (void)chi2; (void)dtheta;
  (void)stream;
  return SYN_EUNSUPPORTED;
}

void syn_batch_destroy(syn_batch* plan) { free(plan); }

}  // extern "C"
