// Host/device interface of the many-set kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sm_params.h"

namespace sm {

struct FreqArgs1 {
  int32_t n_freq;
  double sI[1], sP[1], kappa[1], dlnsI[1], dlnsP[1];
};

struct BatchSet {
  GeomArgs g;
  FreqArgs1 fa;
  EmitArgs ea;
  M16Args m;         // field of a MODEL16 plan
  WmapArgs w;        // field of a WMAP plan
  int64_t map_off;   // ragged offset of this set's pixel 0
  int32_t item0;     // first work item of this set
  int32_t n_items;
};

struct BatchChi2Args {
  double inv_s2[3];
};

struct BatchLaunch {
  int S;
  bool wmap;             // the sets' field: WMAP (true) or MODEL16
  const BatchSet* sets;  // device
  int n_sets, n_items;
  int64_t total;
  unsigned int* counters;  // device, 2 work counters
  double* phi;             // device, [total]
  double* partials;        // device, [n_items][16]
  int blocks_fwd, blocks_adj;
  const float* target;
  BatchChi2Args chi2_args;
  float* maps;
  float* dmaps;
  double* chi2;
  double* dtheta;
};

hipError_t launch_batch(const BatchLaunch& L, hipStream_t st);
int batch_blocks_per_cu(int S, bool adjoint, bool wmap);

}  // namespace sm
