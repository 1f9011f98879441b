// Forward march kernels and their launch-shape dispatch, templated on free-free
// (FF) and the spectral model (SP).  Included by one march_fwd*.hip file per
// (FF, SP) pair so that the sets of kernels compile in parallel.
#pragma once

#include <type_traits>

#include "march_body.h"
#include "sm_launch.h"

namespace sm {

// PC: also store the piece snapshots (snap_args; grid, spiral-disk and WMAP fields).
template <class F, int S, int MF, bool FF, int SP, bool PC = false>
__global__ __launch_bounds__(256) void k_forward(GeomArgs g, FreqArgs fa, EmitArgs ea, F fld,
                                                 float* __restrict__ maps,
                                                 double* __restrict__ phi_end,
                                                 double* __restrict__ em_end) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t tid = blk * 256 + threadIdx.x;
  const int sub = (int)(threadIdx.x & (S - 1));
  int64_t q = tid / S;
  const bool valid = q < g.npix;
  if (!valid) q = g.npix - 1;  // idle lanes march a real sightline, results dropped
  fwd_lane<F, S, MF, FF, SP, PC>(g, fa, ea, fld, q, sub, valid, maps, MapAddr{g.npix, 0},
                                 phi_end, em_end);
}

template <bool FF, int SP, bool PC, class F, int S>
static hipError_t fwd_mf_pc(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                            float* maps, double* phi_end, double* em_end, hipStream_t st) {
  const int64_t nb = march_blocks(g.npix, S);
  const dim3 grid((unsigned)nb), block(256);
  if (fa.n_freq <= 1)
    k_forward<F, S, 1, FF, SP, PC><<<grid, block, 0, st>>>(g, fa, ea, f, maps, phi_end, em_end);
  else if (std::is_same_v<F, GridL> && fa.n_freq == 3)  // the three-frequency gridded maps
    k_forward<F, S, 3, FF, SP, PC><<<grid, block, 0, st>>>(g, fa, ea, f, maps, phi_end, em_end);
  else if (fa.n_freq <= 4)
    k_forward<F, S, 4, FF, SP, PC><<<grid, block, 0, st>>>(g, fa, ea, f, maps, phi_end, em_end);
  else
    k_forward<F, S, 16, FF, SP, PC><<<grid, block, 0, st>>>(g, fa, ea, f, maps, phi_end, em_end);
  return hipGetLastError();
}

// grid, spiral-disk and WMAP fields write piece snapshots when asked to
// (snap_args(fld).snap set)
template <bool FF, int SP, class F, int S>
static hipError_t fwd_mf(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         float* maps, double* phi_end, double* em_end, hipStream_t st) {
  if constexpr (kHasSnapshots<F>) {
    if (snap_args(f).snap != nullptr) return fwd_mf_pc<FF, SP, true, F, S>(g, fa, ea, f, maps, phi_end, em_end, st);
  }
  return fwd_mf_pc<FF, SP, false, F, S>(g, fa, ea, f, maps, phi_end, em_end, st);
}

template <bool FF, int SP, class F>
static hipError_t fwd_s(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                        int S, float* maps, double* phi_end, double* em_end, hipStream_t st) {
  switch (S) {
    case 1: return fwd_mf<FF, SP, F, 1>(g, fa, ea, f, maps, phi_end, em_end, st);
    case 4: return fwd_mf<FF, SP, F, 4>(g, fa, ea, f, maps, phi_end, em_end, st);
    case 8: return fwd_mf<FF, SP, F, 8>(g, fa, ea, f, maps, phi_end, em_end, st);
    case 16: return fwd_mf<FF, SP, F, 16>(g, fa, ea, f, maps, phi_end, em_end, st);
    case 64: return fwd_mf<FF, SP, F, 64>(g, fa, ea, f, maps, phi_end, em_end, st);
    default: return hipErrorInvalidValue;
  }
}

// SP: spectral model (kSpecPower, kSpecGridAlpha: gridded index, grid fields
// only; kSpecBroken: broken power law).
template <bool FF, int SP>
static hipError_t launch_forward_t(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                   const FieldPack& fp, int S, float* maps, double* phi_end,
                                   double* em_end, hipStream_t st) {
  if (fp.kind == kGrid) {
    if (fp.grid_path == kGridShared)
      return fwd_s<FF, SP>(g, fa, ea, GridL{fp.grid, Model16{fp.m16}}, S, maps, phi_end, em_end, st);
    if (fp.grid_path != kGridGlobal)
      return fwd_s<FF, SP>(g, fa, ea, GridB{fp.grid, Model16{fp.m16}}, S, maps, phi_end, em_end, st);
    return fwd_s<FF, SP>(g, fa, ea, Grid{fp.grid, Model16{fp.m16}}, S, maps, phi_end, em_end, st);
  }
  if constexpr (SP != kSpecGridAlpha) {
    switch (fp.kind) {
      case kModel16: return fwd_s<FF, SP>(g, fa, ea, Model16{fp.m16, fp.snap}, S, maps, phi_end, em_end, st);
      case kSphere: return fwd_s<FF, SP>(g, fa, ea, Sphere{fp.sph}, S, maps, phi_end, em_end, st);
      case kWmap: return fwd_s<FF, SP>(g, fa, ea, Wmap{fp.wmap, fp.snap}, S, maps, phi_end, em_end, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace sm
