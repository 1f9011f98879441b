// Forward sightline march (Sec. 2.3, Eqs. ji, jp, rm, chi, int).
//
// Work decomposition: a sightline is handled by S consecutive lanes of a
// wavefront (S = 1, 4, 16 or 64).  Lanes of a group take consecutive steps of
// the same sightline in chunks of S; the Faraday sum of Eq. rm is carried in
// FP64 from chunk to chunk and combined inside a chunk with a wavefront prefix
// scan.  Sightlines are enumerated in HEALPix NESTED order, so one wavefront
// covers a compact sky patch and its rays sample neighbouring grid cells; the
// result is written at the RING index.
#include "march_body.h"
#include "sm_launch.h"

namespace sm {

template <class F, int S, int MF>
__global__ __launch_bounds__(256) void k_forward(GeomArgs g, FreqArgs fa, EmitArgs ea, F fld,
                                                 float* __restrict__ maps,
                                                 double* __restrict__ phi_end) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t tid = blk * 256 + threadIdx.x;
  const int sub = (int)(threadIdx.x & (S - 1));
  int64_t q = tid / S;
  const bool valid = q < g.npix;
  if (!valid) q = g.npix - 1;  // idle lanes march a real sightline, results dropped
  fwd_lane<F, S, MF>(g, fa, ea, fld, q, sub, valid, maps, MapAddr{g.npix, 0}, phi_end);
}

template <class F, int S>
static hipError_t fwd_mf(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         float* maps, double* phi_end, hipStream_t st) {
  const int64_t nb = march_blocks(g.npix, S);
  if (fa.n_freq <= 1)
    k_forward<F, S, 1><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, fa, ea, f, maps, phi_end);
  else if (std::is_same_v<F, GridL> && fa.n_freq == 3)  // the three-frequency gridded maps
    k_forward<F, S, 3><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, fa, ea, f, maps, phi_end);
  else if (fa.n_freq <= 4)
    k_forward<F, S, 4><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, fa, ea, f, maps, phi_end);
  else
    k_forward<F, S, 16><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, fa, ea, f, maps, phi_end);
  return hipGetLastError();
}

template <class F>
static hipError_t fwd_s(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                        int S, float* maps, double* phi_end, hipStream_t st) {
  switch (S) {
    case 1: return fwd_mf<F, 1>(g, fa, ea, f, maps, phi_end, st);
    case 4: return fwd_mf<F, 4>(g, fa, ea, f, maps, phi_end, st);
    case 16: return fwd_mf<F, 16>(g, fa, ea, f, maps, phi_end, st);
    case 64: return fwd_mf<F, 64>(g, fa, ea, f, maps, phi_end, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_forward(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                          const FieldPack& fp, int S, float* maps, double* phi_end,
                          hipStream_t st) {
  switch (fp.kind) {
    case kModel16: return fwd_s(g, fa, ea, Model16{fp.m16}, S, maps, phi_end, st);
    case kGrid:
      if (fp.grid_path == kGridShared)
        return fwd_s(g, fa, ea, GridL{fp.grid, Model16{fp.m16}}, S, maps, phi_end, st);
      if (fp.grid_path == kGridBuffer)
        return fwd_s(g, fa, ea, GridB{fp.grid, Model16{fp.m16}}, S, maps, phi_end, st);
      return fwd_s(g, fa, ea, Grid{fp.grid, Model16{fp.m16}}, S, maps, phi_end, st);
    case kSphere: return fwd_s(g, fa, ea, Sphere{fp.sph}, S, maps, phi_end, st);
    case kWmap: return fwd_s(g, fa, ea, Wmap{fp.wmap}, S, maps, phi_end, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sm
