// Forward sightline march (Sec. 2.3, Eqs. ji, jp, rm, chi, int).
//
// Work decomposition: a sightline is handled by S consecutive lanes of a
// wavefront (S = 1, 4, 16 or 64).  Lanes of a group take consecutive steps of
// the same sightline in chunks of S; the Faraday sum of Eq. rm is carried in
// FP64 from chunk to chunk and combined inside a chunk with a wavefront prefix
// scan.  Sightlines are enumerated in HEALPix NESTED order, so one wavefront
// covers a compact sky patch and its rays sample neighbouring grid cells; the
// result is written at the RING index.
#include "sm_device.h"
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
  const Ray ray = make_ray(g, q);

  double carry = 0.0;  // Faraday sum (n_e B_par, uG cm^-3) of all earlier chunks
  double accI = 0.0;
  double accQ[MF], accU[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) accQ[f] = accU[f] = 0.0;

  for (int c0 = 0; c0 < g.n_steps; c0 += S) {
    const int n = c0 + sub;
    const bool act = n < g.n_steps;
    const double s = ((double)n + 0.5) * ray.dkpc;  // midpoint of segment n
    const float x = (float)(g.r_obs[0] + s * ray.nx);
    const float y = (float)(g.r_obs[1] + s * ray.ny);
    const float z = (float)(g.r_obs[2] + s * ray.nz);
    const FV v = fld.eval(x, y, z);
    const float bl = v.bx * ray.elx + v.by * ray.ely;
    const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
    const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
    const double cn = act ? (double)v.ne * bpar : 0.0;
    double psi;  // Faraday sum at the midpoint: earlier segments + half of this one
    if constexpr (S == 1) {
      psi = carry + 0.5 * cn;
      carry += cn;
    } else {
      const double incl = group_inclusive_scan<S>(cn, sub);
      psi = carry + incl - 0.5 * cn;
      carry += group_bcast<S>(incl, S - 1);
    }
    Emit e = emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
    if (!act) e.u = e.zr = e.zi = 0.0f;
    accI += (double)e.u;
    const double psid = psi * ray.dkpc;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < fa.n_freq) {
        const double t = psid * fa.kappa[f];  // turns of 2 RM lambda^2
        const float fr = (float)(t - rint(t));
        float sn, cs;
        sincos_turns(fr, &sn, &cs);
        accQ[f] += (double)(e.zr * cs - e.zi * sn);
        accU[f] += (double)(e.zr * sn + e.zi * cs);
      }
    }
  }

  if constexpr (S > 1) {
    accI = group_sum<S>(accI);
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      accQ[f] = group_sum<S>(accQ[f]);
      accU[f] = group_sum<S>(accU[f]);
    }
  }
  if (valid && sub == 0) {
    const int64_t np = g.npix;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < fa.n_freq) {
        maps[(3 * f + 0) * np + ray.ring] = (float)(fa.sI[f] * ray.dkpc * accI);
        maps[(3 * f + 1) * np + ray.ring] = (float)(fa.sP[f] * ray.dkpc * accQ[f]);
        maps[(3 * f + 2) * np + ray.ring] = (float)(fa.sP[f] * ray.dkpc * accU[f]);
      }
    }
    if (phi_end != nullptr) phi_end[ray.ring] = carry;
  }
}

template <class F, int S>
static hipError_t fwd_mf(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         float* maps, double* phi_end, hipStream_t st) {
  const int64_t nb = march_blocks(g.npix, S);
  if (fa.n_freq <= 1)
    k_forward<F, S, 1><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, fa, ea, f, maps, phi_end);
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
    case kGrid: return fwd_s(g, fa, ea, Grid{fp.grid, Model16{fp.m16}}, S, maps, phi_end, st);
    case kSphere: return fwd_s(g, fa, ea, Sphere{fp.sph}, S, maps, phi_end, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sm
