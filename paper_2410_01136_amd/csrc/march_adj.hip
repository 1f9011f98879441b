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
#include "sm_device.h"
#include "sm_launch.h"

namespace sm {

constexpr double kTwoPi = 6.283185307179586;

template <class F, int S, int MF, bool THETA, bool GRID>
__global__ __launch_bounds__(256) void k_adjoint(GeomArgs g, FreqArgs fa, EmitArgs ea, F fld,
                                                 const float* __restrict__ dmaps,
                                                 const double* __restrict__ phi_end,
                                                 double* __restrict__ partials, float* gbn,
                                                 float* gc) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t tid = blk * 256 + threadIdx.x;
  const int sub = (int)(threadIdx.x & (S - 1));
  int64_t q = tid / S;
  const bool valid = q < g.npix;
  if (!valid) q = g.npix - 1;
  const Ray ray = make_ray(g, q);
  const double dk = ray.dkpc;
  const int64_t np = g.npix;

  // per-sightline cotangent constants
  double GI = 0.0;
  double hr[MF], hi[MF], kr[MF], ki[MF], gi_f[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) {
    hr[f] = hi[f] = kr[f] = ki[f] = gi_f[f] = 0.0;
    if (f < fa.n_freq && valid) {
      const double dI = dmaps[(3 * f + 0) * np + ray.ring];
      const double dQ = dmaps[(3 * f + 1) * np + ray.ring];
      const double dU = dmaps[(3 * f + 2) * np + ray.ring];
      gi_f[f] = dI * fa.sI[f] * dk;
      GI += gi_f[f];
      hr[f] = fa.sP[f] * dk * dQ;  // h = conj(dQ + i dU) sP dk
      hi[f] = -fa.sP[f] * dk * dU;
      const double a = -kTwoPi * fa.kappa[f] * dk;  // d(phase turns)/d(sum) with the 2 pi i
      kr[f] = a * hr[f];
      ki[f] = a * hi[f];
    }
  }

  double E = valid ? phi_end[ray.ring] : 0.0;  // Faraday sum of all steps before the chunk end
  double suf = 0.0;                            // phase cotangents of all later chunks
  double tb[THETA ? kNParam : 1];
#pragma unroll
  for (int k = 0; k < (THETA ? kNParam : 1); ++k) tb[k] = 0.0;
  double accI = 0.0, accPr[MF], accPi[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) accPr[f] = accPi[f] = 0.0;

  const int nchunk = (g.n_steps + S - 1) / S;
  for (int ch = nchunk - 1; ch >= 0; --ch) {
    const int n = ch * S + sub;
    const bool act = valid && n < g.n_steps;
    const double s = ((double)n + 0.5) * dk;
    const float x = (float)(g.r_obs[0] + s * ray.nx);
    const float y = (float)(g.r_obs[1] + s * ray.ny);
    const float z = (float)(g.r_obs[2] + s * ray.nz);
    const FV v = fld.eval(x, y, z);
    const float bl = v.bx * ray.elx + v.by * ray.ely;
    const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
    const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
    const double cn = (n < g.n_steps) ? (double)v.ne * bpar : 0.0;
    double psi;
    if constexpr (S == 1) {
      E -= cn;
      psi = E + 0.5 * cn;
    } else {
      const double incl = group_inclusive_scan<S>(cn, sub);
      const double tot = group_bcast<S>(incl, S - 1);
      psi = E - tot + incl - 0.5 * cn;
      E -= tot;
    }
    Emit e = emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
    if (!act) e.u = e.zr = e.zi = 0.0f;
    // H = sum_f h_f e^{2 pi i t_f};  K = sum_f k_f e^{2 pi i t_f}
    double Hr = 0.0, Hi = 0.0, Kr = 0.0, Ki = 0.0;
    const double psid = psi * dk;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < fa.n_freq) {
        const double t = psid * fa.kappa[f];
        const float fr = (float)(t - rint(t));
        float sn, cs;
        sincos_turns(fr, &sn, &cs);
        Hr += hr[f] * cs - hi[f] * sn;
        Hi += hr[f] * sn + hi[f] * cs;
        Kr += kr[f] * cs - ki[f] * sn;
        Ki += kr[f] * sn + ki[f] * cs;
        if constexpr (THETA) {
          accPr[f] += (double)(e.zr * cs - e.zi * sn);
          accPi[f] += (double)(e.zr * sn + e.zi * cs);
        }
      }
    }
    if constexpr (THETA) accI += (double)e.u;
    // cotangent of the Faraday sum at this midpoint: Im(zc K)
    const double pb = (double)e.zr * Ki + (double)e.zi * Kr;
    double cbar;  // cotangent of this step's increment: later steps + half of its own
    if constexpr (S == 1) {
      cbar = suf + 0.5 * pb;
      suf += pb;
    } else {
      const double sincl = group_suffix_scan<S>(pb, sub);
      const double stot = group_bcast<S>(sincl, 0);
      cbar = suf + sincl - 0.5 * pb;
      suf += stot;
    }
    // local reverse of the emission and projections
    const EmitBar eb = emission_vjp(v.n0, bl, bb, ea.alpha3 != 0, ea.eI, (float)GI, (float)Hr,
                                    (float)(-Hi));
    const float neb = (float)(cbar * bpar);
    const float bparb = (float)(cbar * (double)v.ne);
    FV gv;
    gv.bx = eb.bl * ray.elx + eb.bb * ray.ebx - bparb * (float)ray.nx;
    gv.by = eb.bl * ray.ely + eb.bb * ray.eby - bparb * (float)ray.ny;
    gv.bz = eb.bb * ray.ebz - bparb * (float)ray.nz;
    gv.ne = neb;
    gv.n0 = eb.n0;
    if (act) {
      if constexpr (THETA) {
        fld.vjp(x, y, z, gv, tb);
        tb[12] += (double)eb.alpha;
      }
      if constexpr (GRID) fld.scatter(x, y, z, gv, gbn, gc);
    }
  }

  if constexpr (THETA) {
    // alpha also enters the per-frequency prefactors: d ln s / d alpha * (this lane's share)
#pragma unroll
    for (int f = 0; f < MF; ++f)
      if (f < fa.n_freq)
        tb[12] += fa.dlnsI[f] * gi_f[f] * accI + fa.dlnsP[f] * (hr[f] * accPr[f] - hi[f] * accPi[f]);
    // block reduction in a fixed order: wavefront butterfly, then the 4 waves
    __shared__ double red[4][kNParam];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNParam; ++k) {
      double v = tb[k];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
      if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNParam) {
      const int k = threadIdx.x;
      partials[blk * kNParam + k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
  }
}

// Sums the per-block partials in a fixed order: 16 strided lanes per
// parameter, then a fixed tree.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partials,
                                                         int64_t nblk, double* __restrict__ out) {
  __shared__ double red[16][17];
  const int k = threadIdx.x & 15, j = threadIdx.x >> 4;
  double acc = 0.0;
  for (int64_t b = j; b < nblk; b += 16) acc += partials[b * kNParam + k];
  red[j][k] = acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    double s = 0.0;
    for (int jj = 0; jj < 16; ++jj) s += red[jj][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

template <class F, int S, int MF, bool TH, bool GR>
static hipError_t adj_go(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         const float* dm, const double* pe, double* part, double* dth, float* gbn,
                         float* gc, hipStream_t st) {
  const int64_t nb = march_blocks(g.npix, S);
  k_adjoint<F, S, MF, TH, GR><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, fa, ea, f, dm, pe, part,
                                                                         gbn, gc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (TH) {
    k_reduce_partials<<<dim3(1), dim3(256), 0, st>>>(part, nb, dth);
    e = hipGetLastError();
  }
  return e;
}

template <class F, int S, int MF>
static hipError_t adj_flags(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                            const float* dm, const double* pe, double* part, double* dth,
                            float* gbn, float* gc, hipStream_t st) {
  const bool th = dth != nullptr, gr = (gbn != nullptr || gc != nullptr);
  if (th && gr) return adj_go<F, S, MF, true, true>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
  if (th) return adj_go<F, S, MF, true, false>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
  if (gr) return adj_go<F, S, MF, false, true>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
  return hipSuccess;
}

template <class F, int S>
static hipError_t adj_mf(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         const float* dm, const double* pe, double* part, double* dth, float* gbn,
                         float* gc, hipStream_t st) {
  if (fa.n_freq <= 1) return adj_flags<F, S, 1>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
  if (fa.n_freq <= 4) return adj_flags<F, S, 4>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
  return adj_flags<F, S, 16>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
}

template <class F>
static hipError_t adj_s(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                        int S, const float* dm, const double* pe, double* part, double* dth,
                        float* gbn, float* gc, hipStream_t st) {
  switch (S) {
    case 1: return adj_mf<F, 1>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
    case 4: return adj_mf<F, 4>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
    case 16: return adj_mf<F, 16>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
    case 64: return adj_mf<F, 64>(g, fa, ea, f, dm, pe, part, dth, gbn, gc, st);
    default: return hipErrorInvalidValue;
  }
}

// Model16 fields have no grid to scatter into.
struct Model16NoGrid : Model16 {
  __device__ inline void scatter(float, float, float, const FV&, float*, float*) const {}
};

hipError_t launch_adjoint(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                          const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                          double* partials, double* dtheta, float* gbn, float* gc,
                          hipStream_t st) {
  switch (fp.kind) {
    case kModel16:
      return adj_s(g, fa, ea, Model16NoGrid{Model16{fp.m16}}, S, dmaps, phi_end, partials, dtheta,
                   nullptr, nullptr, st);
    case kGrid:
      return adj_s(g, fa, ea, Grid{fp.grid, Model16{fp.m16}}, S, dmaps, phi_end, partials, dtheta,
                   gbn, gc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sm
