// Per-lane bodies of the forward and reverse sightline march, shared by the
// one-map kernels and the persistent many-set kernels.
//
// A sightline is owned by S consecutive lanes (S = 1, 4, 16, 64).  Lanes take
// consecutive steps in chunks of S; the Faraday increments of a chunk are
// combined with a wavefront prefix scan and carried across chunks in FP64.
// (The reverse march with a grid gradient splits the steps into contiguous
// pieces instead; see adj_lane.)
// Every lane of a group must call these bodies (the scans are collective);
// idle lanes pass valid = false and march a real sightline with their
// results dropped.
#pragma once

#include <type_traits>

#include "sm_device.h"

namespace sm {

constexpr double kTwoPi = 6.283185307179586;

// Map addressing: element (f, stokes, ring) of a map set sits at
// map[(3 f + stokes) * stride + off + ring].
struct MapAddr {
  int64_t stride, off;
  __device__ inline int64_t at(int f, int k, int64_t ring) const {
    return (3 * f + k) * stride + off + ring;
  }
};

// Forward march of NESTED pixel q.  FA provides n_freq, sI[], sP[], kappa[].
// Whether a field type returns zero fields (hence zero emission and Faraday
// increment) for the steps past the end of the path, so the march need not
// mask them.
template <class F, class = void>
struct ZeroBeyondPath : std::false_type {};
template <class F>
struct ZeroBeyondPath<F, std::void_t<decltype(F::kZeroBeyondPath)>>
    : std::bool_constant<F::kZeroBeyondPath> {};
template <class F>
constexpr bool zero_beyond_path() {
  return ZeroBeyondPath<F>::value;
}

// MF frequencies held in registers: 1 and 3 are exact counts (the frequency
// loops need no test), 4 and 16 upper bounds.
constexpr bool exact_freqs(int MF) { return MF == 1 || MF == 3; }

template <class F, int S, int MF, class FA>
__device__ inline void fwd_lane(const GeomArgs& g, const FA& fa, const EmitArgs& ea, const F& fld,
                                int64_t q, int sub, bool valid, float* __restrict__ maps,
                                MapAddr ma, double* __restrict__ phi_end) {
  const Ray ray = make_ray(g, q);
  const auto rctx = fld.ray_ctx(g, ray);
  constexpr bool zero_beyond = zero_beyond_path<F>();
  double carry = 0.0;  // Faraday sum (n_e B_par, uG cm^-3) of all earlier chunks
  double accI = 0.0;
  double accQ[MF], accU[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) accQ[f] = accU[f] = 0.0;

  for (int c0 = 0; c0 < g.n_steps; c0 += S) {
    const int n = c0 + sub;
    const bool act = n < g.n_steps;
    const double s = ((double)n + 0.5) * ray.dkpc;  // midpoint of segment n
    const FV v = fld.template eval_step<S>(g, ray, rctx, s, n);
    const float bl = v.bx * ray.elx + v.by * ray.ely;
    const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
    const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
    const double cn = (zero_beyond || act) ? (double)v.ne * bpar : 0.0;
    double psi;  // Faraday sum at the midpoint: earlier segments + half of this one
    if constexpr (S == 1) {
      psi = carry + 0.5 * cn;
      carry += cn;
    } else {
      const double incl = group_inclusive_scan<S>(cn, sub);
      psi = carry + incl - 0.5 * cn;
      carry += group_last<S>(incl);
    }
    Emit e = emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
    if (!zero_beyond && !act) e.u = e.zr = e.zi = 0.0f;
    accI += (double)e.u;
    const double psid = psi * ray.dkpc;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (exact_freqs(MF) || f < fa.n_freq) {
        float sn, cs;
        sincos_turns(psid * fa.kappa[f], &sn, &cs);  // turns of 2 RM lambda^2
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
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (exact_freqs(MF) || f < fa.n_freq) {
        maps[ma.at(f, 0, ray.ring)] = (float)(fa.sI[f] * ray.dkpc * accI);
        maps[ma.at(f, 1, ray.ring)] = (float)(fa.sP[f] * ray.dkpc * accQ[f]);
        maps[ma.at(f, 2, ray.ring)] = (float)(fa.sP[f] * ray.dkpc * accU[f]);
      }
    }
    if (phi_end != nullptr) phi_end[ma.off + ray.ring] = carry;
  }
}

// Reverse march of NESTED pixel q for L = sum(dmaps * maps).  Adds this
// lane's share of dL/dtheta into tb (THETA) and scatters grid gradients
// (GRID).  FA additionally provides dlnsI[], dlnsP[].
//
// With a grid gradient and S > 1 the S lanes of a sightline do not interleave
// steps: lane k walks its own contiguous piece of ceil(N / S) steps, so that it
// stays in one cell for as many steps as a single lane would and its register
// accumulator flushes as rarely.  The piece needs two numbers from the pieces
// beyond it: the Faraday sum before its end, and the sum of the phase
// cotangents after it.  A pre-pass over the piece gets both with one march:
// the Faraday sum of the piece, and per frequency the sum of z_n e^{2 pi i t_n}
// with t_n counted from the piece start; once a group scan has given the
// Faraday sum of the earlier pieces, a rotation by its phase turns the latter
// into the piece's phase-cotangent total, and a suffix scan gives each piece
// those of the pieces after it.
template <class F, int S, int MF, bool THETA, bool GRID, class FA>
__device__ inline void adj_lane(const GeomArgs& g, const FA& fa, const EmitArgs& ea, const F& fld,
                                int64_t q, int sub, bool valid, const float* __restrict__ dmaps,
                                MapAddr ma, const double* __restrict__ phi_end, double* tb,
                                float* gbn, float* gc, const AdjBox* lds_box = nullptr,
                                float* lds_stage = nullptr) {
  const Ray ray = make_ray(g, q);
  const double dk = ray.dkpc;

  // per-sightline cotangent constants
  double GI = 0.0;
  double hr[MF], hi[MF], kr[MF], ki[MF], gi_f[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) {
    hr[f] = hi[f] = kr[f] = ki[f] = gi_f[f] = 0.0;
    if (f < fa.n_freq && valid) {
      const double dI = dmaps[ma.at(f, 0, ray.ring)];
      const double dQ = dmaps[ma.at(f, 1, ray.ring)];
      const double dU = dmaps[ma.at(f, 2, ray.ring)];
      gi_f[f] = dI * fa.sI[f] * dk;
      GI += gi_f[f];
      hr[f] = fa.sP[f] * dk * dQ;  // h = conj(dQ + i dU) sP dk
      hi[f] = -fa.sP[f] * dk * dU;
      const double a = -kTwoPi * fa.kappa[f] * dk;  // d(phase)/d(Faraday sum), with the 2 pi i
      kr[f] = a * hr[f];
      ki[f] = a * hi[f];
    }
  }

  typename F::Acc acc;  // grid-gradient accumulator
  if constexpr (GRID) {
    acc.box = *lds_box;
    acc.stage = lds_stage;
  }
  // each lane walks a contiguous run [n_lo, n_hi) of steps (one lane per
  // sightline, or one piece of it) rather than every S-th step
  constexpr bool SPLIT = GRID && S > 1;
  constexpr bool SERIAL = S == 1 || SPLIT;
  int n_lo = 0, n_hi = g.n_steps;
  double E = 0.0;    // Faraday sum over the steps before the current chunk's end
  double suf = 0.0;  // phase cotangents of the steps after it
  if constexpr (SPLIT) {
    const int len = (g.n_steps + S - 1) / S;
    n_lo = min(sub * len, g.n_steps);
    n_hi = min(n_lo + len, g.n_steps);
    double A = 0.0, Wr[MF], Wi[MF];
#pragma unroll
    for (int f = 0; f < MF; ++f) Wr[f] = Wi[f] = 0.0;
    for (int n = n_lo; n < n_hi; ++n) {
      const FV v = fld.eval_at(g, ray, ((double)n + 0.5) * dk);
      const float bl = v.bx * ray.elx + v.by * ray.ely;
      const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
      const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
      const double cn = (double)v.ne * bpar;
      const double psid = (A + 0.5 * cn) * dk;  // Faraday sum from the piece start
      A += cn;
      const Emit e = emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < fa.n_freq) {
          float sn, cs;
          sincos_turns(psid * fa.kappa[f], &sn, &cs);
          Wr[f] += (double)(e.zr * cs - e.zi * sn);
          Wi[f] += (double)(e.zr * sn + e.zi * cs);
        }
      }
    }
    const double incl = group_inclusive_scan<S>(A, sub);
    const double psid0 = (incl - A) * dk;  // Faraday sum of the earlier pieces
    double Bk = 0.0;                       // sum of this piece's phase cotangents
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < fa.n_freq) {
        float sn, cs;
        sincos_turns(psid0 * fa.kappa[f], &sn, &cs);
        const double rr = kr[f] * cs - ki[f] * sn, ri = kr[f] * sn + ki[f] * cs;
        Bk += rr * Wi[f] + ri * Wr[f];  // Im(k e^{2 pi i t0} W)
      }
    }
    E = incl;
    suf = group_suffix_scan<S>(Bk, sub) - Bk;
  } else if (valid) {
    E = phi_end[ma.off + ray.ring];
  }
  double accI = 0.0, accPr[MF], accPi[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) accPr[f] = accPi[f] = 0.0;

  // every lane of a wavefront runs the same number of iterations (the grid
  // scatter is collective); a short or empty last piece idles through the rest
  const int n_iter = SPLIT ? (g.n_steps + S - 1) / S : SERIAL ? g.n_steps : (g.n_steps + S - 1) / S;
  for (int it = n_iter - 1; it >= 0; --it) {
    const int n = SERIAL ? n_lo + it : it * S + sub;
    const bool act = valid && n < n_hi;
    const double s = ((double)n + 0.5) * dk;
    const FV v = fld.eval_at(g, ray, s);
    const float bl = v.bx * ray.elx + v.by * ray.ely;
    const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
    const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
    const double cn = (n < n_hi) ? (double)v.ne * bpar : 0.0;
    double psi;
    if constexpr (SERIAL) {
      E -= cn;
      psi = E + 0.5 * cn;
    } else {
      const double incl = group_inclusive_scan<S>(cn, sub);
      const double tot = group_last<S>(incl);
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
        float sn, cs;
        sincos_turns(psid * fa.kappa[f], &sn, &cs);
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
    if constexpr (SERIAL) {
      cbar = suf + 0.5 * pb;
      suf += pb;
    } else {
      const double sincl = group_suffix_scan<S>(pb, sub);
      const double stot = group_first<S>(sincl);
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
    if constexpr (THETA) {
      if (act) {
        fld.vjp_at(g, ray, s, gv, tb);
        tb[12] += (double)eb.alpha;
      }
    }
    if constexpr (GRID) fld.accumulate_step(g, ray, s, gv, act, acc, gbn, gc);
  }
  if constexpr (GRID) fld.flush_all(acc, gbn, gc);

  if constexpr (THETA) {
    // alpha also enters the per-frequency prefactors: d ln s / d alpha * this lane's share
#pragma unroll
    for (int f = 0; f < MF; ++f)
      if (f < fa.n_freq)
        tb[12] += fa.dlnsI[f] * gi_f[f] * accI + fa.dlnsP[f] * (hr[f] * accPr[f] - hi[f] * accPi[f]);
  }
}

// Sums tb[16] over the 256 threads of a block in a fixed order (wavefront
// butterfly, then the four waves); thread k < 16 returns the total of k.
__device__ inline double block_reduce16(const double* tb, int k_out) {
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
  double r = 0.0;
  if (k_out < kNParam) r = (red[0][k_out] + red[1][k_out]) + (red[2][k_out] + red[3][k_out]);
  __syncthreads();
  return r;
}

}  // namespace sm
