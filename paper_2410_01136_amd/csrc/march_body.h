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
constexpr double kLn2 = 0.6931471805599453;

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

// Free-free emission and absorption (FF): every segment's emission reaches
// the observer attenuated by e^-tau_f, tau_f = kff_f dkpc EM with EM the sum of
// n_e^2 over the earlier segments plus half of this one (a second prefix sum,
// carried like the Faraday sum), and the segment adds T_e dtau_f to I.
//
// Gridded spectral index (VA): the emission of a segment uses the local alpha,
// its exponent in B_perp and its frequency prefactors (one ratio per
// frequency to the prefactors of theta[12]), so the I sum is per frequency.
//
// Spectral model SP: one power law (kSpecPower), a gridded index
// (kSpecGridAlpha, the VA path above) or a broken power law (kSpecBroken): the
// emission of the index below the break scaled per frequency by the
// multipliers of bp_mult (interpolated moment shares), so the I sum is per
// frequency as well.
//
// PC (grid, spiral-disk and WMAP fields): also store the piece snapshots of
// the field (the running sums at the piece ends of a reverse pass in pieces), so
// that pass needs no pre-pass over its pieces.
template <class F>
constexpr bool kHasSnapshots = std::is_base_of_v<Grid, F> || std::is_base_of_v<Model16, F> ||
                               std::is_base_of_v<Wmap, F>;
// The snapshot fields of a field: in GridArgs for grids, beside the arguments
// (SnapArgs) for the analytic and WMAP fields.
template <class F>
__host__ __device__ inline const auto& snap_args(const F& f) {
  if constexpr (std::is_base_of_v<Grid, F>) return f.p;
  else return f.sn;
}

template <class F, int S, int MF, bool FF = false, int SP = kSpecPower, bool PC = false, class FA>
__device__ inline void fwd_lane(const GeomArgs& g, const FA& fa, const EmitArgs& ea, const F& fld,
                                int64_t q, int sub, bool valid, float* __restrict__ maps,
                                MapAddr ma, double* __restrict__ phi_end,
                                double* __restrict__ em_end = nullptr) {
  const Ray ray = make_ray(g, q);
  const auto rctx = fld.ray_ctx(g, ray);
  constexpr bool zero_beyond = zero_beyond_path<F>();
  constexpr bool VA = SP == kSpecGridAlpha, BP = SP == kSpecBroken;
  constexpr bool PF = FF || VA || BP;  // per-frequency I sums
  constexpr int MFF = FF ? MF : 1;
  constexpr int MPF = PF ? MF : 1;
  double carry = 0.0;  // Faraday sum (n_e B_par, uG cm^-3) of all earlier chunks
  double emc = 0.0;    // FF: sum of n_e^2 (cm^-6) of all earlier chunks
  double accI = 0.0;
  double accQ[MF], accU[MF];
  double accIf[MPF], accF[MFF];  // per-frequency synchrotron I; FF: free-free sums
#pragma unroll
  for (int f = 0; f < MF; ++f) accQ[f] = accU[f] = 0.0;
#pragma unroll
  for (int f = 0; f < MPF; ++f) accIf[f] = 0.0;
#pragma unroll
  for (int f = 0; f < MFF; ++f) accF[f] = 0.0;

  constexpr int MPC = PC ? MF : 1;
  double tq[MPC], tu[MPC], ti[PC && PF ? MF : 1], tf[PC && FF ? MF : 1];  // PC: this step's terms
  int pc_k = 1;  // PC: the next piece end to store, k piece_len
  for (int c0 = 0; c0 < g.n_steps; c0 += S) {
    const int n = c0 + sub;
    const bool act = n < g.n_steps;
    const double s = ((double)n + 0.5) * ray.dkpc;  // midpoint of segment n
    const double carry0 = carry, emc0 = emc;  // PC: sums before this chunk
    double fincl = 0.0, eincl = 0.0;          // PC: inclusive chunk scans
    // (the shared-read grid brings a gridded alpha with its cell records)
    constexpr bool VA_SHARED = VA && std::is_same_v<F, GridL>;
    double al = 0.0;
    FV v;
    if constexpr (VA_SHARED)
      v = fld.template eval_step_va<S>(g, ray, rctx, s, n, ea.va_alpha_ref, al);
    else
      v = fld.template eval_step<S>(g, ray, rctx, s, n);
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
      fincl = incl;
    }
    float w = 0.0f, emd = 0.0f;  // FF: n_e^2 of this segment, emission measure * dkpc
    if constexpr (FF) {
      w = (zero_beyond || act) ? v.ne * v.ne : 0.0f;
      double em;
      if constexpr (S == 1) {
        em = emc + 0.5 * (double)w;
        emc += (double)w;
      } else {
        const double incl = group_inclusive_scan<S>((double)w, sub);
        em = emc + incl - 0.5 * (double)w;
        emc += group_last<S>(incl);
        eincl = incl;
      }
      emd = (float)(em * ray.dkpc);
    }
    VaStep vs{};
    if constexpr (VA) {
      if constexpr (!VA_SHARED) al = fld.alpha_at(g, ray, s, ea.va_alpha_ref);
      vs = va_step(al, ea);
    }
    Emit e = VA ? emission(v.n0, bl, bb, false, vs.eI) : emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
    if (!zero_beyond && !act) e.u = e.zr = e.zi = 0.0f;
    if constexpr (!PF) accI += (double)e.u;
    BpStep bs{};
    if constexpr (BP) bs = bp_step(bl, bb, ea);
    const double psid = psi * ray.dkpc;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (exact_freqs(MF) || f < fa.n_freq) {
        float sn, cs;
        sincos_turns(psid * fa.kappa[f], &sn, &cs);  // turns of 2 RM lambda^2
        float zr = e.zr, zi = e.zi;
        if constexpr (PF) {
          float mI = 1.0f, mP = 1.0f;  // per-frequency multipliers of I and of Q + iU
          if constexpr (VA) {
            mI = va_ratio(vs, fa.va_k1l2[f], al, ea);
            mP = mI * vs.prat;
          }
          if constexpr (BP) {
            const BpMult bm = bp_mult<false>(bs, fa.bp_l[f], fa.bp_k1[f], fa.bp_k2[f], fa.bp_ri[f],
                                             fa.bp_rp[f], ea.bp_tab);
            mI = bm.mI;
            mP = bm.mP;
          }
          if constexpr (FF) {
            const float att = exp2f(-(float)fa.kffl2[f] * emd);
            mI *= att;
            mP *= att;
            const double t = (double)(att * w);
            accF[f] += t;
            if constexpr (PC) tf[f] = t;
          }
          zr *= mP;
          zi *= mP;
          const double t = (double)(mI * e.u);
          accIf[f] += t;
          if constexpr (PC) ti[f] = t;
        }
        const double tq1 = (double)(zr * cs - zi * sn), tu1 = (double)(zr * sn + zi * cs);
        accQ[f] += tq1;
        accU[f] += tu1;
        if constexpr (PC) {
          tq[f] = tq1;
          tu[f] = tu1;
        }
      }
    }
    if constexpr (PC) {
      // piece ends inside this chunk (those at or beyond the last step are
      // written after the loop, from the totals): sums over the steps before b
      const auto& sa = snap_args(fld);
      for (; pc_k <= sa.pieces && pc_k * sa.piece_len <= c0 + S && pc_k * sa.piece_len < g.n_steps;
           ++pc_k) {
        const int k = pc_k;
        const int b = k * sa.piece_len;
        const bool before = n < b;
        double* out = sa.snap + (int64_t)(k - 1) * sa.snap_nq * ma.stride + ma.off + ray.ring;
        const int64_t st = ma.stride;
        const double phib = S == 1 ? carry : carry0 + group_bcast<S>(fincl, b - 1 - c0);
        if (valid && sub == 0) out[0] = phib;
#pragma unroll
        for (int f = 0; f < MF; ++f) {
          if (exact_freqs(MF) || f < fa.n_freq) {
            const double pq = group_sum<S>(before ? accQ[f] : accQ[f] - tq[f]);
            const double pu = group_sum<S>(before ? accU[f] : accU[f] - tu[f]);
            if (valid && sub == 0) {
              out[(1 + 2 * f) * st] = pq;
              out[(2 + 2 * f) * st] = pu;
            }
          }
        }
        if constexpr (FF) {
          const int nf = fa.n_freq;
          const double emb = S == 1 ? emc : emc0 + group_bcast<S>(eincl, b - 1 - c0);
          if (valid && sub == 0) out[(1 + 2 * nf) * st] = emb;
#pragma unroll
          for (int f = 0; f < MF; ++f) {
            if (exact_freqs(MF) || f < nf) {
              const double pi = group_sum<S>(before ? accIf[f] : accIf[f] - ti[f]);
              const double pf = group_sum<S>(before ? accF[f] : accF[f] - tf[f]);
              if (valid && sub == 0) {
                out[(2 + 2 * nf + f) * st] = pi;
                out[(2 + 3 * nf + f) * st] = pf;
              }
            }
          }
        }
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
    if constexpr (PF) {
#pragma unroll
      for (int f = 0; f < MF; ++f) accIf[f] = group_sum<S>(accIf[f]);
    }
    if constexpr (FF) {
#pragma unroll
      for (int f = 0; f < MF; ++f) accF[f] = group_sum<S>(accF[f]);
    }
  }
  if (valid && sub == 0) {
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (exact_freqs(MF) || f < fa.n_freq) {
        double tI;
        if constexpr (PF)
          tI = fa.sI[f] * ray.dkpc * accIf[f];
        else
          tI = fa.sI[f] * ray.dkpc * accI;
        if constexpr (FF) tI += fa.tff[f] * ray.dkpc * accF[f];
        maps[ma.at(f, 0, ray.ring)] = (float)tI;
        maps[ma.at(f, 1, ray.ring)] = (float)(fa.sP[f] * ray.dkpc * accQ[f]);
        maps[ma.at(f, 2, ray.ring)] = (float)(fa.sP[f] * ray.dkpc * accU[f]);
      }
    }
    if (phi_end != nullptr) phi_end[ma.off + ray.ring] = carry;
    if constexpr (FF)
      if (em_end != nullptr) em_end[ma.off + ray.ring] = emc;
  }
  if constexpr (PC) {
    // piece ends at or beyond the last step: the totals
    if (valid && sub == 0) {
      const int nf = fa.n_freq;
      const int64_t st = ma.stride;
      const auto& sa = snap_args(fld);
      for (int k = max(1, (g.n_steps + sa.piece_len - 1) / sa.piece_len); k <= sa.pieces; ++k) {
        double* out = sa.snap + (int64_t)(k - 1) * sa.snap_nq * st + ma.off + ray.ring;
        out[0] = carry;
#pragma unroll
        for (int f = 0; f < MF; ++f) {
          if (exact_freqs(MF) || f < nf) {
            out[(1 + 2 * f) * st] = accQ[f];
            out[(2 + 2 * f) * st] = accU[f];
          }
        }
        if constexpr (FF) {
          out[(1 + 2 * nf) * st] = emc;
#pragma unroll
          for (int f = 0; f < MF; ++f) {
            if (exact_freqs(MF) || f < nf) {
              out[(2 + 2 * nf + f) * st] = accIf[f];
              out[(2 + 3 * nf + f) * st] = accF[f];
            }
          }
        }
      }
    }
  }
}

// Reverse march of NESTED pixel q for L = sum(dmaps * maps).  Adds this
// lane's share of dL/dtheta into tb (THETA) and scatters grid gradients
// (GRID).  FA additionally provides dlnsI[], dlnsP[].
//
// With a grid gradient, or PIECES (the theta-only reverse pass of the march
// kernels), and S > 1 the S lanes of a sightline do not interleave steps: lane
// k walks its own contiguous piece of ceil(N / S) steps, so that it stays in
// one cell for as many steps as a single lane would and its register
// accumulator flushes as rarely, and no step needs a lane exchange.  The piece needs two numbers from the pieces
// beyond it: the Faraday sum before its end, and the sum of the phase
// cotangents after it.  A pre-pass over the piece gets both with one march:
// the Faraday sum of the piece, and per frequency the sum of z_n e^{2 pi i t_n}
// with t_n counted from the piece start; once a group scan has given the
// Faraday sum of the earlier pieces, a rotation by its phase turns the latter
// into the piece's phase-cotangent total, and a suffix scan gives each piece
// those of the pieces after it.
template <class F, int S, int MF, bool THETA, bool GRID, bool FF = false, int SP = kSpecPower,
          bool PIECES = false, class FA>
__device__ inline void adj_lane(const GeomArgs& g, const FA& fa, const EmitArgs& ea, const F& fld,
                                int64_t q, int sub, bool valid, const float* __restrict__ dmaps,
                                MapAddr ma, const double* __restrict__ phi_end, double* tb,
                                float* gbn, float* gc, const AdjBox* lds_box = nullptr,
                                float* lds_stage = nullptr,
                                const double* __restrict__ em_end = nullptr) {
  const Ray ray = make_ray(g, q);
  const double dk = ray.dkpc;
  constexpr int MFF = FF ? MF : 1;
  constexpr bool VA = SP == kSpecGridAlpha, BP = SP == kSpecBroken;
  constexpr bool PF = FF || VA || BP;  // per-frequency multipliers of the emission
  // (with a gridded alpha, theta[12] does not enter the maps: no alpha
  // gradient); a broken power law adds the gradient in its index above the
  // break and in ln gamma_b as tb[kNParam], tb[kNParam + 1]
  constexpr bool ALPHA_GRAD = THETA && !VA;
  constexpr bool SPEC_GRAD = THETA && BP;

  // per-sightline cotangent constants
  double GI = 0.0;
  double hr[MF], hi[MF], kr[MF], ki[MF], gi_f[MF];
  double cf[MFF], kd[MFF];  // FF: dI T_e kff dkpc, and d tau / d EM = kff dkpc
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
      if constexpr (FF) cf[f] = dI * fa.tff[f] * dk;
    } else if constexpr (FF) {
      cf[f] = 0.0;
    }
    if constexpr (FF) kd[f] = fa.kffl2[f] * kLn2 * dk;
  }

  typename F::Acc acc;  // grid-gradient accumulator
  if constexpr (GRID) {
    acc.box = *lds_box;
    acc.stage = lds_stage;
  }
  // each lane walks a contiguous run [n_lo, n_hi) of steps (one lane per
  // sightline, or one piece of it) rather than every S-th step
  constexpr bool SPLIT = (GRID || PIECES) && S > 1;
  constexpr bool SERIAL = S == 1 || SPLIT;
  int n_lo = 0, n_hi = g.n_steps;
  double E = 0.0;     // Faraday sum over the steps before the current chunk's end
  double suf = 0.0;   // phase cotangents of the steps after it
  double EM = 0.0;    // FF: sum of n_e^2 over the steps before the current chunk's end
  double sufE = 0.0;  // FF: cotangents of the emission measure after it
  if constexpr (SPLIT) {
    const int len = (g.n_steps + S - 1) / S;
    n_lo = min(sub * len, g.n_steps);
    n_hi = min(n_lo + len, g.n_steps);
    const auto& sa = snap_args(fld);
    if (sa.snap != nullptr) {
      // The forward stored the running sums at every piece end (S pieces of this
      // length): the piece's own sums are differences of those at its two ends,
      // with the absolute phase and attenuation already applied, so
      //   B_k = Im(sum_f k_f dP_f),  X_k = -sum_f kd_f (gi_f dU_f + cf_f dV_f + Re(h_f dP_f)).
      const int nf = fa.n_freq;
      const int64_t st = g.npix;
      const double* hi_end = sa.snap + (int64_t)sub * sa.snap_nq * st + ray.ring;
      const double* lo_end = sa.snap + (int64_t)(sub > 0 ? sub - 1 : 0) * sa.snap_nq * st + ray.ring;
      auto lo_at = [&](int j) { return sub > 0 ? lo_end[j * st] : 0.0; };
      double Bk = 0.0, Xk = 0.0;
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < nf) {
          const double dPr = hi_end[(1 + 2 * f) * st] - lo_at(1 + 2 * f);
          const double dPi = hi_end[(2 + 2 * f) * st] - lo_at(2 + 2 * f);
          Bk += kr[f] * dPi + ki[f] * dPr;
          if constexpr (FF) {
            const double dU = hi_end[(2 + 2 * nf + f) * st] - lo_at(2 + 2 * nf + f);
            const double dV = hi_end[(2 + 3 * nf + f) * st] - lo_at(2 + 3 * nf + f);
            Xk -= kd[f] * (gi_f[f] * dU + cf[f] * dV + hr[f] * dPr - hi[f] * dPi);
          }
        }
      }
      E = hi_end[0];
      suf = group_suffix_scan<S>(Bk, sub) - Bk;
      if constexpr (FF) {
        EM = hi_end[(1 + 2 * nf) * st];
        sufE = group_suffix_scan<S>(Xk, sub) - Xk;
      }
    } else {
      // per frequency: W = sum z a e^{2 pi i t}, U = sum u a, V = sum w a, with the
      // phase t and the attenuation a counted from the piece start
      double A = 0.0, Ak = 0.0, Wr[MF], Wi[MF], Uf[MFF], Vf[MFF];
#pragma unroll
      for (int f = 0; f < MF; ++f) Wr[f] = Wi[f] = 0.0;
#pragma unroll
      for (int f = 0; f < MFF; ++f) Uf[f] = Vf[f] = 0.0;
      for (int n = n_lo; n < n_hi; ++n) {
        const FV v = fld.eval_at(g, ray, ((double)n + 0.5) * dk);
        const float bl = v.bx * ray.elx + v.by * ray.ely;
        const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
        const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
        const double cn = (double)v.ne * bpar;
        const double psid = (A + 0.5 * cn) * dk;  // Faraday sum from the piece start
        A += cn;
        float w = 0.0f, emd = 0.0f;
        if constexpr (FF) {
          w = v.ne * v.ne;
          emd = (float)((Ak + 0.5 * (double)w) * dk);
          Ak += (double)w;
        }
        double al = 0.0;
        VaStep vs{};
        if constexpr (VA) {
          al = fld.alpha_at(g, ray, ((double)n + 0.5) * dk, ea.va_alpha_ref);
          vs = va_step(al, ea);
        }
        const Emit e =
            VA ? emission(v.n0, bl, bb, false, vs.eI) : emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
        BpStep bs{};
        if constexpr (BP) bs = bp_step(bl, bb, ea);
#pragma unroll
        for (int f = 0; f < MF; ++f) {
          if (f < fa.n_freq) {
            float sn, cs;
            sincos_turns(psid * fa.kappa[f], &sn, &cs);
            float zr = e.zr, zi = e.zi;
            if constexpr (PF) {
              float mI = 1.0f, mP = 1.0f;
              if constexpr (VA) {
                mI = va_ratio(vs, fa.va_k1l2[f], al, ea);
                mP = mI * vs.prat;
              }
              if constexpr (BP) {
                const BpMult bm = bp_mult<false>(bs, fa.bp_l[f], fa.bp_k1[f], fa.bp_k2[f],
                                                 fa.bp_ri[f], fa.bp_rp[f], ea.bp_tab);
                mI = bm.mI;
                mP = bm.mP;
              }
              if constexpr (FF) {
                const float att = exp2f(-(float)fa.kffl2[f] * emd);
                mI *= att;
                mP *= att;
                Vf[f] += (double)(att * w);
              }
              zr *= mP;
              zi *= mP;
              if constexpr (FF) Uf[f] += (double)(mI * e.u);
            }
            Wr[f] += (double)(zr * cs - zi * sn);
            Wi[f] += (double)(zr * sn + zi * cs);
          }
        }
      }
      const double incl = group_inclusive_scan<S>(A, sub);
      const double psid0 = (incl - A) * dk;  // Faraday sum of the earlier pieces
      double emincl = 0.0, emd0 = 0.0;
      if constexpr (FF) {
        emincl = group_inclusive_scan<S>(Ak, sub);
        emd0 = (emincl - Ak) * dk;  // emission measure of the earlier pieces
      }
      double Bk = 0.0;  // sum of this piece's phase cotangents
      double Xk = 0.0;  // FF: sum of this piece's emission-measure cotangents
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < fa.n_freq) {
          float sn, cs;
          sincos_turns(psid0 * fa.kappa[f], &sn, &cs);
          double a0 = 1.0;
          if constexpr (FF) a0 = (double)exp2f(-(float)(fa.kffl2[f] * emd0));
          const double rr = kr[f] * cs - ki[f] * sn, ri = kr[f] * sn + ki[f] * cs;
          Bk += a0 * (rr * Wi[f] + ri * Wr[f]);  // Im(k e^{2 pi i t0} a0 W)
          if constexpr (FF) {
            const double Rr = hr[f] * cs - hi[f] * sn, Ri = hr[f] * sn + hi[f] * cs;
            Xk -= kd[f] * a0 * (gi_f[f] * Uf[f] + cf[f] * Vf[f] + Rr * Wr[f] - Ri * Wi[f]);
          }
        }
      }
      E = incl;
      suf = group_suffix_scan<S>(Bk, sub) - Bk;
      if constexpr (FF) {
        EM = emincl;
        sufE = group_suffix_scan<S>(Xk, sub) - Xk;
      }
    }
  } else if (valid) {
    E = phi_end[ma.off + ray.ring];
    if constexpr (FF) EM = em_end[ma.off + ray.ring];
  }
  // this lane's theta cotangents, summed in FP32 over its steps (a few hundred
  // terms at most) and added to the FP64 tb at the end
  float tbf[THETA ? kNParam : 1];
#pragma unroll
  for (int k = 0; k < (THETA ? kNParam : 1); ++k) tbf[k] = 0.0f;
  float spg[3] = {0.0f, 0.0f, 0.0f};  // SPEC_GRAD: d L / d (alpha_lo, alpha_hi, ln gamma_b)
  constexpr int MPF = PF ? MF : 1;
  // A step's cotangent rotations and multipliers, and this lane's alpha sums,
  // are FP32: each step's terms are FP32 products; the sums over steps that
  // need it (the Faraday and emission-measure cotangents) stay FP64.
  float accI = 0, accPr[MF], accPi[MF], accIf[MPF];
  float hrs[MF], his[MF], krs[MF], kis[MF], gis[MF], cfs[MFF], kds[MFF];
#pragma unroll
  for (int f = 0; f < MF; ++f) {
    accPr[f] = accPi[f] = 0;
    hrs[f] = (float)hr[f];
    his[f] = (float)hi[f];
    krs[f] = (float)kr[f];
    kis[f] = (float)ki[f];
    gis[f] = (float)gi_f[f];
  }
#pragma unroll
  for (int f = 0; f < MFF; ++f) {
    cfs[f] = (float)cf[f];
    kds[f] = (float)kd[f];
  }
#pragma unroll
  for (int f = 0; f < MPF; ++f) accIf[f] = 0;

  // every lane of a wavefront runs the same number of iterations (the grid
  // scatter is collective); a short or empty last piece idles through the rest
  const int n_iter = SPLIT ? (g.n_steps + S - 1) / S : SERIAL ? g.n_steps : (g.n_steps + S - 1) / S;
  auto step_of = [&](int it) { return SERIAL ? n_lo + it : it * S + sub; };
  // GRID: the corner reads of the step visited next (the one before it along
  // the sightline) are issued before the current step's work, so that their
  // latency overlaps it
  using FetchT = std::conditional_t<GRID, Grid::Fetch, int>;
  using CellT = std::conditional_t<GRID, Grid::Cell, int>;
  FetchT fnext{};
  if constexpr (GRID) fld.fetch(g, ray, ((double)step_of(n_iter - 1) + 0.5) * dk, fnext);
  for (int it = n_iter - 1; it >= 0; --it) {
    const int n = step_of(it);
    const bool act = valid && n < n_hi;
    const double s = ((double)n + 0.5) * dk;
    FV v;
    CellT cell{};
    if constexpr (GRID) {
      const FetchT fcur = fnext;
      if (it > 0) fld.fetch(g, ray, ((double)step_of(it - 1) + 0.5) * dk, fnext);
      v = fld.interp(g, ray, s, fcur);
      cell = fcur.c;
    } else {
      v = fld.eval_at(g, ray, s);
    }
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
    float w = 0.0f, emd = 0.0f;
    if constexpr (FF) {
      w = (n < n_hi) ? v.ne * v.ne : 0.0f;
      double em;
      if constexpr (SERIAL) {
        EM -= (double)w;
        em = EM + 0.5 * (double)w;
      } else {
        const double incl = group_inclusive_scan<S>((double)w, sub);
        const double tot = group_last<S>(incl);
        em = EM - tot + incl - 0.5 * (double)w;
        EM -= tot;
      }
      emd = (float)(em * dk);
    }
    double al = 0.0;
    VaStep vs{};
    if constexpr (VA) {
      al = fld.alpha_at(g, ray, s, ea.va_alpha_ref);
      vs = va_step(al, ea);
    }
    const float eI = VA ? vs.eI : ea.eI;
    const bool a3 = VA ? false : ea.alpha3 != 0;
    Emit e = emission(v.n0, bl, bb, a3, eI);
    if (!act) e.u = e.zr = e.zi = 0.0f;
    BpStep bs{};
    float xlg = 0.0f;  // BP: d L / d log2 B_perp^2 through the multipliers
    if constexpr (BP) bs = bp_step(bl, bb, ea);
    // H = sum_f mP_f h_f e^{2 pi i t_f};  K = sum_f mP_f k_f e^{2 pi i t_f}
    // (mI_f, mP_f the per-frequency multipliers of I and Q + iU: the free-free
    // attenuation and the local-alpha prefactor ratio; 1 without either)
    float Hr = 0, Hi = 0, Kr = 0, Ki = 0;
    float GIe = (float)GI;  // sum_f mI_f gi_f
    float Cw = 0.0f;  // FF: d L / d w of this segment's own free-free emission
    float X = 0.0f;   // FF: d L / d EM at this midpoint
    if constexpr (PF) GIe = 0.0f;
    const double psid = psi * dk;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < fa.n_freq) {
        float sn, cs;
        sincos_turns(psid * fa.kappa[f], &sn, &cs);
        if constexpr (PF) {
          const float hrf = hrs[f] * cs - his[f] * sn, hif = hrs[f] * sn + his[f] * cs;
          const float krf = krs[f] * cs - kis[f] * sn, kif = krs[f] * sn + kis[f] * cs;
          float mI = 1.0f, mP = 1.0f, att = 1.0f, dmI = 0.0f, dmP = 0.0f;
          if constexpr (VA) {
            mI = va_ratio(vs, fa.va_k1l2[f], al, ea);
            mP = mI * vs.prat;
          }
          BpMult bm{};
          if constexpr (BP) {
            bm = bp_mult<true, SPEC_GRAD>(
                bs, fa.bp_l[f], fa.bp_k1[f], fa.bp_k2[f], fa.bp_ri[f], fa.bp_rp[f], ea.bp_tab,
                BpSpecArgs{fa.bp_dri1[f], fa.bp_dri2[f], fa.bp_drp1[f], fa.bp_drp2[f]});
            mI = bm.mI;
            mP = bm.mP;
            dmI = bm.dI;
            dmP = bm.dP;
          }
          if constexpr (FF) {
            att = exp2f(-(float)fa.kffl2[f] * emd);
            mI *= att;
            mP *= att;
          }
          if constexpr (BP) {
            // cotangents of this step's multipliers of I and of Q + iU
            const float wI = att * gis[f] * e.u, wP = att * (hrf * e.zr - hif * e.zi);
            xlg += wI * dmI + wP * dmP;
            if constexpr (SPEC_GRAD) {
#pragma unroll
              for (int j = 0; j < 3; ++j) spg[j] += wI * bm.sI[j] + wP * bm.sP[j];
            }
          }
          Hr += mP * hrf;
          Hi += mP * hif;
          Kr += mP * krf;
          Ki += mP * kif;
          GIe += mI * gis[f];
          if constexpr (FF) {
            Cw += att * cfs[f];
            X -= kds[f] * (mI * gis[f] * e.u + att * cfs[f] * w + mP * (hrf * e.zr - hif * e.zi));
          }
          if constexpr (ALPHA_GRAD) {
            accIf[f] += mI * e.u;
            accPr[f] += mP * (e.zr * cs - e.zi * sn);
            accPi[f] += mP * (e.zr * sn + e.zi * cs);
          }
        } else {
          Hr += hrs[f] * cs - his[f] * sn;
          Hi += hrs[f] * sn + his[f] * cs;
          Kr += krs[f] * cs - kis[f] * sn;
          Ki += krs[f] * sn + kis[f] * cs;
          if constexpr (ALPHA_GRAD) {
            accPr[f] += e.zr * cs - e.zi * sn;
            accPi[f] += e.zr * sn + e.zi * cs;
          }
        }
      }
    }
    if constexpr (ALPHA_GRAD && !PF) accI += e.u;
    // cotangent of the Faraday sum at this midpoint: Im(zc K)
    const double pb = (double)(e.zr * Ki + e.zi * Kr);
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
    double wbar = 0.0;  // FF: cotangent of this segment's n_e^2
    if constexpr (FF) {
      if (!act) X = Cw = 0.0f;
      const double Xd = (double)X;
      double ebar;  // through the emission measure: later midpoints + half of its own
      if constexpr (SERIAL) {
        ebar = sufE + 0.5 * Xd;
        sufE += Xd;
      } else {
        const double sincl = group_suffix_scan<S>(Xd, sub);
        const double stot = group_first<S>(sincl);
        ebar = sufE + sincl - 0.5 * Xd;
        sufE += stot;
      }
      wbar = (double)Cw + ebar;
    }
    // local reverse of the emission and projections
    EmitBar eb = emission_vjp(v.n0, bl, bb, a3, eI, GIe, Hr, -Hi);
    if constexpr (BP) {
      // the multipliers' dependence on B_perp: d log2 B_perp^2 / d B_perp^2 = log2(e) / B_perp^2
      const float bt2 = bl * bl + bb * bb;
      if (bt2 > 0.0f) {
        const float xb = xlg * 1.4426950408889634f * frcp(bt2);
        eb.bl += 2.0f * bl * xb;
        eb.bb += 2.0f * bb * xb;
      }
    }
    float neb = (float)(cbar * bpar);
    if constexpr (FF) neb += (float)(2.0 * wbar) * v.ne;
    const float bparb = (float)(cbar * (double)v.ne);
    FV gv;
    gv.bx = eb.bl * ray.elx + eb.bb * ray.ebx - bparb * (float)ray.nx;
    gv.by = eb.bl * ray.ely + eb.bb * ray.eby - bparb * (float)ray.ny;
    gv.bz = eb.bb * ray.ebz - bparb * (float)ray.nz;
    gv.ne = neb;
    gv.n0 = eb.n0;
    if constexpr (THETA) {
      if (act) {
        fld.vjp_at(g, ray, s, gv, tbf);
        if constexpr (ALPHA_GRAD) tbf[12] += eb.alpha;
      }
    }
    if constexpr (GRID) fld.accumulate_cell(cell, gv, act, acc, gbn, gc);
  }
  if constexpr (GRID) fld.flush_all(acc, gbn, gc);
  if constexpr (THETA) {
#pragma unroll
    for (int k = 0; k < kNParam; ++k) tb[k] += (double)tbf[k];
  }
  if constexpr (SPEC_GRAD) {
    tb[12] += (double)spg[0];
    tb[kNParam] += (double)spg[1];
    tb[kNParam + 1] += (double)spg[2];
  }

  if constexpr (ALPHA_GRAD) {
    // alpha also enters the per-frequency prefactors: d ln s / d alpha * this lane's share
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < fa.n_freq) {
        const double aI = (double)(PF ? accIf[f] : accI);
        tb[12] += fa.dlnsI[f] * gi_f[f] * aI +
                  fa.dlnsP[f] * (hr[f] * (double)accPr[f] - hi[f] * (double)accPi[f]);
      }
    }
  }
}

// Sums tb[NP] over the 256 threads of a block in a fixed order (wavefront
// butterfly, then the four waves); thread k < NP returns the total of k.
template <int NP>
__device__ inline double block_reduce(const double* tb, int k_out) {
  __shared__ double red[4][NP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double v = tb[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  double r = 0.0;
  if (k_out < NP) r = (red[0][k_out] + red[1][k_out]) + (red[2][k_out] + red[3][k_out]);
  __syncthreads();
  return r;
}
__device__ inline double block_reduce16(const double* tb, int k_out) {
  return block_reduce<kNParam>(tb, k_out);
}

}  // namespace sm
