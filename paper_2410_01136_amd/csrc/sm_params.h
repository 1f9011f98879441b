// Kernel argument blocks (plain data, filled on the host, passed by value).
#pragma once

#include <stdint.h>

namespace sm {

constexpr int kMaxFreq = 16;
constexpr int kNParam = 16;

struct GeomArgs {
  int32_t nside, order;  // order = log2(nside)
  int32_t n_steps;
  int64_t npix;
  double r_obs[3];
  double r_max;
  double box_lo[3], box_hi[3];
};

struct M16Args {
  float B0, psi0, psi1, chiB0;
  float sin_psi0, cos_psi0;
  float invRB, invzB, l2_invRB, l2_invzB;
  float BH0, invzH, invRH, l2_invzH, l2_invRH;
  float C0, invhr, invhz, l2_invhr, l2_invhz;
  float n0, invhne, l2_invhne, l2_kappa;
  float log2_rsun;
};

// WMAP field of Sec. 3.1 (FP32 constants derived on the host).
struct WmapArgs {
  float b0, psi0, psi1, chi0;
  float rin, rout;
  float C0, invhr, invhz;
  float n0, invhne, l2_invhne, l2_kappa;
};

// Piece snapshots of the analytic and WMAP fields (as in GridArgs; snap
// nullptr: none).  Kept beside their argument blocks, not in them, so that the
// batch kernels' per-set descriptors do not carry them.
struct SnapArgs {
  double* snap;
  int32_t pieces, piece_len, snap_nq;
};

struct GridArgs {
  const float4* bn;  // [nz][ny][nx] x (Bx, By, Bz, n_e)
  const float* c;    // [nz][ny][nx] N0 or nullptr
  const float* alpha;  // [nz][ny][nx] CR spectral index or nullptr (theta[12])
  int32_t n[3];
  double lo[3], inv_h[3], umax[3];  // umax = n - 1
  // 32-bit buffer addressing (grids under 4 GiB): sizes in bytes and the byte
  // strides of one y row and one z plane in the float4 grid and in the N0 grid
  uint32_t bn_bytes, c_bytes;
  uint32_t sy16, sz16, sy4, sz4;
  // Piece snapshots of a forward that a reverse pass in pieces will follow
  // (nullptr: none).  The analytic and WMAP fields carry the same (SnapArgs).  The reverse pass cuts each sightline into `pieces`
  // contiguous pieces of `piece_len` steps; at each piece end b_k = k piece_len
  // (k = 1 .. pieces, capped at n_steps) the forward stores, per pixel, the
  // running sums over the steps before b_k: the Faraday sum, per frequency the
  // Q and U sums, and with free-free the emission-measure sum and per
  // frequency the I and free-free sums.  Layout [k - 1][quantity][npix] with
  // `snap_nq` quantities.
  double* snap;
  int32_t pieces, piece_len, snap_nq;
};

// Box of grid nodes in which one workgroup of the grid adjoint accumulates its
// gradients in LDS (5 floats per node, x fastest) before adding them to memory
// once; nodes outside it get global atomic adds.
//
// Each wavefront also has a staging area in LDS for the cell records (8 corners
// x 5 channels plus the cell index) of the lanes that leave their cell in one
// step, from which the whole wavefront adds them out.
constexpr int kStageRecs = 16;    // records per wavefront and round
constexpr int kStageFloats = 44;  // 40 values, 3 cell indices, 1 pad (16-byte rows)
constexpr int kStageBytesPerBlock = 4 * kStageRecs * kStageFloats * 4;  // 4 wavefronts
// LDS of a CU, and what the kernel's static LDS takes besides the box and the
// staging areas.
constexpr int kAdjLdsBytes = 160 * 1024;
constexpr int kAdjStaticLds = 1024;
// Box nodes of a workgroup that has 1/per_cu of the LDS, a multiple of 4 (so
// the staging areas after the box stay 16-byte aligned).
constexpr int adj_box_cap(int per_cu) {
  return ((kAdjLdsBytes / per_cu - kAdjStaticLds - kStageBytesPerBlock) / 20) & ~3;
}
constexpr int kAdjBoxNodesMax = adj_box_cap(1);

struct AdjBox {
  float* lds = nullptr;  // [d[2]][d[1]][d[0]][5], or nullptr (no box)
  int b0[3] = {0, 0, 0};  // first node
  int d[3] = {0, 0, 0};   // nodes per axis
};

struct SphereArgs {
  float b[3];
  float ne, n0, r2;
  float c[3];
};

// Per-frequency constants of the sums, all FP64:
//   T_I = sI * dkpc * sum u,   T_Q + i T_U = sP * dkpc * sum zc e^{2 pi i t},
//   t = kappa * dkpc * (Faraday sum of n_e B_par in uG cm^-3 units).
struct FreqArgs {
  int32_t n_freq;
  double sI[kMaxFreq];
  double sP[kMaxFreq];
  double kappa[kMaxFreq];
  // d ln sI / d alpha, d ln sP / d alpha (adjoint only)
  double dlnsI[kMaxFreq];
  double dlnsP[kMaxFreq];
  // free-free: tau = kffl2 ln 2 * dkpc * (emission-measure sum of n_e^2 in
  // cm^-6), and the free-free term of T_I = tff * dkpc * sum e^-tau n_e^2
  double kffl2[kMaxFreq];
  double tff[kMaxFreq];
  // gridded alpha: log2(e) d ln sI / d alpha without the Gamma-function part
  double va_k1l2[kMaxFreq];
  // broken power law (prefactors sI, sP above are those of alpha_lo = theta[12]):
  // log2 of xb B_perp [uG], 2^(p_lo bp_l), 2^(p_hi bp_l), and the prefactor
  // ratios sI(alpha_hi) / sI(alpha_lo), sP(alpha_hi) / sP(alpha_lo) with the
  // normalisation gamma_b^(alpha_hi - alpha_lo) of the upper law
  float bp_l[kMaxFreq];
  float bp_k1[kMaxFreq];
  float bp_k2[kMaxFreq];
  float bp_ri[kMaxFreq];
  float bp_rp[kMaxFreq];
  // d ln(bp_ri) / d alpha_lo, d ln(bp_ri) / d alpha_hi, and the same of bp_rp
  // (gradient in the spectral parameters)
  float bp_dri1[kMaxFreq];
  float bp_dri2[kMaxFreq];
  float bp_drp1[kMaxFreq];
  float bp_drp2[kMaxFreq];
};

// Spectral model of the CR electrons: one power law of index theta[12], a
// gridded index, or a broken power law (alpha_lo = theta[12] below the break
// Lorentz factor, alpha_hi above it).
constexpr int kSpecPower = 0;
constexpr int kSpecGridAlpha = 1;
constexpr int kSpecBroken = 2;

struct EmitArgs {
  int32_t alpha3;  // alpha == 3 exactly: integer powers, no log/exp
  float eI;        // (alpha + 1) / 4
  // gridded alpha: the prefactors above are those of alpha_ref = theta[12];
  // at a local alpha they scale by exp(k1_f (alpha - alpha_ref) + G(alpha) -
  // G(alpha_ref)), G = ln Gamma(alpha/4 - 1/12) + ln Gamma(alpha/4 + 19/12)
  // - ln(alpha + 1), and j_P / j_I by (alpha + 1) / (alpha + 7/3)
  double va_alpha_ref;
  double va_pref;  // (alpha_ref + 1) / (alpha_ref + 7/3)
  // G at alpha_ref in the form the device differences against: the shifted
  // Gamma arguments y = x + 6 (x = alpha/4 - 1/12 and alpha/4 + 19/12), 1/y,
  // ln y and the Stirling correction terms at them, and the product
  // Q = x1 (x1 + 1) .. (x1 + 5) x2 (x2 + 1) .. (x2 + 5) (alpha + 1)
  double va_y[2], va_iy[2], va_ly[2], va_ser[2], va_iq;  // va_iq = 1 / Q(alpha_ref)
  // broken power law: the table of spectrum.h (kBpNodes nodes of two float4:
  // the four g values, then h dg/dt) and, in powers of B_perp^2, -p_lo / 2,
  // -p_hi / 2 and (alpha_hi - alpha_lo) / 4
  const float4* bp_tab;
  float bp_h1, bp_h2, bp_q;
};

}  // namespace sm
