// Device building blocks of the sightline march (gfx950).
//
// Everything here is __host__ __device__ where it can be, so the host build of
// the library can run the same pixel and geometry code for CPU-side checks.
// Precision plan (FP32 bulk, FP64 where an error would be coherent along the
// sightline):
//   * sightline direction, step length and the step position in FP64, rounded
//     to FP32 only for the field evaluation (rounding noise is then random from
//     step to step instead of a fixed direction error);
//   * field evaluation, projections and emissivities in FP32;
//   * B_par = -B.n and the Faraday increment n_e B_par in FP64, summed in FP64;
//   * the rotation angle in turns, reduced modulo one in FP64, then FP32 sincos;
//   * the Stokes sums in FP64; physical prefactors applied once at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sm_params.h"

namespace sm {

// ---------------------------------------------------------------------------
// HEALPix: NESTED pixel -> (RING index, z, phi)  (Gorski et al. 2005 layout)
// ---------------------------------------------------------------------------

// Gathers the even bits (0, 2, 4, ...) of v into the low half.
__host__ __device__ inline uint32_t compact_even_bits(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0f0f0f0fu;
  v = (v | (v >> 4)) & 0x00ff00ffu;
  v = (v | (v >> 8)) & 0x0000ffffu;
  return v;
}

struct PixelDir {
  int64_t ring;  // RING index of the pixel
  double z;      // cos(colatitude) = sin(b)
  double s;      // sin(colatitude) = cos(b), computed without cancellation
  double phi;    // longitude l
};

// Base-face tables: ring-number offset and longitude offset of the 12 faces.
__host__ __device__ inline int face_ring_row(int f) { return 2 + (f >> 2); }
__host__ __device__ inline int face_phi_col(int f) {
  return (f < 4) ? 2 * f + 1 : (f < 8 ? 2 * (f - 4) : 2 * (f - 8) + 1);
}

__host__ __device__ inline PixelDir nest_pixel(int nside, int order, int64_t q) {
  const int64_t N = nside;
  const int64_t npf = N * N;
  const int face = (int)(q >> (2 * order));
  const uint32_t ipf = (uint32_t)(q & (npf - 1));
  const int64_t ix = compact_even_bits(ipf);
  const int64_t iy = compact_even_bits(ipf >> 1);
  const int64_t jr = (int64_t)face_ring_row(face) * N - ix - iy - 1;  // ring, 1 .. 4N-1
  int64_t nr, start;
  int kshift;
  PixelDir d;
  const double inv3n2 = 1.0 / (3.0 * (double)(N * N));
  if (jr < N) {  // north cap
    nr = jr;
    start = 2 * nr * (nr - 1);
    kshift = 0;
    const double e = (double)(nr * nr) * inv3n2;  // 1 - z
    d.z = 1.0 - e;
    d.s = sqrt(e * (2.0 - e));
  } else if (jr > 3 * N) {  // south cap
    nr = 4 * N - jr;
    start = 12 * N * N - 2 * nr * (nr + 1);
    kshift = 0;
    const double e = (double)(nr * nr) * inv3n2;
    d.z = e - 1.0;
    d.s = sqrt(e * (2.0 - e));
  } else {  // equatorial belt
    nr = N;
    start = 2 * N * (N - 1) + (jr - N) * 4 * N;
    kshift = (int)((jr - N) & 1);
    d.z = (double)(2 * N - jr) * (2.0 / (3.0 * (double)N));
    d.s = sqrt((1.0 - d.z) * (1.0 + d.z));
  }
  int64_t jp = ((int64_t)face_phi_col(face) * nr + ix - iy + 1 + kshift) / 2;
  if (jp > 4 * nr) jp -= 4 * nr;
  if (jp < 1) jp += 4 * nr;
  d.phi = ((double)jp - 0.5 * (double)(kshift + 1)) * (1.5707963267948966 / (double)nr);
  d.ring = start + jp - 1;
  return d;
}

// ---------------------------------------------------------------------------
// Sightline set-up (Sec. 2.3): direction, sky-plane basis, box exit, step.
// ---------------------------------------------------------------------------
struct Ray {
  double nx, ny, nz;     // unit direction (FP64)
  float elx, ely;        // e_l = (-sin l, cos l, 0)
  float ebx, eby, ebz;   // e_b = (-sin b cos l, -sin b sin l, cos b)
  double dkpc;           // segment length [kpc]
  int64_t ring;
};

__host__ __device__ inline Ray make_ray(const GeomArgs& g, int64_t q) {
  const PixelDir d = nest_pixel(g.nside, g.order, q);
  Ray r;
  double sl, cl;
#ifdef __HIP_DEVICE_COMPILE__
  sincos(d.phi, &sl, &cl);
#else
  sl = sin(d.phi);
  cl = cos(d.phi);
#endif
  const double cb = d.s, sb = d.z;
  r.nx = cb * cl;
  r.ny = cb * sl;
  r.nz = sb;
  r.elx = (float)(-sl);
  r.ely = (float)cl;
  r.ebx = (float)(-sb * cl);
  r.eby = (float)(-sb * sl);
  r.ebz = (float)cb;
  // distance to the first box face met along n, capped at r_max
  double t = g.r_max;
  const double n3[3] = {r.nx, r.ny, r.nz};
  for (int k = 0; k < 3; ++k) {
    if (n3[k] > 0.0) {
      const double tk = (g.box_hi[k] - g.r_obs[k]) / n3[k];
      t = tk < t ? tk : t;
    } else if (n3[k] < 0.0) {
      const double tk = (g.box_lo[k] - g.r_obs[k]) / n3[k];
      t = tk < t ? tk : t;
    }
  }
  r.dkpc = t / (double)g.n_steps;
  r.ring = d.ring;
  return r;
}

// ---------------------------------------------------------------------------
// Field values and the fields' vector-Jacobian products.
// ---------------------------------------------------------------------------
struct FV {
  float bx, by, bz;  // uG
  float ne;          // cm^-3
  float n0;          // cm^-3
};

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kRsun = 8.5f;
constexpr float kRhoMin = 1e-3f;

__device__ inline float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 16-parameter analytic model, evaluated in FP32 with host-prepared constants
// (reciprocal scale lengths pre-multiplied by log2(e)).
struct Model16 {
  M16Args p;

  __device__ inline FV eval(float x, float y, float z) const {
    const float rho = __builtin_sqrtf(x * x + y * y);
    const float rg = fmaxf(rho, kRhoMin);
    const float ir = frcp(rg);
    const float rhx = x * ir, rhy = y * ir;  // rho^
    const float az = fabsf(z);
    const float dR = rho - kRsun;
    FV v;
    const float ed = p.B0 * fexp2(-(dR * p.l2_invRB + az * p.l2_invzB));
    float sp = p.sin_psi0, cp = p.cos_psi0;
    if (p.psi1 != 0.0f) {
      const float psi = p.psi0 + p.psi1 * (flog2(rg) - p.log2_rsun) * 0.6931471805599453f;
      __sincosf(psi, &sp, &cp);
    }
    float sc = 0.0f, cc = 1.0f;
    if (p.chiB0 != 0.0f) {
      const float e2 = fexp2(-2.0f * kLog2e * az);
      const float th = copysignf((1.0f - e2) / (1.0f + e2), z);
      __sincosf(p.chiB0 * th, &sc, &cc);
    }
    const float ar = ed * sp * cc;   // rho^ coefficient
    float af = ed * cp * cc;         // phi^ coefficient
    if (p.BH0 != 0.0f) af += p.BH0 * z * p.invzH * fexp2(-(az * p.l2_invzH + dR * p.l2_invRH));
    v.bx = ar * rhx - af * rhy;
    v.by = ar * rhy + af * rhx;
    v.bz = ed * sc;
    v.n0 = p.C0 * fexp2(-(dR * p.l2_invhr + az * p.l2_invhz));
    v.ne = p.n0 * fexp2(-(az * p.l2_invhne + dR * p.l2_kappa));
    return v;
  }

  // cosmic-ray normalisation alone (grids with an analytic N0)
  __device__ inline float n0_at(float x, float y, float z) const {
    const float rho = __builtin_sqrtf(x * x + y * y);
    return p.C0 * fexp2(-((rho - kRsun) * p.l2_invhr + fabsf(z) * p.l2_invhz));
  }

  // Adds dL/dtheta given dL/d(B, n_e, N0) at (x, y, z).  tb[16] in FP64.
  __device__ inline void vjp(float x, float y, float z, const FV& g, double* tb) const {
    const float rho = __builtin_sqrtf(x * x + y * y);
    const float rg = fmaxf(rho, kRhoMin);
    const float ir = frcp(rg);
    const float rhx = x * ir, rhy = y * ir;
    const float az = fabsf(z);
    const float dR = rho - kRsun;
    const float Ed = fexp2(-(dR * p.l2_invRB + az * p.l2_invzB));
    float lnr = 0.0f, sp = p.sin_psi0, cp = p.cos_psi0;
    lnr = (flog2(rg) - p.log2_rsun) * 0.6931471805599453f;
    if (p.psi1 != 0.0f) __sincosf(p.psi0 + p.psi1 * lnr, &sp, &cp);
    const float e2 = fexp2(-2.0f * kLog2e * az);
    const float tz = copysignf((1.0f - e2) / (1.0f + e2), z);
    float sc = 0.0f, cc = 1.0f;
    if (p.chiB0 != 0.0f) __sincosf(p.chiB0 * tz, &sc, &cc);
    // project the cotangent of B on rho^, phi^, z^
    const float gr = g.bx * rhx + g.by * rhy;
    const float gf = -g.bx * rhy + g.by * rhx;
    const float gz = g.bz;
    const float bd = sp * cc * gr + cp * cc * gf + sc * gz;     // . dir
    const float bp = cp * cc * gr - sp * cc * gf;               // . d dir / d psi
    const float bc = -sp * sc * gr - cp * sc * gf + cc * gz;    // . d dir / d chi
    const float disk = p.B0 * Ed * bd;
    tb[0] += (double)(Ed * bd);
    tb[1] += (double)(p.B0 * Ed * bp);
    tb[2] += (double)(p.B0 * Ed * bp * lnr);
    tb[3] += (double)(p.B0 * Ed * bc * tz);
    tb[4] += (double)(disk * dR * p.invRB * p.invRB);
    tb[5] += (double)(disk * az * p.invzB * p.invzB);
    const float Eh = fexp2(-(az * p.l2_invzH + dR * p.l2_invRH));
    const float zq = z * p.invzH;
    tb[6] += (double)(zq * Eh * gf);
    const float hal = p.BH0 * zq * Eh * gf;
    tb[7] += (double)(p.BH0 * Eh * gf * (-z * p.invzH * p.invzH + zq * az * p.invzH * p.invzH));
    tb[8] += (double)(hal * dR * p.invRH * p.invRH);
    const float Ec = fexp2(-(dR * p.l2_invhr + az * p.l2_invhz));
    const float n0 = p.C0 * Ec;
    tb[9] += (double)(g.n0 * Ec);
    tb[10] += (double)(g.n0 * n0 * dR * p.invhr * p.invhr);
    tb[11] += (double)(g.n0 * n0 * az * p.invhz * p.invhz);
    const float En = fexp2(-(az * p.l2_invhne + dR * p.l2_kappa));
    const float ne = p.n0 * En;
    tb[13] += (double)(g.ne * En);
    tb[14] += (double)(g.ne * ne * az * p.invhne * p.invhne);
    tb[15] += (double)(-g.ne * ne * dR);
  }

  // dL/dtheta of the cosmic-ray normalisation alone (theta 9..11)
  __device__ inline void vjp_n0(float x, float y, float z, float gn0, double* tb) const {
    const float rho = __builtin_sqrtf(x * x + y * y);
    const float az = fabsf(z);
    const float dR = rho - kRsun;
    const float Ec = fexp2(-(dR * p.l2_invhr + az * p.l2_invhz));
    const float n0 = p.C0 * Ec;
    tb[9] += (double)(gn0 * Ec);
    tb[10] += (double)(gn0 * n0 * dR * p.invhr * p.invhr);
    tb[11] += (double)(gn0 * n0 * az * p.invhz * p.invhz);
  }
};

// Trilinear interpolation of node-centred grids.
struct Grid {
  GridArgs p;
  Model16 cr;  // analytic N0 when p.c == nullptr

  struct Cell {
    int64_t base;  // node index of the (0, 0, 0) corner
    float tx, ty, tz;
    bool inside;
  };

  __device__ inline Cell cell(float x, float y, float z) const {
    Cell c;
    c.inside = (x >= p.lo[0]) & (x <= p.hi[0]) & (y >= p.lo[1]) & (y <= p.hi[1]) &
               (z >= p.lo[2]) & (z <= p.hi[2]);
    // clamping before the integer conversion keeps every index in bounds, also
    // for non-finite coordinates (fmaxf/fminf return the non-NaN operand)
    const float ux = fminf(fmaxf((x - p.lo[0]) * p.inv_h[0], 0.0f), p.umax[0]);
    const float uy = fminf(fmaxf((y - p.lo[1]) * p.inv_h[1], 0.0f), p.umax[1]);
    const float uz = fminf(fmaxf((z - p.lo[2]) * p.inv_h[2], 0.0f), p.umax[2]);
    const int ix = min((int)ux, p.n[0] - 2);
    const int iy = min((int)uy, p.n[1] - 2);
    const int iz = min((int)uz, p.n[2] - 2);
    c.tx = ux - (float)ix;
    c.ty = uy - (float)iy;
    c.tz = uz - (float)iz;
    c.base = (int64_t)ix + (int64_t)p.n[0] * ((int64_t)iy + (int64_t)p.n[1] * (int64_t)iz);
    return c;
  }

  __device__ inline FV eval(float x, float y, float z) const {
    const Cell c = cell(x, y, z);
    const int64_t sy = p.n[0], sz = (int64_t)p.n[0] * p.n[1];
    const float4* g = p.bn;
    const float4 v000 = g[c.base], v100 = g[c.base + 1];
    const float4 v010 = g[c.base + sy], v110 = g[c.base + sy + 1];
    const float4 v001 = g[c.base + sz], v101 = g[c.base + sz + 1];
    const float4 v011 = g[c.base + sy + sz], v111 = g[c.base + sy + sz + 1];
    const float wx0 = 1.0f - c.tx, wy0 = 1.0f - c.ty, wz0 = 1.0f - c.tz;
    const float w00 = wy0 * wz0, w10 = c.ty * wz0, w01 = wy0 * c.tz, w11 = c.ty * c.tz;
    auto tri = [&](float a000, float a100, float a010, float a110, float a001, float a101,
                   float a011, float a111) {
      return w00 * (wx0 * a000 + c.tx * a100) + w10 * (wx0 * a010 + c.tx * a110) +
             w01 * (wx0 * a001 + c.tx * a101) + w11 * (wx0 * a011 + c.tx * a111);
    };
    FV v;
    const float in = c.inside ? 1.0f : 0.0f;
    v.bx = in * tri(v000.x, v100.x, v010.x, v110.x, v001.x, v101.x, v011.x, v111.x);
    v.by = in * tri(v000.y, v100.y, v010.y, v110.y, v001.y, v101.y, v011.y, v111.y);
    v.bz = in * tri(v000.z, v100.z, v010.z, v110.z, v001.z, v101.z, v011.z, v111.z);
    v.ne = in * tri(v000.w, v100.w, v010.w, v110.w, v001.w, v101.w, v011.w, v111.w);
    if (p.c != nullptr) {
      const float* gc = p.c;
      v.n0 = in * tri(gc[c.base], gc[c.base + 1], gc[c.base + sy], gc[c.base + sy + 1],
                      gc[c.base + sz], gc[c.base + sz + 1], gc[c.base + sy + sz],
                      gc[c.base + sy + sz + 1]);
    } else {
      v.n0 = cr.n0_at(x, y, z);
    }
    return v;
  }

  // theta-gradient of a grid field: only an analytic N0 depends on theta
  __device__ inline void vjp(float x, float y, float z, const FV& g, double* tb) const {
    if (p.c == nullptr) cr.vjp_n0(x, y, z, g.n0, tb);
  }

  // Scatters dL/d(field) at (x, y, z) onto the 8 corner nodes (atomic adds).
  __device__ inline void scatter(float x, float y, float z, const FV& g, float* gbn,
                                 float* gc) const {
    const Cell c = cell(x, y, z);
    if (!c.inside) return;
    const int64_t sy = p.n[0], sz = (int64_t)p.n[0] * p.n[1];
    const float wx[2] = {1.0f - c.tx, c.tx};
    const float wy[2] = {1.0f - c.ty, c.ty};
    const float wz[2] = {1.0f - c.tz, c.tz};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
      const float w = wx[dx] * wy[dy] * wz[dz];
      const int64_t v = c.base + dx + dy * sy + dz * sz;
      if (gbn != nullptr) {
        unsafeAtomicAdd(gbn + 4 * v + 0, w * g.bx);
        unsafeAtomicAdd(gbn + 4 * v + 1, w * g.by);
        unsafeAtomicAdd(gbn + 4 * v + 2, w * g.bz);
        unsafeAtomicAdd(gbn + 4 * v + 3, w * g.ne);
      }
      if (gc != nullptr && p.c != nullptr) unsafeAtomicAdd(gc + v, w * g.n0);
    }
  }
};

// Homogeneous sphere (Sec. 2.4 test).
struct Sphere {
  SphereArgs p;
  __device__ inline FV eval(float x, float y, float z) const {
    const float dx = x - p.c[0], dy = y - p.c[1], dz = z - p.c[2];
    const bool in = (p.r2 <= 0.0f) || (dx * dx + dy * dy + dz * dz < p.r2);
    FV v;
    v.bx = in ? p.b[0] : 0.0f;
    v.by = in ? p.b[1] : 0.0f;
    v.bz = in ? p.b[2] : 0.0f;
    v.ne = in ? p.ne : 0.0f;
    v.n0 = in ? p.n0 : 0.0f;
    return v;
  }
};

// ---------------------------------------------------------------------------
// Emission (Eqs. ji, jp): the field-dependent factors.
//   u  = N0 (B_perp^2)^{(alpha+1)/4}                        -> I
//   zc = N0 (B_perp^2)^{(alpha-3)/4} (B_l - i B_b)^2        -> (Q + iU) e^{-2i RM lambda^2}
// (B_l - i B_b)^2 / B_perp^2 = e^{2 i chi_0} with tan chi_0 = B_b / (-B_l).
// The physical prefactors (Gamma functions, nu, units, Rayleigh-Jeans) are
// applied per frequency at the end.
// ---------------------------------------------------------------------------
struct Emit {
  float u, zr, zi;
};

__device__ inline Emit emission(float n0, float bl, float bb, bool alpha3, float eI) {
  const float bt2 = bl * bl + bb * bb;
  const float cr = bl * bl - bb * bb, ci = -2.0f * bl * bb;
  Emit e;
  if (alpha3) {
    e.u = n0 * bt2;
    e.zr = n0 * cr;
    e.zi = n0 * ci;
  } else {
    float w = 0.0f, wp = 0.0f;
    if (bt2 > 0.0f) {
      w = fexp2(eI * flog2(bt2));
      wp = w * frcp(bt2);
    }
    e.u = n0 * w;
    e.zr = n0 * wp * cr;
    e.zi = n0 * wp * ci;
  }
  return e;
}

// Reverse of emission(): given dL/du and dL/d(zr, zi), returns dL/dN0, dL/dB_l,
// dL/dB_b and dL/dalpha (the exponents carry alpha).
struct EmitBar {
  float n0, bl, bb, alpha;
};

__device__ inline EmitBar emission_vjp(float n0, float bl, float bb, bool alpha3, float eI,
                                       float ub, float zrb, float zib) {
  const float bt2 = bl * bl + bb * bb;
  const float cr = bl * bl - bb * bb, ci = -2.0f * bl * bb;
  EmitBar r;
  float bt2b, crb, cib;
  if (alpha3) {
    r.n0 = ub * bt2 + zrb * cr + zib * ci;
    bt2b = ub * n0;
    crb = zrb * n0;
    cib = zib * n0;
    r.alpha = 0.0f;
    if (bt2 > 0.0f)
      r.alpha = 0.25f * 0.6931471805599453f * flog2(bt2) * n0 * (ub * bt2 + zrb * cr + zib * ci);
  } else {
    float w = 0.0f, wp = 0.0f, lg = 0.0f, ib = 0.0f;
    if (bt2 > 0.0f) {
      lg = flog2(bt2);
      w = fexp2(eI * lg);
      ib = frcp(bt2);
      wp = w * ib;
    }
    const float zdot = zrb * cr + zib * ci;
    r.n0 = ub * w + zdot * wp;
    const float wpb = n0 * zdot;
    crb = zrb * n0 * wp;
    cib = zib * n0 * wp;
    const float wb = ub * n0 + wpb * ib;
    bt2b = -wpb * wp * ib + wb * eI * wp;
    r.alpha = wb * w * lg * 0.25f * 0.6931471805599453f;
  }
  r.bl = 2.0f * bl * (bt2b + crb) - 2.0f * bb * cib;
  r.bb = 2.0f * bb * (bt2b - crb) - 2.0f * bl * cib;
  return r;
}

// sin and cos of 2 pi t for |t| <= 1/2.
__device__ inline void sincos_turns(float t, float* s, float* c) { sincospif(2.0f * t, s, c); }

// ---------------------------------------------------------------------------
// Sub-wavefront scans over groups of S consecutive lanes.
// ---------------------------------------------------------------------------
template <int S>
__device__ inline double group_inclusive_scan(double v, int sub) {
#pragma unroll
  for (int d = 1; d < S; d <<= 1) {
    const double y = __shfl_up(v, d, S);
    if (sub >= d) v += y;
  }
  return v;
}

template <int S>
__device__ inline double group_suffix_scan(double v, int sub) {
#pragma unroll
  for (int d = 1; d < S; d <<= 1) {
    const double y = __shfl_down(v, d, S);
    if (sub + d < S) v += y;
  }
  return v;
}

template <int S>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int d = S / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, S);
  return v;
}

template <int S>
__device__ inline double group_bcast(double v, int lane_in_group) {
  return (S == 1) ? v : __shfl(v, lane_in_group, S);
}

// Hardware block id -> logical block id such that consecutive logical blocks
// (neighbouring pixels) land on the same XCD and share its L2.  Blocks are
// dealt round-robin over the 8 XCDs; the map below is a bijection on [0, G).
__device__ inline int64_t xcd_block(int64_t h, int64_t G) {
  constexpr int64_t kX = 8;
  const int64_t q = G / kX, r = G % kX;
  const int64_t xcd = h % kX, slot = h / kX;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

}  // namespace sm
