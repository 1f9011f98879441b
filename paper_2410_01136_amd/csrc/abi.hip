// C ABI of the synchrotron march: argument checks, physical prefactors, launch
// shapes and dispatch.  Every check runs on the host before anything is
// launched; no exception crosses the ABI.
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/synmarch.h"
#include "batch.h"
#include "sm_device.h"
#include "sm_launch.h"
#include "tune_table.h"

namespace {

// ---- physical constants (cgs, CODATA 2018) --------------------------------
constexpr double kQe = 4.80320471e-10;        // esu
constexpr double kMe = 9.1093837015e-28;      // g
constexpr double kC = 2.99792458e10;          // cm s^-1
constexpr double kKb = 1.380649e-16;          // erg K^-1
constexpr double kKpcCm = 3.0856775814913673e21;
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_err;

syn_status fail(syn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

syn_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return SYN_EHIP;
}

bool finite3(const double* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

int ilog2_pow2(int32_t v) {
  if (v < 1 || (v & (v - 1)) != 0) return -1;
  int o = 0;
  while ((1 << o) < v) ++o;
  return o;
}

// Digamma: upward recurrence to x >= 10, then the Stirling-type asymptotic
// series in 1/x^2 (Abramowitz & Stegun 6.3.18).
double digamma_host(double x) {
  double r = 0.0;
  while (x < 10.0) {
    r -= 1.0 / x;
    x += 1.0;
  }
  const double f = 1.0 / (x * x);
  const double t = f * (-1.0 / 12 + f * (1.0 / 120 + f * (-1.0 / 252 + f * (1.0 / 240 + f * (-1.0 / 132 + f * (691.0 / 32760))))));
  return r + log(x) - 0.5 / x + t;
}

// ---- launch shapes ----------------------------------------------------------
std::atomic<int> g_lanes[3][5];  // [kernel family][field kind], 0 = default
std::atomic<int> g_grid_addressing{0};  // 0 automatic, 1 64-bit, 2 buffer per lane, 3 shared

// Built-in lanes per sightline, from autotuner runs on MI355X: small maps need
// many lanes per sightline to fill 256 CUs; large maps prefer fewer (less scan
// work, better locality).  The many-set kernels and the grid-gradient adjoint
// (which accumulates per cell in registers along consecutive steps) use 1.
int default_lanes(int kernel, int kind, int64_t npix) {
  if (kernel == SYN_KERNEL_BATCH) return 1;
  if (kernel == SYN_KERNEL_ADJOINT) {
    // contiguous pieces per sightline: eight (the fastest for both reverse
    // passes at N_side 64; with a grid gradient its wavefronts then fill the
    // chip in whole rounds), or sixteen for small maps
    if (kind == SYN_FIELD_GRID) return 8;
    return npix < (1 << 14) ? 16 : 8;
  }
  if (npix < (1 << 14)) return 64;
  // gridded fields share cell reads across the 16 steps of a sightline chunk
  if (kind == SYN_FIELD_GRID) return 16;
  return npix < (1 << 22) ? 16 : 4;
}

int lanes_for(int kernel, int kind, int64_t npix) {
  const int s = (kernel >= 0 && kernel < 3 && kind >= 0 && kind < 5) ? g_lanes[kernel][kind].load()
                                                                      : 0;
  return s > 0 ? s : default_lanes(kernel, kind, npix);
}

// Launch shape of a call: a lane count set with syn_set_lanes_per_ray wins,
// then the autotuned table for this exact shape (syn_autotune_load), then the
// built-in choice.  *grid_mode receives the table's grid read mode (0: none).
int lanes_for_shape(int kernel, int kind, int64_t npix, int steps, int freqs, int* grid_mode) {
  *grid_mode = 0;
  const int s = (kernel >= 0 && kernel < 3 && kind >= 0 && kind < 5) ? g_lanes[kernel][kind].load()
                                                                      : 0;
  int tl = 0, tm = 0;
  const bool tuned = sm::tune_lookup(kernel, kind, npix, steps, freqs, &tl, &tm);
  if (tuned) *grid_mode = tm;
  if (s > 0) return s;
  return tuned ? tl : default_lanes(kernel, kind, npix);
}

// ---- argument checks --------------------------------------------------------
syn_status check_geom(const syn_geom* g, sm::GeomArgs* ga) {
  if (g == nullptr) return fail(SYN_EINVAL, "geom is NULL");
  const int order = ilog2_pow2(g->nside);
  if (order < 0 || g->nside > SYN_MAX_NSIDE)
    return fail(SYN_EINVAL, "nside must be a power of two in [1, 8192]");
  if (g->n_steps < 1 || g->n_steps > (1 << 24)) return fail(SYN_EINVAL, "n_steps must be in [1, 2^24]");
  if (g->n_freq < 1 || g->n_freq > SYN_MAX_FREQ) return fail(SYN_EINVAL, "n_freq must be in [1, 16]");
  for (int f = 0; f < g->n_freq; ++f)
    if (!(isfinite(g->freq_hz[f]) && g->freq_hz[f] > 0.0))
      return fail(SYN_EINVAL, "frequencies must be finite and > 0");
  if (!finite3(g->r_obs_kpc)) return fail(SYN_EINVAL, "observer must be finite");
  if (!(g->r_max_kpc > 0.0)) return fail(SYN_EINVAL, "r_max must be > 0");
  bool all_faces = true;
  for (int k = 0; k < 3; ++k) {
    const double lo = g->box_lo_kpc[k], hi = g->box_hi_kpc[k];
    if (isnan(lo) || isnan(hi) || !(lo < hi)) return fail(SYN_EINVAL, "box needs lo < hi on every axis");
    if (!(g->r_obs_kpc[k] > lo && g->r_obs_kpc[k] < hi))
      return fail(SYN_EINVAL, "observer must lie strictly inside the box");
    all_faces = all_faces && isfinite(lo) && isfinite(hi);
  }
  if (!isfinite(g->r_max_kpc) && !all_faces)
    return fail(SYN_EINVAL, "an infinite r_max needs six finite box faces");
  ga->nside = g->nside;
  ga->order = order;
  ga->n_steps = g->n_steps;
  ga->npix = 12LL * g->nside * g->nside;
  for (int k = 0; k < 3; ++k) {
    ga->r_obs[k] = g->r_obs_kpc[k];
    ga->box_lo[k] = g->box_lo_kpc[k];
    ga->box_hi[k] = g->box_hi_kpc[k];
  }
  ga->r_max = g->r_max_kpc;
  return SYN_OK;
}

sm::M16Args m16_args(const double* th) {
  const double l2e = 1.4426950408889634;
  sm::M16Args m{};
  m.B0 = (float)th[0];
  m.psi0 = (float)th[1];
  m.psi1 = (float)th[2];
  m.chiB0 = (float)th[3];
  m.sin_psi0 = (float)sin(th[1]);
  m.cos_psi0 = (float)cos(th[1]);
  m.invRB = (float)(1.0 / th[4]);
  m.invzB = (float)(1.0 / th[5]);
  m.l2_invRB = (float)(l2e / th[4]);
  m.l2_invzB = (float)(l2e / th[5]);
  m.BH0 = (float)th[6];
  m.invzH = (float)(1.0 / th[7]);
  m.invRH = (float)(1.0 / th[8]);
  m.l2_invzH = (float)(l2e / th[7]);
  m.l2_invRH = (float)(l2e / th[8]);
  m.C0 = (float)th[9];
  m.invhr = (float)(1.0 / th[10]);
  m.invhz = (float)(1.0 / th[11]);
  m.l2_invhr = (float)(l2e / th[10]);
  m.l2_invhz = (float)(l2e / th[11]);
  m.n0 = (float)th[13];
  m.invhne = (float)(1.0 / th[14]);
  m.l2_invhne = (float)(l2e / th[14]);
  m.l2_kappa = (float)(l2e * th[15]);
  m.log2_rsun = (float)log2(8.5);
  return m;
}

// ---- broken power-law tables --------------------------------------------------
// syn_spectrum_table records the indices it built each table for, per device
// address; a broken-spectrum field is accepted only with a table recorded for
// its own indices.
struct SpecRecord {
  double a1, a2;
};
std::mutex g_spec_mu;
std::unordered_map<uintptr_t, SpecRecord> g_spec_tables;

void spec_record(const void* t, double a1, double a2) {
  std::lock_guard<std::mutex> lk(g_spec_mu);
  if (g_spec_tables.size() >= (1u << 16)) g_spec_tables.clear();
  g_spec_tables[(uintptr_t)t] = SpecRecord{a1, a2};
}

bool spec_matches(const void* t, double a1, double a2) {
  std::lock_guard<std::mutex> lk(g_spec_mu);
  auto it = g_spec_tables.find((uintptr_t)t);
  return it != g_spec_tables.end() && it->second.a1 == a1 && it->second.a2 == a2;
}

bool bp_alpha_ok(double a) { return a > sm::kBpAlphaMin && a <= sm::kBpAlphaMax; }

syn_status check_m16_theta(const double* th) {
  for (int k : {4, 5, 7, 8, 10, 11, 14})
    if (!(th[k] > 0.0)) return fail(SYN_EINVAL, "model16 scale lengths (theta 4,5,7,8,10,11,14) must be > 0");
  return SYN_OK;
}

syn_status check_field(const syn_field* f, sm::FieldPack* fp, bool for_adjoint) {
  if (f == nullptr) return fail(SYN_EINVAL, "field is NULL");
  for (int k = 0; k < SYN_NPARAM; ++k)
    if (!isfinite(f->theta[k])) return fail(SYN_EINVAL, "theta must be finite");
  if (!(f->theta[12] > 1.0 / 3.0))
    return fail(SYN_EINVAL, "alpha (theta[12]) must exceed 1/3, the pole of Gamma(alpha/4 - 1/12)");
  memset(fp, 0, sizeof(*fp));
  fp->kind = f->kind;
  if (!(isfinite(f->te_k) && f->te_k >= 0.0))
    return fail(SYN_EINVAL, "te_k must be finite and >= 0");
  fp->ff = f->te_k > 0.0;
  if (fp->ff && f->kind == SYN_FIELD_MLP)
    return fail(SYN_EUNSUPPORTED, "free-free (te_k > 0) is not available for the MLP surrogate");
  if (f->grid_alpha != nullptr) {
    if (f->kind != SYN_FIELD_GRID) return fail(SYN_EINVAL, "grid_alpha needs a GRID field");
    if (((uintptr_t)f->grid_alpha & 3) != 0) return fail(SYN_EINVAL, "grid_alpha must be 4-byte aligned");
  }
  if (f->spectrum != SYN_SPEC_POWER_LAW && f->spectrum != SYN_SPEC_BROKEN)
    return fail(SYN_EINVAL, "spectrum must be SYN_SPEC_POWER_LAW or SYN_SPEC_BROKEN");
  if (f->spectrum == SYN_SPEC_BROKEN) {
    if (f->grid_alpha != nullptr)
      return fail(SYN_EINVAL, "a broken power law takes its indices from theta[12] and alpha_hi, not grid_alpha");
    if (f->kind == SYN_FIELD_MLP)
      return fail(SYN_EUNSUPPORTED, "the broken power law is not available for the MLP surrogate");
    if (!bp_alpha_ok(f->theta[12]) || !bp_alpha_ok(f->alpha_hi))
      return fail(SYN_EINVAL, "broken power law: theta[12] and alpha_hi must lie in (1/3, 6]");
    if (!(f->gamma_break >= 1.0 && f->gamma_break <= 1e12))
      return fail(SYN_EINVAL, "broken power law: gamma_break must lie in [1, 1e12]");
    if (f->spectrum_table == nullptr || ((uintptr_t)f->spectrum_table & 15) != 0 ||
        !spec_matches(f->spectrum_table, f->theta[12], f->alpha_hi))
      return fail(SYN_EINVAL, "spectrum_table was not filled by syn_spectrum_table for theta[12] and alpha_hi");
    fp->spec = sm::kSpecBroken;
  }
  switch (f->kind) {
    case SYN_FIELD_MODEL16: {
      syn_status s = check_m16_theta(f->theta);
      if (s != SYN_OK) return s;
      fp->m16 = m16_args(f->theta);
      return SYN_OK;
    }
    case SYN_FIELD_GRID: {
      if (f->grid_bn == nullptr) return fail(SYN_EINVAL, "grid_bn is NULL");
      if (((uintptr_t)f->grid_bn & 15) != 0) return fail(SYN_EINVAL, "grid_bn must be 16-byte aligned");
      if (f->grid_c != nullptr && ((uintptr_t)f->grid_c & 3) != 0)
        return fail(SYN_EINVAL, "grid_c must be 4-byte aligned");
      for (int k = 0; k < 3; ++k) {
        if (f->grid_n[k] < 2 || f->grid_n[k] > (1 << 16))
          return fail(SYN_EINVAL, "grid_n must be in [2, 65536] on every axis");
        if (!(isfinite(f->grid_lo_kpc[k]) && isfinite(f->grid_hi_kpc[k]) &&
              f->grid_lo_kpc[k] < f->grid_hi_kpc[k]))
          return fail(SYN_EINVAL, "grid box needs finite lo < hi");
      }
      if ((int64_t)f->grid_n[0] * f->grid_n[1] * f->grid_n[2] > (int64_t)1 << 34)
        return fail(SYN_EINVAL, "grid too large");
      if (f->grid_c == nullptr) {
        syn_status s = check_m16_theta(f->theta);
        if (s != SYN_OK) return s;
      }
      fp->m16 = m16_args(f->theta);
      sm::GridArgs& ga = fp->grid;
      ga.bn = reinterpret_cast<const float4*>(f->grid_bn);
      ga.c = f->grid_c;
      ga.alpha = f->grid_alpha;
      for (int k = 0; k < 3; ++k) {
        ga.n[k] = f->grid_n[k];
        ga.lo[k] = f->grid_lo_kpc[k];
        ga.inv_h[k] = (double)(f->grid_n[k] - 1) / (f->grid_hi_kpc[k] - f->grid_lo_kpc[k]);
        ga.umax[k] = (double)(f->grid_n[k] - 1);
      }
      const uint64_t nx = (uint64_t)f->grid_n[0], nxy = nx * (uint64_t)f->grid_n[1];
      const uint64_t nodes = nxy * (uint64_t)f->grid_n[2];
      // 32-bit sizes and strides, used only when the whole grid fits them
      ga.bn_bytes = (uint32_t)std::min<uint64_t>(nodes * 16, 0xFFFFFFFFull);
      ga.c_bytes = (uint32_t)std::min<uint64_t>(nodes * 4, 0xFFFFFFFFull);
      ga.sy16 = (uint32_t)std::min<uint64_t>(nx * 16, 0xFFFFFFFFull);
      ga.sz16 = (uint32_t)std::min<uint64_t>(nxy * 16, 0xFFFFFFFFull);
      ga.sy4 = (uint32_t)(nx * 4);
      ga.sz4 = (uint32_t)std::min<uint64_t>(nxy * 4, 0xFFFFFFFFull);
      return SYN_OK;
    }
    case SYN_FIELD_WMAP: {
      const double* th = f->theta;
      for (int k : {10, 11, 14})
        if (!(th[k] > 0.0)) return fail(SYN_EINVAL, "WMAP scale lengths (theta 10, 11, 14) must be > 0");
      if (!(th[4] >= 0.0 && th[4] < th[5]))
        return fail(SYN_EINVAL, "WMAP ring radii need 0 <= theta[4] < theta[5]");
      sm::WmapArgs& w = fp->wmap;
      w.b0 = (float)th[0];
      w.psi0 = (float)th[1];
      w.psi1 = (float)th[2];
      w.chi0 = (float)th[3];
      w.rin = (float)th[4];
      w.rout = (float)th[5];
      w.C0 = (float)th[9];
      w.invhr = (float)(1.0 / th[10]);
      w.invhz = (float)(1.0 / th[11]);
      w.n0 = (float)th[13];
      w.invhne = (float)(1.0 / th[14]);
      w.l2_invhne = (float)(1.4426950408889634 / th[14]);
      w.l2_kappa = (float)(1.4426950408889634 * th[15]);
      return SYN_OK;
    }
    case SYN_FIELD_SPHERE: {
      if (for_adjoint) return fail(SYN_EUNSUPPORTED, "the sphere field has no adjoint");
      sm::SphereArgs& s = fp->sph;
      for (int k = 0; k < 3; ++k) {
        s.b[k] = (float)f->theta[k];
        s.c[k] = (float)f->theta[6 + k];
      }
      s.ne = (float)f->theta[3];
      s.n0 = (float)f->theta[4];
      s.r2 = f->theta[5] > 0.0 ? (float)(f->theta[5] * f->theta[5]) : 0.0f;
      return SYN_OK;
    }
    case SYN_FIELD_MLP: {
      if (for_adjoint) return fail(SYN_EUNSUPPORTED, "the MLP surrogate has no adjoint");
      if (f->mlp == nullptr || ((uintptr_t)f->mlp & 15) != 0)
        return fail(SYN_EINVAL, "mlp must be a 16-byte aligned device pointer to syn_mlp_pack output");
      for (int k = 0; k < 3; ++k)
        if (!(isfinite(f->grid_lo_kpc[k]) && isfinite(f->grid_hi_kpc[k]) &&
              f->grid_lo_kpc[k] < f->grid_hi_kpc[k]))
          return fail(SYN_EINVAL, "the MLP needs a finite normalisation box grid_lo < grid_hi");
      fp->mlp.packed = f->mlp;
      for (int k = 0; k < 3; ++k) {
        fp->mlp.lo[k] = (float)f->grid_lo_kpc[k];
        fp->mlp.scale[k] = (float)(2.0 / (f->grid_hi_kpc[k] - f->grid_lo_kpc[k]));
      }
      return SYN_OK;
    }
    default:
      return fail(SYN_EINVAL, "unknown field kind");
  }
}

// Per-frequency prefactors of the sums (Eqs. ji, jp, rm and Rayleigh-Jeans),
// and with te_k > 0 those of free-free absorption and emission: optical depth
// 0.08235 T_e^-1.35 (nu / GHz)^-2.1 per pc per (n_e / cm^-3)^2 (Mezger &
// Henderson 1967), source function T_e (Rayleigh-Jeans).
void freq_args(const syn_geom* g, double alpha, double te_k, sm::FreqArgs* fa) {
  memset(fa, 0, sizeof(*fa));
  fa->n_freq = g->n_freq;
  const double krm = kQe * kQe * kQe / (2.0 * kPi * kMe * kMe * kC * kC * kC * kC);
  const double gam = tgamma(alpha / 4.0 - 1.0 / 12.0) * tgamma(alpha / 4.0 + 19.0 / 12.0);
  const double dig = 0.25 * digamma_host(alpha / 4.0 - 1.0 / 12.0) +
                     0.25 * digamma_host(alpha / 4.0 + 19.0 / 12.0);
  for (int f = 0; f < g->n_freq; ++f) {
    const double nu = g->freq_hz[f];
    const double lam = kC / nu;
    const double base = 4.0 * kPi * nu * kMe * kC / (3.0 * kQe);
    // Eq. ji with B_perp in uG inside the sums: (1e-6 B)^{(alpha+1)/2}
    const double aI = sqrt(3.0) * kQe * kQe * kQe / (8.0 * kPi * kMe * kC * kC) *
                      pow(base, (1.0 - alpha) / 2.0) * pow(2.0, (alpha + 1.0) / 2.0) /
                      (alpha + 1.0) * gam * pow(1e-6, (alpha + 1.0) / 2.0);
    const double rj = kC * kC / (2.0 * kKb * nu * nu);
    fa->sI[f] = rj * aI * kKpcCm;
    fa->sP[f] = fa->sI[f] * (alpha + 1.0) / (alpha + 7.0 / 3.0);  // Eq. jp / Eq. ji
    fa->kappa[f] = krm * 1e-6 * kKpcCm * lam * lam / kPi;       // turns of 2 RM lambda^2
    fa->dlnsI[f] = -0.5 * log(base) + 0.5 * log(2.0) - 1.0 / (alpha + 1.0) + dig + 0.5 * log(1e-6);
    fa->dlnsP[f] = fa->dlnsI[f] + 1.0 / (alpha + 1.0) - 1.0 / (alpha + 7.0 / 3.0);
    // the part of d ln sI / d alpha outside Gamma(..) and 1 / (alpha + 1), per log2
    fa->va_k1l2[f] = (-0.5 * log(base) + 0.5 * log(2.0) + 0.5 * log(1e-6)) / log(2.0);
    if (te_k > 0.0) {
      const double kff_kpc = 1e3 * 0.08235 * pow(te_k, -1.35) * pow(nu / 1e9, -2.1);
      fa->kffl2[f] = kff_kpc / log(2.0);
      fa->tff[f] = te_k * kff_kpc;
    }
  }
}

sm::EmitArgs emit_args(double alpha) {
  sm::EmitArgs e;
  e.alpha3 = alpha == 3.0 ? 1 : 0;
  e.eI = (float)((alpha + 1.0) / 4.0);
  // reference point of a gridded alpha: the prefactors above belong to theta[12]
  e.va_alpha_ref = alpha;
  e.va_pref = (alpha + 1.0) / (alpha + 7.0 / 3.0);
  const double x[2] = {alpha / 4.0 - 1.0 / 12.0, alpha / 4.0 + 19.0 / 12.0};
  double q = alpha + 1.0;
  for (int k = 0; k < 2; ++k) {
    const double y = x[k] + 6.0, iy = 1.0 / y, iy2 = iy * iy;
    e.va_y[k] = y;
    e.va_iy[k] = iy;
    e.va_ly[k] = log(y);
    e.va_ser[k] = iy * (1.0 / 12.0 - iy2 * (1.0 / 360.0 - iy2 * (1.0 / 1260.0)));
    q *= x[k] * (x[k] + 1.0) * (x[k] + 2.0) * (x[k] + 3.0) * (x[k] + 4.0) * (x[k] + 5.0);
  }
  e.va_iq = 1.0 / q;
  return e;
}

// Broken power law: the per-frequency constants of FreqArgs and the table and
// exponents of EmitArgs.  In ln: Eq. ji's prefactor at index a without the
// factors common to both indices, with B_perp in uG (the kernels' units).
double bp_ln_prefactor(double a, double base) {
  return 0.5 * (1.0 - a) * log(base) + 0.5 * (a + 1.0) * log(2.0) - log(a + 1.0) +
         lgamma(a / 4.0 - 1.0 / 12.0) + lgamma(a / 4.0 + 19.0 / 12.0) + 0.5 * (a + 1.0) * log(1e-6);
}
// its derivative in a, and that of ln (j_P / j_I) = ln((a + 1) / (a + 7/3))
double bp_dln_prefactor(double a, double base) {
  return -0.5 * log(base) + 0.5 * log(2.0) - 1.0 / (a + 1.0) +
         0.25 * digamma_host(a / 4.0 - 1.0 / 12.0) + 0.25 * digamma_host(a / 4.0 + 19.0 / 12.0) +
         0.5 * log(1e-6);
}
double bp_dln_pol(double a) { return 1.0 / (a + 1.0) - 1.0 / (a + 7.0 / 3.0); }

syn_status bp_args(const syn_geom* g, const syn_field* f, sm::FreqArgs* fa, sm::EmitArgs* ea) {
  const double a1 = f->theta[12], a2 = f->alpha_hi, gb = f->gamma_break;
  const double p1 = sm::bp_power(a1), p2 = sm::bp_power(a2), q = 0.25 * (a2 - a1);
  ea->bp_tab = reinterpret_cast<const float4*>(f->spectrum_table);
  ea->bp_h1 = (float)(-0.5 * p1);
  ea->bp_h2 = (float)(-0.5 * p2);
  ea->bp_q = (float)q;
  const double pol = log((a2 + 1.0) / (a2 + 7.0 / 3.0)) - log((a1 + 1.0) / (a1 + 7.0 / 3.0));
  for (int k = 0; k < g->n_freq; ++k) {
    const double base = 4.0 * kPi * g->freq_hz[k] * kMe * kC / (3.0 * kQe);
    const double L = log2(base / (gb * gb * 1e-6));  // log2 of xb B_perp [uG]
    const double lr = ((a2 - a1) * log(gb) + bp_ln_prefactor(a2, base) - bp_ln_prefactor(a1, base)) / log(2.0);
    const double lrp = lr + pol / log(2.0);
    // log2 of every power the kernels form, at both ends of the B_perp range
    // they allow (B_perp^2 = 2^+-40 uG^2), must stay inside FP32's normal range
    double worst = fmax(fmax(fabs(p1 * L), fabs(p2 * L)), fmax(fabs(lr), fabs(lrp)));
    for (double lg : {-40.0, 40.0}) {
      worst = fmax(worst, fabs(p1 * (L - 0.5 * lg)));
      worst = fmax(worst, fabs(p2 * (L - 0.5 * lg)));
      worst = fmax(worst, fabs(lr + q * lg));
      worst = fmax(worst, fabs(lrp + q * lg));
    }
    if (!(worst < 120.0)) {
      char msg[160];
      snprintf(msg, sizeof(msg),
               "broken power law: the break (gamma_break %.3g) is out of the FP32 range of the "
               "kernels at %.4g Hz",
               gb, g->freq_hz[k]);
      return fail(SYN_EUNSUPPORTED, msg);
    }
    fa->bp_l[k] = (float)L;
    fa->bp_k1[k] = (float)exp2(p1 * L);
    fa->bp_k2[k] = (float)exp2(p2 * L);
    fa->bp_ri[k] = (float)exp2(lr);
    fa->bp_rp[k] = (float)exp2(lrp);
    fa->bp_dri1[k] = (float)(-log(gb) - bp_dln_prefactor(a1, base));
    fa->bp_dri2[k] = (float)(log(gb) + bp_dln_prefactor(a2, base));
    fa->bp_drp1[k] = fa->bp_dri1[k] - (float)bp_dln_pol(a1);
    fa->bp_drp2[k] = fa->bp_dri2[k] + (float)bp_dln_pol(a2);
  }
  return SYN_OK;
}

size_t ws_phi_bytes(int64_t npix) { return (size_t)((npix * 8 + 255) / 256 * 256); }

// Workspace: the Faraday sum of every sightline, with free-free also its
// emission-measure sum, then the per-block theta partials (with a broken
// spectrum, two more per block: its index above the break and ln gamma_b).
size_t ws_bytes_for(int64_t npix, bool adjoint, bool ff, bool bp) {
  if (!adjoint) return 0;
  return ws_phi_bytes(npix) * (ff ? 2 : 1) +
         (size_t)sm::march_blocks(npix, 64) * (sm::kNParam + (bp ? 2 : 0)) * sizeof(double);
}

// Piece snapshots for a reverse pass of `pieces` pieces (see GridArgs):
// quantities per piece end, and their bytes (0 when there are no pieces or they
// would take more than kMaxSnapBytes; the reverse pass then recomputes its
// pieces' sums itself).  Grid, spiral-disk and WMAP fields have reverse passes.
constexpr size_t kMaxSnapBytes = (size_t)1 << 31;
int snap_quantities(int n_freq, bool ff) { return 1 + 2 * n_freq + (ff ? 1 + 2 * n_freq : 0); }

// (a theta-only reverse pass under a broken power law interleaves steps
// instead, so its analytic and WMAP forwards store none)
bool has_snapshots(int kind, int spec) {
  return kind == SYN_FIELD_GRID ||
         ((kind == SYN_FIELD_MODEL16 || kind == SYN_FIELD_WMAP) && spec != sm::kSpecBroken);
}

// Points the field's argument block at the snapshots (nullptr: none).
void set_snapshots(sm::FieldPack* fp, int kind, double* snap, int pieces, int n_steps, int nq) {
  const int len = pieces > 0 ? (n_steps + pieces - 1) / pieces : 0;
  auto put = [&](auto& a) {
    a.snap = snap;
    a.pieces = pieces;
    a.piece_len = len;
    a.snap_nq = nq;
  };
  if (kind == SYN_FIELD_GRID) put(fp->grid);
  if (kind == SYN_FIELD_MODEL16 || kind == SYN_FIELD_WMAP) put(fp->snap);
}

size_t snap_bytes(int64_t npix, int pieces, int n_freq, bool ff) {
  if (pieces < 2) return 0;
  const size_t b = (size_t)pieces * (size_t)snap_quantities(n_freq, ff) * (size_t)npix * sizeof(double);
  return b > kMaxSnapBytes ? 0 : (b + 255) / 256 * 256;
}

// ---- workspace tags --------------------------------------------------------
// syn_forward records, per workspace address, a hash of the geometry and field
// it ran with; syn_adjoint accepts a workspace only under the same hash, so a
// workspace from another geometry, field or parameter vector (whose stored
// Faraday totals would give a silently wrong gradient), or one no forward has
// written, is refused.  Host-side only: nothing is read back from the device.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <class T>
  void add(const T& v) { bytes(&v, sizeof(v)); }
};

uint64_t ws_tag(const syn_geom* g, const syn_field* f) {
  Fnv x;
  x.add(g->nside);
  x.add(g->n_steps);
  x.bytes(g->r_obs_kpc, sizeof(g->r_obs_kpc));
  x.add(g->r_max_kpc);
  x.bytes(g->box_lo_kpc, sizeof(g->box_lo_kpc));
  x.bytes(g->box_hi_kpc, sizeof(g->box_hi_kpc));
  x.add(g->n_freq);
  x.bytes(g->freq_hz, sizeof(double) * (size_t)g->n_freq);
  x.add(f->kind);
  x.bytes(f->theta, sizeof(f->theta));
  x.bytes(f->grid_n, sizeof(f->grid_n));
  x.bytes(f->grid_lo_kpc, sizeof(f->grid_lo_kpc));
  x.bytes(f->grid_hi_kpc, sizeof(f->grid_hi_kpc));
  x.add(f->grid_bn);
  x.add(f->grid_c);
  x.add(f->mlp);
  x.add(f->te_k);
  x.add(f->grid_alpha);
  x.add(f->spectrum);
  if (f->spectrum == SYN_SPEC_BROKEN) {
    x.add(f->alpha_hi);
    x.add(f->gamma_break);
    x.add(f->spectrum_table);
  }
  return x.h;
}

// With the tag goes the piece count of the snapshots the forward stored (0:
// none).
struct WsRecord {
  uint64_t tag;
  int pieces;
};
std::mutex g_ws_mu;
std::unordered_map<uintptr_t, WsRecord> g_ws_tags;
constexpr size_t kMaxWsTags = 1u << 20;  // the table is cleared when it grows past this

void ws_record(const void* ws, uint64_t tag, int pieces) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (g_ws_tags.size() >= kMaxWsTags) g_ws_tags.clear();
  g_ws_tags[(uintptr_t)ws] = WsRecord{tag, pieces};
}

void ws_forget(const void* ws) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  g_ws_tags.erase((uintptr_t)ws);
}

// The piece count recorded with a matching tag (>= 0), or -1 for no match.
int ws_matches(const void* ws, uint64_t tag) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_ws_tags.find((uintptr_t)ws);
  if (it == g_ws_tags.end() || it->second.tag != tag) return -1;
  return it->second.pieces;
}

}  // namespace

extern "C" {

int32_t syn_version(void) { return 100; }

const char* syn_last_error(void) { return g_err.c_str(); }

size_t syn_spectrum_table_bytes(void) { return sm::kBpTableBytes; }

syn_status syn_spectrum_table_host(double alpha_lo, double alpha_hi, float* table,
                                   size_t table_bytes) {
  if (!bp_alpha_ok(alpha_lo) || !bp_alpha_ok(alpha_hi))
    return fail(SYN_EINVAL, "broken power law: indices must lie in (1/3, 6]");
  if (table == nullptr || table_bytes < sm::kBpTableBytes)
    return fail(SYN_EINVAL, "table must hold syn_spectrum_table_bytes() bytes");
  std::string err;
  if (!sm::bp_build_table(alpha_lo, alpha_hi, table, &err)) return fail(SYN_EINVAL, err);
  return SYN_OK;
}

syn_status syn_spectrum_table(double alpha_lo, double alpha_hi, void* table, size_t table_bytes,
                              hipStream_t stream) {
  if (!bp_alpha_ok(alpha_lo) || !bp_alpha_ok(alpha_hi))
    return fail(SYN_EINVAL, "broken power law: indices must lie in (1/3, 6]");
  if (table == nullptr || ((uintptr_t)table & 15) != 0 || table_bytes < sm::kBpTableBytes)
    return fail(SYN_EINVAL, "table must be a 16-byte aligned device buffer of syn_spectrum_table_bytes()");
  std::vector<float> host(sm::kBpTableBytes / sizeof(float));
  const syn_status s = syn_spectrum_table_host(alpha_lo, alpha_hi, host.data(), sm::kBpTableBytes);
  if (s != SYN_OK) return s;
  // the copy is synchronised before the host buffer goes
  hipError_t e = hipMemcpyAsync(table, host.data(), sm::kBpTableBytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "spectrum table copy");
  spec_record(table, alpha_lo, alpha_hi);
  return SYN_OK;
}

size_t syn_workspace_bytes(const syn_geom* geom, const syn_field* field, int32_t with_adjoint) {
  sm::GeomArgs ga;
  sm::FieldPack fp;
  if (check_geom(geom, &ga) != SYN_OK) return 0;
  if (check_field(field, &fp, false) != SYN_OK) return 0;
  if (with_adjoint == 0) return 0;
  size_t b = ws_bytes_for(ga.npix, true, fp.ff, fp.spec == sm::kSpecBroken);
  if (has_snapshots(field->kind, fp.spec)) {
    int tm = 0;
    const int pieces = lanes_for_shape(SYN_KERNEL_ADJOINT, field->kind, ga.npix, ga.n_steps,
                                       geom->n_freq, &tm);
    b += snap_bytes(ga.npix, pieces, geom->n_freq, fp.ff);
  }
  return b;
}

// Whether the forward may read this grid with 32-bit buffer offsets: the float4
// grid (and so the N0 grid) is under 4 GiB, (nz * ny) fits the 24-bit multiplies
// of the node index, and the cell coordinate of any point a sightline of this
// geometry reaches stays below 2^30 in magnitude (so its integer part fits).
bool grid_buffer_ok(const sm::GeomArgs& ga, const sm::GridArgs& gr) {
  const uint64_t nodes = (uint64_t)gr.n[0] * (uint64_t)gr.n[1] * (uint64_t)gr.n[2];
  if (nodes * 16 > 0xFFFFFF00ull) return false;
  if ((uint64_t)gr.n[1] * (uint64_t)gr.n[2] >= (1u << 24)) return false;
  // longest sightline: r_max, or the distance to the farthest box corner
  double corner = 0.0;
  bool faces = true;
  for (int k = 0; k < 3; ++k) {
    const double d = fmax(ga.r_obs[k] - ga.box_lo[k], ga.box_hi[k] - ga.r_obs[k]);
    faces = faces && isfinite(d);
    corner += d * d;
  }
  const double L = faces ? fmin(ga.r_max, sqrt(corner)) : ga.r_max;
  if (!isfinite(L)) return false;
  for (int k = 0; k < 3; ++k)
    if ((fabs(ga.r_obs[k] - gr.lo[k]) + L) * gr.inv_h[k] + 2.0 >= 1073741824.0) return false;
  return true;
}

syn_status syn_forward(const syn_geom* geom, const syn_field* field, float* maps, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  sm::GeomArgs ga;
  sm::FieldPack fp;
  syn_status s = check_geom(geom, &ga);
  if (s != SYN_OK) return s;
  s = check_field(field, &fp, false);
  if (s != SYN_OK) return s;
  if (maps == nullptr || ((uintptr_t)maps & 3) != 0) return fail(SYN_EINVAL, "maps must be a 4-byte aligned device pointer");
  double* phi_end = nullptr;
  double* em_end = nullptr;
  int pieces = 0;  // snapshots stored for a reverse pass of this many pieces
  if (ws != nullptr) {
    const size_t base = ws_bytes_for(ga.npix, true, fp.ff, fp.spec == sm::kSpecBroken);
    if (ws_bytes < base || ((uintptr_t)ws & 7) != 0)
      return fail(SYN_EWORKSPACE, "workspace smaller than syn_workspace_bytes(...,1) or misaligned");
    phi_end = static_cast<double*>(ws);
    if (fp.ff) em_end = reinterpret_cast<double*>(static_cast<char*>(ws) + ws_phi_bytes(ga.npix));
    if (has_snapshots(field->kind, fp.spec)) {
      int tm = 0;
      const int p = lanes_for_shape(SYN_KERNEL_ADJOINT, field->kind, ga.npix, ga.n_steps,
                                    geom->n_freq, &tm);
      const size_t sb = snap_bytes(ga.npix, p, geom->n_freq, fp.ff);
      if (sb > 0 && ws_bytes >= base + sb) {
        pieces = p;
        set_snapshots(&fp, field->kind, reinterpret_cast<double*>(static_cast<char*>(ws) + base), p,
                      ga.n_steps, snap_quantities(geom->n_freq, fp.ff));
      }
    }
  }
  sm::FreqArgs fa;
  freq_args(geom, field->theta[12], field->te_k, &fa);
  sm::EmitArgs ea = emit_args(field->theta[12]);
  if (fp.spec == sm::kSpecBroken) {
    s = bp_args(geom, field, &fa, &ea);
    if (s != SYN_OK) return s;
  }
  hipError_t e;
  if (field->kind == SYN_FIELD_MLP) {
    e = sm::launch_forward_mlp(ga, fa, ea, fp.mlp, maps, phi_end, stream);
  } else {
    int tuned_mode = 0;
    const int S = lanes_for_shape(SYN_KERNEL_FORWARD, field->kind, ga.npix, ga.n_steps,
                                  geom->n_freq, &tuned_mode);
    if (field->kind == SYN_FIELD_GRID) {
      int mode = g_grid_addressing.load();
      if (mode == 0 && tuned_mode != 0) mode = tuned_mode;
      // automatic: shared cell reads pay off once there are enough wavefronts
      // to hide their longer dependency chain (measured: N_side 256 gains 1.3x,
      // N_side 64 loses 10%)
      const bool shared = mode == 3 || (mode == 0 && ga.npix >= (1 << 18));
      fp.grid_path = (mode == 1 || !grid_buffer_ok(ga, fp.grid)) ? sm::kGridGlobal
                     : shared                                    ? sm::kGridShared
                                                                 : sm::kGridBuffer;
    }
    e = sm::launch_forward(ga, fa, ea, fp, S, maps, phi_end, em_end, stream);
  }
  if (e != hipSuccess) {
    if (ws != nullptr) ws_forget(ws);
    return hip_fail(e, "forward launch");
  }
  if (ws != nullptr) ws_record(ws, ws_tag(geom, field), pieces);
  return SYN_OK;
}

syn_status syn_adjoint(const syn_geom* geom, const syn_field* field, const float* dmaps, void* ws,
                       size_t ws_bytes, double* dtheta, float* dgrid_bn, float* dgrid_c,
                       hipStream_t stream) {
  sm::GeomArgs ga;
  sm::FieldPack fp;
  syn_status s = check_geom(geom, &ga);
  if (s != SYN_OK) return s;
  s = check_field(field, &fp, true);
  if (s != SYN_OK) return s;
  if (dmaps == nullptr || ((uintptr_t)dmaps & 3) != 0) return fail(SYN_EINVAL, "dmaps must be a 4-byte aligned device pointer");
  const bool bp = fp.spec == sm::kSpecBroken;
  if (ws == nullptr || ws_bytes < ws_bytes_for(ga.npix, true, fp.ff, bp) || ((uintptr_t)ws & 7) != 0)
    return fail(SYN_EWORKSPACE, "adjoint needs the workspace of the matching forward");
  if (field->kind != SYN_FIELD_GRID && (dgrid_bn != nullptr || dgrid_c != nullptr))
    return fail(SYN_EINVAL, "grid gradients need a GRID field");
  if (dgrid_bn != nullptr && ((uintptr_t)dgrid_bn & 3) != 0) return fail(SYN_EINVAL, "dgrid_bn misaligned");
  if (dgrid_c != nullptr && ((uintptr_t)dgrid_c & 3) != 0) return fail(SYN_EINVAL, "dgrid_c misaligned");
  if (dgrid_c != nullptr && field->kind == SYN_FIELD_GRID && field->grid_c == nullptr)
    return fail(SYN_EINVAL, "dgrid_c needs a gridded N0 (grid_c)");
  if (dtheta != nullptr && ((uintptr_t)dtheta & 7) != 0) return fail(SYN_EINVAL, "dtheta misaligned");
  const int pieces = ws_matches(ws, ws_tag(geom, field));
  if (pieces < 0)
    return fail(SYN_EWORKSPACE, "workspace was not written by a syn_forward with this geometry and field");
  if (dtheta == nullptr && dgrid_bn == nullptr && dgrid_c == nullptr) return SYN_OK;
  sm::FreqArgs fa;
  freq_args(geom, field->theta[12], field->te_k, &fa);
  sm::EmitArgs ea = emit_args(field->theta[12]);
  if (fp.spec == sm::kSpecBroken) {
    s = bp_args(geom, field, &fa, &ea);
    if (s != SYN_OK) return s;
  }
  int tuned_mode = 0;
  int S = lanes_for_shape(SYN_KERNEL_ADJOINT, field->kind, ga.npix, ga.n_steps, geom->n_freq,
                          &tuned_mode);
  char* w = static_cast<char*>(ws);
  double* phi_end = reinterpret_cast<double*>(w);
  double* em_end = fp.ff ? reinterpret_cast<double*>(w + ws_phi_bytes(ga.npix)) : nullptr;
  double* partials = reinterpret_cast<double*>(w + ws_phi_bytes(ga.npix) * (fp.ff ? 2 : 1));
  if (pieces >= 2 && has_snapshots(field->kind, fp.spec)) {
    // the forward stored the sums at the ends of `pieces` pieces: split the
    // sightlines the same way and skip the pre-pass over each piece
    S = pieces;
    set_snapshots(&fp, field->kind,
                  reinterpret_cast<double*>(w + ws_bytes_for(ga.npix, true, fp.ff, bp)), pieces,
                  ga.n_steps, snap_quantities(geom->n_freq, fp.ff));
  }
  hipError_t e = sm::launch_adjoint(ga, fa, ea, fp, S, dmaps, phi_end, em_end, partials, dtheta,
                                    dgrid_bn, dgrid_c, stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return SYN_OK;
}

size_t syn_chi2_workspace_bytes(int64_t n_pix, int32_t n_maps) {
  if (n_pix < 1 || n_maps < 1 || n_maps > 3 * SYN_MAX_FREQ) return 0;
  return (size_t)sm::chi2_partials(n_pix, n_maps) * sizeof(double);
}

syn_status syn_chi2(int64_t n_pix, int32_t n_maps, const float* maps, const float* target,
                    const double* inv_sigma2, float* dmaps, double* chi2, void* ws,
                    size_t ws_bytes, hipStream_t stream) {
  if (n_pix < 1 || n_maps < 1 || n_maps > 3 * SYN_MAX_FREQ) return fail(SYN_EINVAL, "need n_pix >= 1 and 1 <= n_maps <= 48");
  if (maps == nullptr || target == nullptr || inv_sigma2 == nullptr || chi2 == nullptr)
    return fail(SYN_EINVAL, "maps, target, inv_sigma2 and chi2 are required");
  if (((uintptr_t)chi2 & 7) != 0) return fail(SYN_EINVAL, "chi2 misaligned");
  for (int i = 0; i < n_maps; ++i)
    if (!(isfinite(inv_sigma2[i]) && inv_sigma2[i] >= 0.0)) return fail(SYN_EINVAL, "inv_sigma2 must be finite and >= 0");
  const int64_t np = sm::chi2_partials(n_pix, n_maps);
  if (ws == nullptr || ws_bytes < (size_t)np * sizeof(double) || ((uintptr_t)ws & 7) != 0)
    return fail(SYN_EWORKSPACE, "chi2 workspace smaller than syn_chi2_workspace_bytes or misaligned");
  hipError_t e = sm::launch_chi2(n_pix, n_maps, maps, target, inv_sigma2, dmaps, chi2,
                                 static_cast<double*>(ws), np, stream);
  if (e != hipSuccess) return hip_fail(e, "chi2 launch");
  return SYN_OK;
}

syn_status syn_chi2_cotangent(int64_t n_pix, int32_t n_maps, const float* maps,
                              const float* target, const double* inv_sigma2, float* dmaps,
                              double* chi2, hipStream_t stream) {
  if (n_pix < 1 || n_maps < 1 || n_maps > 3 * SYN_MAX_FREQ) return fail(SYN_EINVAL, "need n_pix >= 1 and 1 <= n_maps <= 48");
  if (n_pix > SYN_CHI2_MAX_VALUES / n_maps)
    return fail(SYN_EINVAL, "n_pix * n_maps exceeds SYN_CHI2_MAX_VALUES (2^36)");
  if (maps == nullptr || target == nullptr || inv_sigma2 == nullptr || chi2 == nullptr)
    return fail(SYN_EINVAL, "maps, target, inv_sigma2 and chi2 are required");
  if (((uintptr_t)chi2 & 7) != 0) return fail(SYN_EINVAL, "chi2 misaligned");
  for (int i = 0; i < n_maps; ++i)
    if (!(isfinite(inv_sigma2[i]) && inv_sigma2[i] >= 0.0)) return fail(SYN_EINVAL, "inv_sigma2 must be finite and >= 0");
  const int64_t np = sm::chi2_partials(n_pix, n_maps);
  if (np > sm::kChi2MaxPartials) return fail(SYN_EINVAL, "more chi2 partial sums than the static scratch holds");
  double* scratch = nullptr;
  hipError_t e = sm::chi2_scratch(&scratch);
  if (e != hipSuccess) return hip_fail(e, "chi2 scratch address");
  e = sm::launch_chi2(n_pix, n_maps, maps, target, inv_sigma2, dmaps, chi2, scratch, np, stream);
  if (e != hipSuccess) return hip_fail(e, "chi2 launch");
  return SYN_OK;
}

syn_status syn_sample_model16(const double* theta, const int32_t n[3], const double lo[3],
                              const double hi[3], float* out_bn, float* out_c,
                              hipStream_t stream) {
  if (theta == nullptr || n == nullptr || lo == nullptr || hi == nullptr) return fail(SYN_EINVAL, "NULL argument");
  for (int k = 0; k < SYN_NPARAM; ++k)
    if (!isfinite(theta[k])) return fail(SYN_EINVAL, "theta must be finite");
  syn_status s = check_m16_theta(theta);
  if (s != SYN_OK) return s;
  for (int k = 0; k < 3; ++k)
    if (n[k] < 2 || !(isfinite(lo[k]) && isfinite(hi[k]) && lo[k] < hi[k]))
      return fail(SYN_EINVAL, "grid needs >= 2 nodes and finite lo < hi per axis");
  if (out_bn != nullptr && ((uintptr_t)out_bn & 15) != 0) return fail(SYN_EINVAL, "out_bn must be 16-byte aligned");
  if (out_bn == nullptr && out_c == nullptr) return SYN_OK;
  hipError_t e = sm::launch_sample_model16(m16_args(theta), n, lo, hi, out_bn, out_c, stream);
  if (e != hipSuccess) return hip_fail(e, "sample launch");
  return SYN_OK;
}

syn_status syn_eval_fields(const syn_field* field, int64_t n, const float* xyz, float* out,
                           hipStream_t stream) {
  sm::FieldPack fp;
  syn_status s = check_field(field, &fp, false);
  if (s != SYN_OK) return s;
  if (n < 0) return fail(SYN_EINVAL, "n must be >= 0");
  if (n == 0) return SYN_OK;
  if (xyz == nullptr || out == nullptr) return fail(SYN_EINVAL, "xyz and out are required");
  hipError_t e = field->kind == SYN_FIELD_MLP ? sm::launch_eval_mlp(fp.mlp, n, xyz, out, stream)
                                              : sm::launch_eval_fields(fp, n, xyz, out, stream);
  if (e != hipSuccess) return hip_fail(e, "eval launch");
  return SYN_OK;
}

syn_status syn_set_lanes_per_ray(int32_t kernel, int32_t field_kind, int32_t lanes) {
  if (kernel < 0 || kernel > 2 || field_kind < 0 || field_kind > 4)
    return fail(SYN_EINVAL, "unknown kernel family or field kind");
  if (!(lanes == 0 || sm::lanes_valid(kernel, lanes)))
    return fail(SYN_EINVAL, kernel == SYN_KERNEL_BATCH
                                ? "lanes per sightline of the batch kernels must be 0, 1, 4, 16 or 64"
                                : "lanes per sightline must be 0, 1, 4, 8, 16 or 64");
  g_lanes[kernel][field_kind].store(lanes);
  return SYN_OK;
}

syn_status syn_adam_step(int64_t n, int32_t period, uint32_t mask, float* params,
                         const float* grads, float* m, float* v, int32_t t, double lr,
                         double beta1, double beta2, double eps, hipStream_t stream) {
  if (n < 0) return fail(SYN_EINVAL, "n must be >= 0");
  if (period < 1 || period > 32) return fail(SYN_EINVAL, "period must be in [1, 32]");
  if (t < 1) return fail(SYN_EINVAL, "t counts updates from 1");
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
    return fail(SYN_EINVAL, "beta1 and beta2 must lie in [0, 1)");
  if (!(eps >= 0.0) || !isfinite(lr)) return fail(SYN_EINVAL, "eps must be >= 0 and lr finite");
  if (n == 0) return SYN_OK;
  for (const void* ptr : {(const void*)params, (const void*)grads, (const void*)m, (const void*)v})
    if (ptr == nullptr || ((uintptr_t)ptr & 3) != 0)
      return fail(SYN_EINVAL, "params, grads, m, v must be 4-byte aligned device pointers");
  hipError_t e = sm::launch_adam(n, period, mask, params, grads, m, v, t, lr, beta1, beta2, eps,
                                 stream);
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return SYN_OK;
}

syn_status syn_set_grid_addressing(int32_t mode) {
  if (mode < 0 || mode > 3) return fail(SYN_EINVAL, "grid addressing mode must be 0, 1, 2 or 3");
  g_grid_addressing.store(mode);
  return SYN_OK;
}

int32_t syn_get_grid_addressing(void) { return g_grid_addressing.load(); }

syn_status syn_autotune_load(const char* path) {
  if (path == nullptr) return fail(SYN_EINVAL, "path is NULL");
  int kept = 0;
  std::string err;
  if (!sm::tune_load(path, &kept, &err)) return fail(SYN_EINVAL, err);
  return SYN_OK;
}

void syn_autotune_clear(void) { sm::tune_clear(); }

int32_t syn_autotune_entries(void) { return sm::tune_entries(); }

int32_t syn_autotune_lookup(int32_t kernel, int32_t field_kind, int64_t npix, int32_t n_steps,
                            int32_t n_freq, int32_t* lanes, int32_t* grid_mode) {
  int l = 0, m = 0;
  if (!sm::tune_lookup(kernel, field_kind, npix, n_steps, n_freq, &l, &m)) return 0;
  if (lanes != nullptr) *lanes = l;
  if (grid_mode != nullptr) *grid_mode = m;
  return 1;
}

const char* syn_build_id(void) { return sm::build_id(); }

int32_t syn_get_lanes_per_ray(int32_t kernel, int32_t field_kind, int64_t npix) {
  return lanes_for(kernel, field_kind, npix);
}

syn_status syn_host_nest_pixel(int32_t nside, int64_t q, int64_t* ring, double* z, double* phi) {
  const int order = ilog2_pow2(nside);
  if (order < 0 || nside > SYN_MAX_NSIDE) return fail(SYN_EINVAL, "nside must be a power of two");
  if (q < 0 || q >= 12LL * nside * nside) return fail(SYN_EINVAL, "pixel out of range");
  const sm::PixelDir d = sm::nest_pixel(nside, order, q);
  if (ring) *ring = d.ring;
  if (z) *z = d.z;
  if (phi) *phi = d.phi;
  return SYN_OK;
}

// ---- many parameter sets -----------------------------------------------------
}  // extern "C"

struct syn_batch {
  sm::BatchLaunch L{};
  std::vector<int64_t> offsets;
  std::vector<sm::BatchSet> h_sets;  // host copy of the device set table
  int32_t kind = SYN_FIELD_MODEL16;
  double freq_hz = 0.0;
  int device = 0;
  int use_graph = 1;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool captured = false;
  const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double key_inv[3] = {0, 0, 0};
};

namespace {

void batch_free(syn_batch* b) {
  if (b == nullptr) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->L.sets) hipFree(const_cast<sm::BatchSet*>(b->L.sets));
  if (b->L.counters) hipFree(b->L.counters);
  if (b->L.phi) hipFree(b->L.phi);
  if (b->L.partials) hipFree(b->L.partials);
  delete b;
}

}  // namespace

extern "C" {

namespace {

// The field, emission and frequency constants of one set from its theta.
syn_status fill_set_field(sm::BatchSet* B, const syn_geom* g, int32_t kind, const double* theta) {
  syn_field f{};
  f.kind = kind;
  memcpy(f.theta, theta, sizeof(f.theta));
  sm::FieldPack fp;
  syn_status st = check_field(&f, &fp, true);
  if (st != SYN_OK) return st;
  B->m = fp.m16;
  B->w = fp.wmap;
  sm::FreqArgs fa;
  freq_args(g, f.theta[12], 0.0, &fa);  // batch plans march without free-free
  B->fa.n_freq = 1;
  B->fa.sI[0] = fa.sI[0];
  B->fa.sP[0] = fa.sP[0];
  B->fa.kappa[0] = fa.kappa[0];
  B->fa.dlnsI[0] = fa.dlnsI[0];
  B->fa.dlnsP[0] = fa.dlnsP[0];
  B->ea = emit_args(f.theta[12]);
  return SYN_OK;
}

}  // namespace

syn_status syn_batch_create(const syn_batch_desc* desc, syn_batch** plan) {
  if (plan == nullptr) return fail(SYN_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (desc == nullptr || desc->nside == nullptr || desc->theta == nullptr)
    return fail(SYN_EINVAL, "desc, nside and theta are required");
  if (desc->n_sets < 1 || desc->n_sets > 65536) return fail(SYN_EINVAL, "n_sets must be in [1, 65536]");
  if (desc->geom.n_freq != 1) return fail(SYN_EUNSUPPORTED, "batches use exactly one frequency");
  if (desc->kind != SYN_FIELD_MODEL16 && desc->kind != SYN_FIELD_WMAP)
    return fail(SYN_EUNSUPPORTED, "batches take MODEL16 or WMAP fields");
  int64_t all_pix = 0;
  for (int s = 0; s < desc->n_sets; ++s) {
    syn_geom g = desc->geom;
    g.nside = desc->nside[s];
    sm::GeomArgs ga;
    syn_status st = check_geom(&g, &ga);
    if (st != SYN_OK) return st;
    all_pix += ga.npix;
  }
  int tuned_mode = 0;
  const int S = lanes_for_shape(SYN_KERNEL_BATCH, desc->kind, all_pix, desc->geom.n_steps, 1,
                                &tuned_mode);
  std::vector<sm::BatchSet> sets(desc->n_sets);
  std::vector<int64_t> offsets(desc->n_sets);
  int64_t total = 0, items = 0;
  for (int s = 0; s < desc->n_sets; ++s) {
    syn_geom g = desc->geom;
    g.nside = desc->nside[s];
    sm::BatchSet& B = sets[s];
    memset(&B, 0, sizeof(B));
    syn_status st = check_geom(&g, &B.g);
    if (st != SYN_OK) return st;
    st = fill_set_field(&B, &g, desc->kind, desc->theta + 16 * (int64_t)s);
    if (st != SYN_OK) return st;
    B.map_off = total;
    offsets[s] = total;
    const int64_t ni = sm::march_blocks(B.g.npix, S);
    if (items + ni > (int64_t)INT32_MAX) return fail(SYN_EINVAL, "batch too large");
    B.item0 = (int32_t)items;
    B.n_items = (int32_t)ni;
    total += B.g.npix;
    items += ni;
  }
  syn_batch* b = new syn_batch();
  b->offsets = offsets;
  b->h_sets = sets;
  b->kind = desc->kind;
  b->freq_hz = desc->geom.freq_hz[0];
  b->use_graph = desc->use_graph != 0;
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "hipGetDevice");
  }
  sm::BatchLaunch& L = b->L;
  L.S = S;
  L.wmap = desc->kind == SYN_FIELD_WMAP;
  L.n_sets = desc->n_sets;
  L.n_items = (int)items;
  L.total = total;
  sm::BatchSet* dsets = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&dsets), sizeof(sm::BatchSet) * sets.size()) != hipSuccess ||
      (L.sets = dsets, hipMalloc(reinterpret_cast<void**>(&L.counters), 2 * sizeof(unsigned int))) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&L.phi), sizeof(double) * (size_t)total) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&L.partials), sizeof(double) * 16 * (size_t)items) != hipSuccess) {
    (void)hipGetLastError();
    batch_free(b);
    return fail(SYN_ENOMEM, "device allocation of the batch plan failed");
  }
  e = hipMemcpy(dsets, sets.data(), sizeof(sm::BatchSet) * sets.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "hipMemcpy batch sets");
  }
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess || cus < 1) cus = 256;
  L.blocks_fwd = cus * sm::batch_blocks_per_cu(S, false, L.wmap);
  L.blocks_adj = cus * sm::batch_blocks_per_cu(S, true, L.wmap);
  if (b->use_graph) {
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "hipStreamCreate");
    }
  }
  *plan = b;
  return SYN_OK;
}

int64_t syn_batch_total_pixels(const syn_batch* plan) { return plan ? plan->L.total : -1; }

int64_t syn_batch_offset(const syn_batch* plan, int32_t set) {
  if (plan == nullptr || set < 0 || set >= plan->L.n_sets) return -1;
  return plan->offsets[set];
}

syn_status syn_batch_set_theta(syn_batch* plan, const double* theta, hipStream_t stream) {
  if (plan == nullptr || theta == nullptr) return fail(SYN_EINVAL, "plan and theta are required");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device) return fail(SYN_EINVAL, "plan belongs to another device");
  std::vector<sm::BatchSet> sets = plan->h_sets;
  for (size_t s = 0; s < sets.size(); ++s) {
    // the set's geometry (one frequency) is rebuilt from its stored arguments
    syn_geom g{};
    g.nside = sets[s].g.nside;
    g.n_steps = sets[s].g.n_steps;
    for (int k = 0; k < 3; ++k) {
      g.r_obs_kpc[k] = sets[s].g.r_obs[k];
      g.box_lo_kpc[k] = sets[s].g.box_lo[k];
      g.box_hi_kpc[k] = sets[s].g.box_hi[k];
    }
    g.r_max_kpc = sets[s].g.r_max;
    g.n_freq = 1;
    g.freq_hz[0] = plan->freq_hz;
    syn_status st = fill_set_field(&sets[s], &g, plan->kind, theta + 16 * (int64_t)s);
    if (st != SYN_OK) return st;  // nothing changed
  }
  // earlier work on `stream` may still read the table
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  e = hipMemcpy(const_cast<sm::BatchSet*>(plan->L.sets), sets.data(),
                sizeof(sm::BatchSet) * sets.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy of the set table");
  plan->h_sets = sets;
  return SYN_OK;
}

syn_status syn_batch_run(syn_batch* plan, const float* target, const double* inv_sigma2,
                         float* maps, float* dmaps, double* chi2, double* dtheta,
                         hipStream_t stream) {
  if (plan == nullptr) return fail(SYN_EINVAL, "plan is NULL");
  if (target == nullptr || inv_sigma2 == nullptr || maps == nullptr || dmaps == nullptr ||
      chi2 == nullptr || dtheta == nullptr)
    return fail(SYN_EINVAL, "target, inv_sigma2, maps, dmaps, chi2 and dtheta are required");
  if (((uintptr_t)chi2 & 7) != 0 || ((uintptr_t)dtheta & 7) != 0) return fail(SYN_EINVAL, "chi2/dtheta misaligned");
  for (int k = 0; k < 3; ++k)
    if (!(isfinite(inv_sigma2[k]) && inv_sigma2[k] >= 0.0)) return fail(SYN_EINVAL, "inv_sigma2 must be finite and >= 0");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device) return fail(SYN_EINVAL, "plan belongs to another device");
  sm::BatchLaunch& L = plan->L;
  L.target = target;
  for (int k = 0; k < 3; ++k) L.chi2_args.inv_s2[k] = inv_sigma2[k];
  L.maps = maps;
  L.dmaps = dmaps;
  L.chi2 = chi2;
  L.dtheta = dtheta;
  if (!plan->use_graph) {
    e = sm::launch_batch(L, stream);
    return e == hipSuccess ? SYN_OK : hip_fail(e, "batch launch");
  }
  const void* key[5] = {target, maps, dmaps, chi2, dtheta};
  bool same = plan->captured;
  for (int k = 0; k < 5 && same; ++k) same = key[k] == plan->key[k];
  for (int k = 0; k < 3 && same; ++k) same = inv_sigma2[k] == plan->key_inv[k];
  if (!same) {
    if (plan->exec) {
      hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    if (plan->graph) {
      hipGraphDestroy(plan->graph);
      plan->graph = nullptr;
    }
    plan->captured = false;
    e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = sm::launch_batch(L, plan->cap);
    e = hipStreamEndCapture(plan->cap, &plan->graph);
    if (le != hipSuccess) return hip_fail(le, "batch capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    for (int k = 0; k < 5; ++k) plan->key[k] = key[k];
    for (int k = 0; k < 3; ++k) plan->key_inv[k] = inv_sigma2[k];
    plan->captured = true;
  }
  e = hipGraphLaunch(plan->exec, stream);
  return e == hipSuccess ? SYN_OK : hip_fail(e, "hipGraphLaunch");
}

void syn_batch_destroy(syn_batch* plan) { batch_free(plan); }

}  // extern "C"
