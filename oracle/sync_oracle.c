/*
 * FP64 CPU oracle of the synchrotron sightline march -- TEST INFRASTRUCTURE.
 *
 * This file is the plain, slow, obviously-correct reference that the GPU path
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the product path never does.  It
 * shares no source, header, table or constant with the HIP library: every
 * constant below is typed here on purpose.
 *
 * What it computes (Diao et al., "synax", arXiv:2410.01136):
 *   - pixel centres of a HEALPix RING map (Gorski et al. 2005, the pixelisation
 *     the paper uses through healpy; Sec. 2.3),
 *   - the sightline from the observer to the box boundary split into N equal
 *     segments sampled at their midpoints (Sec. 2.3, the integration-point
 *     construction),
 *   - the fields B, n_e, N0 at each midpoint (analytic model or trilinear
 *     interpolation over a regular grid, Sec. 2.3),
 *   - the emissivities j_I and j_P (Eqs. ji and jp, Sec. 2.1-2.2), and, as a
     reading of the fuller CR spectrum left to future work in Sec. 2.1, those
     of a broken power law (incomplete synchrotron moments, see below),
 *   - the rotation measure as a running integral (Eq. rm) and the angle
 *     chi = RM lambda^2 + chi_0 with chi_0 from Eq. chi (Sec. 2.2),
 *   - the Riemann sums of Eq. int, then the Rayleigh-Jeans brightness
 *     temperature (maps are in Kelvin, Fig. acc_func caption).
 *   - the hand-derived reverse pass (gradient of sum(dmaps * maps) with
 *     respect to the 16 analytic parameters and to grid voxels), which the
 *     tests pin against central finite differences of this same forward.
 *
 * Readings of passages the paper leaves open:
 *   - B_LOS is signed, B_par = -B.n (positive toward the observer); the paper
 *     writes an absolute value, which would stop field reversals cancelling.
 *   - The denominator of Eq. chi is read as -B.e_l = B_x sin l - B_y cos l
 *     (the printed form is not a sky-plane component); the numerator is B.e_b.
 *   - The RM at a midpoint is the sum of all earlier segments plus half of its
 *     own segment (second-order midpoint prefix).
 *   - Units: cgs inside the physics (B in gauss, lengths in cm, N0 and n_e in
 *     cm^-3), positions in kpc, fields handed in as micro-gauss.
 *
 * Free-free emission and absorption (named as future work in Sec. 5; the paper
 * gives no formulas, so this is a reading):
 *   - opacity of a fully ionised hydrogen plasma at electron temperature T_e
 *     in the approximation of Mezger & Henderson (1967, ApJ 147, 471):
 *     d tau = 0.08235 T_e^-1.35 (nu / GHz)^-2.1 n_e^2 dl, dl in pc, n_e in cm^-3;
 *   - the thermal source function in the Rayleigh-Jeans limit is T_e, so a
 *     segment adds T_e d tau to the brightness temperature of I;
 *   - everything a segment emits (synchrotron I, Q, U and free-free) reaches the
 *     observer attenuated by e^-tau, tau the optical depth from the observer to
 *     the segment's midpoint: all earlier segments plus half of its own (the
 *     same midpoint prefix as the rotation measure).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants, cgs, CODATA 2018 -------------------------------- */
static const double OR_QE = 4.80320471e-10;      /* electron charge [esu]   */
static const double OR_ME = 9.1093837015e-28;    /* electron mass [g]       */
static const double OR_C = 2.99792458e10;        /* speed of light [cm/s]   */
static const double OR_KB = 1.380649e-16;        /* Boltzmann [erg/K]       */
static const double OR_PC = 3.0856775814913673e18; /* parsec [cm]           */
static const double OR_PI = 3.14159265358979323846;

#define OR_NPARAM 16
#define OR_MAX_FREQ 16

enum { OR_MODEL16 = 0, OR_GRID = 1, OR_SPHERE = 2, OR_WMAP = 4 };

/* Geometry and step schedule. */
typedef struct {
  int32_t nside;
  int32_t n_steps;
  double r_obs[3];     /* observer [kpc], Galactocentric Cartesian          */
  double r_max;        /* cap on the sightline length [kpc]; may be +inf    */
  double box_lo[3];    /* box faces [kpc]; +-inf allowed                    */
  double box_hi[3];
  int32_t n_freq;
  double freq_hz[OR_MAX_FREQ];
} or_geom;

/* Field description. */
typedef struct {
  int32_t kind;
  double theta[OR_NPARAM];
  int32_t grid_n[3];   /* nx, ny, nz nodes                                  */
  double grid_lo[3];   /* node-centred: first node on lo, last node on hi   */
  double grid_hi[3];
  const float* grid_bn; /* [nz][ny][nx][4] = Bx, By, Bz [uG], n_e [cm^-3]   */
  const float* grid_c;  /* [nz][ny][nx] N0 [cm^-3], or NULL -> analytic N0  */
  double te_k;          /* electron temperature [K]; > 0 adds free-free      */
  const float* grid_alpha; /* [nz][ny][nx] CR spectral index, or NULL -> theta[12] */
  int32_t spectrum;     /* OR_SPEC_POWER (index theta[12]) or OR_SPEC_BROKEN       */
  double alpha_hi;      /* broken: index above the break                           */
  double gamma_break;   /* broken: Lorentz factor of the break                     */
} or_field;

enum { OR_SPEC_POWER = 0, OR_SPEC_BROKEN = 1 };

/* ========================================================================== */
/* HEALPix RING pixel centres (Gorski et al. 2005)                           */
/* ========================================================================== */

/* Largest integer i with i*i <= v, for v >= 0. */
static int64_t or_isqrt(int64_t v) {
  int64_t r = (int64_t)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

/* Pixel p of a RING map -> (z = cos(colatitude), phi = longitude). */
void or_pix2zphi_ring(int32_t nside, int64_t p, double* z, double* phi) {
  const int64_t N = nside;
  const int64_t npix = 12 * N * N;
  const int64_t ncap = 2 * N * (N - 1);
  if (p < ncap) {
    /* north polar cap: ring i holds 4i pixels, 2i(i-1) pixels before it */
    int64_t i = (1 + or_isqrt(1 + 2 * p)) / 2;
    while (2 * i * (i - 1) > p) --i;
    while (2 * (i + 1) * i <= p) ++i;
    int64_t j = p - 2 * i * (i - 1) + 1;
    *z = 1.0 - (double)(i * i) / (3.0 * (double)(N * N));
    *phi = OR_PI / (2.0 * (double)i) * ((double)j - 0.5);
  } else if (p < npix - ncap) {
    /* equatorial belt: rings N..3N, 4N pixels each; rings alternate between
       a pixel centred on phi = 0 and a half-pixel offset */
    int64_t q = p - ncap;
    int64_t i = q / (4 * N) + N;
    int64_t j = q % (4 * N) + 1;
    double shift = ((i + N) & 1) ? 1.0 : 0.5;
    *z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * (double)N);
    *phi = OR_PI / (2.0 * (double)N) * ((double)j - shift);
  } else {
    /* south polar cap, mirror of the north cap */
    int64_t q = npix - p; /* 1-based count from the south pole end */
    int64_t i = (1 + or_isqrt(2 * q - 1)) / 2;
    while (2 * i * (i - 1) >= q) --i;
    while (2 * (i + 1) * i < q) ++i;
    int64_t j = 4 * i + 1 - (q - 2 * i * (i - 1));
    *z = -(1.0 - (double)(i * i) / (3.0 * (double)(N * N)));
    *phi = OR_PI / (2.0 * (double)i) * ((double)j - 0.5);
  }
}

/* Inverse map (z, phi) -> RING pixel, written from the zone geometry of the
   same paper; used only to pin pix2zphi by a round trip. */
int64_t or_zphi2pix_ring(int32_t nside, double z, double phi) {
  const int64_t N = nside;
  const double twopi = 2.0 * OR_PI;
  phi = fmod(phi, twopi);
  if (phi < 0) phi += twopi;
  double t = phi / (0.5 * OR_PI); /* in [0, 4) */
  double za = fabs(z);
  if (za <= 2.0 / 3.0) {
    /* belt: two families of lines of constant jp, jm cut the zone */
    int64_t jp = (int64_t)floor((double)N * (0.5 + t - 0.75 * z));
    int64_t jm = (int64_t)floor((double)N * (0.5 + t + 0.75 * z));
    int64_t ir = N + 1 + jp - jm; /* 1 .. 2N+1, counted from z = 2/3 */
    int64_t kshift = 1 - (ir & 1);
    int64_t ip = (jp + jm - N + kshift + 1) / 2;
    ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
    return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
  } else {
    double tp = t - floor(t);
    double tmp = (double)N * sqrt(3.0 * (1.0 - za));
    int64_t jp = (int64_t)floor(tp * tmp);
    int64_t jm = (int64_t)floor((1.0 - tp) * tmp);
    int64_t ir = jp + jm + 1; /* ring counted from the nearer pole */
    int64_t ip = (int64_t)floor(t * (double)ir);
    ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
    if (z > 0) return 2 * ir * (ir - 1) + ip;
    return 12 * N * N - 2 * ir * (ir + 1) + ip;
  }
}

/* Galactic longitude l and latitude b of a pixel centre; the sightline unit
   vector n = (cos b cos l, cos b sin l, sin b) with x from the Sun toward the
   Galactic centre (Sec. 2.3: pixel coordinates {l_i, b_i}). */
void or_pixel_lb(int32_t nside, int64_t p, double* l, double* b) {
  double z, phi;
  or_pix2zphi_ring(nside, p, &z, &phi);
  *l = phi;
  *b = asin(z);
}

/* ========================================================================== */
/* Sightline construction (Sec. 2.3)                                         */
/* ========================================================================== */

/* Distance from the observer to the box boundary along n, capped at r_max. */
double or_path_length(const or_geom* g, const double n[3]) {
  double t = INFINITY;
  for (int k = 0; k < 3; ++k) {
    if (n[k] > 0.0 && isfinite(g->box_hi[k])) {
      double tk = (g->box_hi[k] - g->r_obs[k]) / n[k];
      if (tk < t) t = tk;
    } else if (n[k] < 0.0 && isfinite(g->box_lo[k])) {
      double tk = (g->box_lo[k] - g->r_obs[k]) / n[k];
      if (tk < t) t = tk;
    }
  }
  return (g->r_max < t) ? g->r_max : t;
}

/* ========================================================================== */
/* Field models (Sec. 2.3: analytic callables or gridded interpolation)       */
/* ========================================================================== */

/*
 * The 16-parameter axisymmetric model of the spiral-disk test configuration.
 * theta: 0 B0[uG] 1 psi0 2 psi1 3 chiB0 4 R_B 5 z_B 6 BH0[uG] 7 z_H 8 R_H
 *        9 C0[cm^-3] 10 hr_CR 11 hz_CR 12 alpha 13 n0[cm^-3] 14 hz_ne 15 kappa_ne
 * Sun at R = 8.5 kpc.  The pitch psi is measured from the azimuthal direction,
 * tan(psi) = B_rho / B_phi; the psi1 log-radius term and the tanh(z / 1 kpc)
 * out-of-plane tilt take the forms of the paper's WMAP field (Sec. 3.1).
 */
static const double OR_RSUN = 8.5;
static const double OR_RHO_MIN = 1e-3;

void or_model16(const double* th, const double r[3], double B[3], double* ne, double* n0) {
  const double x = r[0], y = r[1], z = r[2];
  const double rho = sqrt(x * x + y * y);
  const double rg = rho > OR_RHO_MIN ? rho : OR_RHO_MIN;
  const double rhat[3] = {x / rg, y / rg, 0.0};
  const double fhat[3] = {-y / rg, x / rg, 0.0};
  const double az = fabs(z);

  const double Ed = exp(-(rho - OR_RSUN) / th[4] - az / th[5]);
  const double psi = th[1] + th[2] * log(rg / OR_RSUN);
  const double chiB = th[3] * tanh(z);
  const double sp = sin(psi), cp = cos(psi), sc = sin(chiB), cc = cos(chiB);
  const double Eh = exp(-az / th[7] - (rho - OR_RSUN) / th[8]);
  const double bh = th[6] * (z / th[7]) * Eh;
  for (int k = 0; k < 3; ++k)
    B[k] = th[0] * Ed * (sp * cc * rhat[k] + cp * cc * fhat[k]) + bh * fhat[k];
  B[2] += th[0] * Ed * sc;
  *n0 = th[9] * exp(-(rho - OR_RSUN) / th[10] - az / th[11]);
  *ne = th[13] * exp(-az / th[14] - th[15] * (rho - OR_RSUN));
}

/* Vector-Jacobian product of or_model16 with respect to theta (adds into tb). */
static void or_model16_vjp(const double* th, const double r[3], const double Bb[3], double neb,
                           double n0b, double* tb) {
  const double x = r[0], y = r[1], z = r[2];
  const double rho = sqrt(x * x + y * y);
  const double rg = rho > OR_RHO_MIN ? rho : OR_RHO_MIN;
  const double rhat[3] = {x / rg, y / rg, 0.0};
  const double fhat[3] = {-y / rg, x / rg, 0.0};
  const double zhat[3] = {0.0, 0.0, 1.0};
  const double az = fabs(z);
  const double dR = rho - OR_RSUN;

  const double Ed = exp(-dR / th[4] - az / th[5]);
  const double lnr = log(rg / OR_RSUN);
  const double psi = th[1] + th[2] * lnr;
  const double tz = tanh(z);
  const double chiB = th[3] * tz;
  const double sp = sin(psi), cp = cos(psi), sc = sin(chiB), cc = cos(chiB);
  const double Eh = exp(-az / th[7] - dR / th[8]);

  double dir[3], dpsi[3], dchi[3];
  for (int k = 0; k < 3; ++k) {
    dir[k] = sp * cc * rhat[k] + cp * cc * fhat[k] + sc * zhat[k];
    dpsi[k] = cp * cc * rhat[k] - sp * cc * fhat[k];
    dchi[k] = -sp * sc * rhat[k] - cp * sc * fhat[k] + cc * zhat[k];
  }
  double bd = 0, bp = 0, bc = 0, bf = 0;
  for (int k = 0; k < 3; ++k) {
    bd += Bb[k] * dir[k];
    bp += Bb[k] * dpsi[k];
    bc += Bb[k] * dchi[k];
    bf += Bb[k] * fhat[k];
  }
  const double disk = th[0] * Ed * bd; /* = Bbar . B_disk */
  tb[0] += Ed * bd;
  tb[1] += th[0] * Ed * bp;
  tb[2] += th[0] * Ed * bp * lnr;
  tb[3] += th[0] * Ed * bc * tz;
  tb[4] += disk * dR / (th[4] * th[4]);
  tb[5] += disk * az / (th[5] * th[5]);
  /* halo: B_H0 (z / z_H) Eh fhat */
  const double hal = th[6] * (z / th[7]) * Eh * bf; /* = Bbar . B_halo */
  tb[6] += (z / th[7]) * Eh * bf;
  tb[7] += th[6] * Eh * bf * (-z / (th[7] * th[7]) + (z / th[7]) * az / (th[7] * th[7]));
  tb[8] += hal * dR / (th[8] * th[8]);
  /* cosmic-ray normalisation */
  const double Ec = exp(-dR / th[10] - az / th[11]);
  const double n0 = th[9] * Ec;
  tb[9] += n0b * Ec;
  tb[10] += n0b * n0 * dR / (th[10] * th[10]);
  tb[11] += n0b * n0 * az / (th[11] * th[11]);
  /* thermal electrons */
  const double En = exp(-az / th[14] - th[15] * dR);
  const double ne = th[13] * En;
  tb[13] += neb * En;
  tb[14] += neb * ne * az / (th[14] * th[14]);
  tb[15] += neb * (-ne * dR);
}

/*
 * The WMAP field and cosmic-ray density of Sec. 3.1 (after Page et al. 2007):
 *   B = b0 [cos psi cos chi rho^ + sin psi cos chi phi^ + sin chi z^] for
 *   rho_in <= rho <= rho_out, with psi = psi0 + psi1 ln(rho / 8 kpc) and
 *   chi = chi0 tanh(z / 1 kpc); N0 = C0 exp(-rho / h_r) sech^2(z / h_z).
 * Outside the ring the paper sets psi and chi to zero; that would leave a
 * radial field of full strength at every other radius, so B is read as zero
 * there.  The paper's n_e (YMW16) is not available; the exponential disk of
 * the 16-parameter model stands in for it.
 * theta: 0 b0 [uG] 1 psi0 2 psi1 3 chi0 4 rho_in 5 rho_out [kpc] 9 C0 [cm^-3]
 *        10 h_r 11 h_z [kpc] 12 alpha 13 n0 [cm^-3] 14 hz_ne 15 kappa_ne
 */
static const double OR_WMAP_RREF = 8.0;

static void or_wmap(const double* th, const double r[3], double B[3], double* ne, double* n0) {
  const double x = r[0], y = r[1], z = r[2];
  const double rho = sqrt(x * x + y * y);
  B[0] = B[1] = B[2] = 0.0;
  if (rho >= th[4] && rho <= th[5] && rho > 0.0) {
    const double rhat[3] = {x / rho, y / rho, 0.0};
    const double fhat[3] = {-y / rho, x / rho, 0.0};
    const double psi = th[1] + th[2] * log(rho / OR_WMAP_RREF);
    const double chi = th[3] * tanh(z / 1.0);
    for (int k = 0; k < 3; ++k)
      B[k] = th[0] * (cos(psi) * cos(chi) * rhat[k] + sin(psi) * cos(chi) * fhat[k]);
    B[2] += th[0] * sin(chi);
  }
  const double ch = cosh(z / th[11]);
  *n0 = th[9] * exp(-rho / th[10]) / (ch * ch);
  *ne = th[13] * exp(-fabs(z) / th[14] - th[15] * (rho - OR_RSUN));
}

/* Vector-Jacobian product of or_wmap with respect to theta (adds into tb;
   the ring radii get none: the field is discontinuous there). */
static void or_wmap_vjp(const double* th, const double r[3], const double Bb[3], double neb,
                        double n0b, double* tb) {
  const double x = r[0], y = r[1], z = r[2];
  const double rho = sqrt(x * x + y * y);
  if (rho >= th[4] && rho <= th[5] && rho > 0.0) {
    const double rhat[3] = {x / rho, y / rho, 0.0};
    const double fhat[3] = {-y / rho, x / rho, 0.0};
    const double zhat[3] = {0.0, 0.0, 1.0};
    const double lnr = log(rho / OR_WMAP_RREF);
    const double psi = th[1] + th[2] * lnr;
    const double tz = tanh(z / 1.0);
    const double chi = th[3] * tz;
    const double sp = sin(psi), cp = cos(psi), sc = sin(chi), cc = cos(chi);
    double bd = 0.0, bp = 0.0, bc = 0.0;
    for (int k = 0; k < 3; ++k) {
      bd += Bb[k] * (cp * cc * rhat[k] + sp * cc * fhat[k] + sc * zhat[k]);
      bp += Bb[k] * (-sp * cc * rhat[k] + cp * cc * fhat[k]);
      bc += Bb[k] * (-cp * sc * rhat[k] - sp * sc * fhat[k] + cc * zhat[k]);
    }
    tb[0] += bd;
    tb[1] += th[0] * bp;
    tb[2] += th[0] * bp * lnr;
    tb[3] += th[0] * bc * tz;
  }
  const double u = z / th[11];
  const double ch = cosh(u);
  const double E = exp(-rho / th[10]) / (ch * ch);
  const double n0 = th[9] * E;
  tb[9] += n0b * E;
  tb[10] += n0b * n0 * rho / (th[10] * th[10]);
  tb[11] += n0b * n0 * 2.0 * tanh(u) * z / (th[11] * th[11]);
  const double dR = rho - OR_RSUN;
  const double En = exp(-fabs(z) / th[14] - th[15] * dR);
  const double ne = th[13] * En;
  tb[13] += neb * En;
  tb[14] += neb * ne * fabs(z) / (th[14] * th[14]);
  tb[15] += neb * (-ne * dR);
}

/* Homogeneous sphere (Sec. 2.4 test): uniform fields within radius R0 of a
   centre, zero outside.  theta: 0-2 B [uG], 3 n_e, 4 N0, 5 R0 [kpc] (<= 0 means
   everywhere), 6-8 centre [kpc], 12 alpha. */
static void or_sphere(const double* th, const double r[3], double B[3], double* ne, double* n0) {
  int inside = 1;
  if (th[5] > 0.0) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) d2 += (r[k] - th[6 + k]) * (r[k] - th[6 + k]);
    inside = d2 < th[5] * th[5];
  }
  for (int k = 0; k < 3; ++k) B[k] = inside ? th[k] : 0.0;
  *ne = inside ? th[3] : 0.0;
  *n0 = inside ? th[4] : 0.0;
}

/* Trilinear cell lookup on a node-centred grid.  Returns 0 outside the grid
   box (fields are zero there), else fills the base node index and the eight
   corner weights in the order (dx, dy, dz) = bit (0, 1, 2) of the corner. */
static int or_grid_cell(const or_field* f, const double r[3], int64_t* base, int64_t stride[3],
                        double w[8]) {
  double t[3];
  int64_t i[3];
  for (int k = 0; k < 3; ++k) {
    if (!(r[k] >= f->grid_lo[k] && r[k] <= f->grid_hi[k])) return 0;
    const int64_t n = f->grid_n[k];
    const double u = (r[k] - f->grid_lo[k]) / (f->grid_hi[k] - f->grid_lo[k]) * (double)(n - 1);
    int64_t i0 = (int64_t)floor(u);
    if (i0 < 0) i0 = 0;
    if (i0 > n - 2) i0 = n - 2;
    i[k] = i0;
    t[k] = u - (double)i0;
  }
  stride[0] = 1;
  stride[1] = f->grid_n[0];
  stride[2] = (int64_t)f->grid_n[0] * f->grid_n[1];
  *base = i[0] + i[1] * stride[1] + i[2] * stride[2];
  for (int c = 0; c < 8; ++c) {
    double wc = 1.0;
    for (int k = 0; k < 3; ++k) wc *= ((c >> k) & 1) ? t[k] : 1.0 - t[k];
    w[c] = wc;
  }
  return 1;
}

static int64_t or_corner(int64_t base, const int64_t s[3], int c) {
  return base + ((c & 1) ? s[0] : 0) + ((c & 2) ? s[1] : 0) + ((c & 4) ? s[2] : 0);
}

/* Field values at r: B [uG], n_e and N0 [cm^-3]. */
void or_fields(const or_field* f, const double r[3], double B[3], double* ne, double* n0) {
  if (f->kind == OR_MODEL16) {
    or_model16(f->theta, r, B, ne, n0);
  } else if (f->kind == OR_WMAP) {
    or_wmap(f->theta, r, B, ne, n0);
  } else if (f->kind == OR_SPHERE) {
    or_sphere(f->theta, r, B, ne, n0);
  } else {
    int64_t base, s[3];
    double w[8];
    B[0] = B[1] = B[2] = 0.0;
    *ne = 0.0;
    *n0 = 0.0;
    double Bm[3], nem, n0m;
    if (f->grid_c == NULL) { /* analytic cosmic-ray normalisation */
      or_model16(f->theta, r, Bm, &nem, &n0m);
      *n0 = n0m;
    }
    if (!or_grid_cell(f, r, &base, s, w)) {
      if (f->grid_c != NULL) *n0 = 0.0;
      return;
    }
    for (int c = 0; c < 8; ++c) {
      const int64_t v = or_corner(base, s, c);
      for (int k = 0; k < 3; ++k) B[k] += w[c] * (double)f->grid_bn[4 * v + k];
      *ne += w[c] * (double)f->grid_bn[4 * v + 3];
      if (f->grid_c != NULL) *n0 += w[c] * (double)f->grid_c[v];
    }
  }
}

/* Power-law index of the CR spectrum at r: theta[12], or for a grid field with
   a gridded index its trilinear interpolation (Eqs. ji and jp then use the
   local value; a spatially varying index is the first step toward the full
   CR spectrum the paper leaves to future work, Sec. 2.1).  Outside the grid
   box the fields vanish and the index is not used. */
double or_alpha_at(const or_field* f, const double r[3]) {
  if (f->kind != OR_GRID || f->grid_alpha == NULL) return f->theta[12];
  int64_t base, s[3];
  double w[8];
  if (!or_grid_cell(f, r, &base, s, w)) return f->theta[12];
  double a = 0.0;
  for (int c = 0; c < 8; ++c) a += w[c] * (double)f->grid_alpha[or_corner(base, s, c)];
  return a;
}

/* ========================================================================== */
/* Emissivities (Sec. 2.1 Eq. ji, Sec. 2.2 Eq. jp)                           */
/* ========================================================================== */

/* Eq. ji, literally, in cgs: B_trans [gauss], N0 [cm^-3], nu [Hz]. */
double or_j_I(double alpha, double nu, double bt, double n0) {
  if (bt <= 0.0) return 0.0;
  const double pre = sqrt(3.0) * pow(OR_QE, 3) * bt * n0 / (8.0 * OR_PI * OR_ME * OR_C * OR_C);
  const double brk = pow(4.0 * OR_PI * nu * OR_ME * OR_C / (3.0 * OR_QE * bt), (1.0 - alpha) / 2.0);
  return pre * brk * pow(2.0, (alpha + 1.0) / 2.0) / (alpha + 1.0) *
         tgamma(alpha / 4.0 - 1.0 / 12.0) * tgamma(alpha / 4.0 + 19.0 / 12.0);
}

/* Eq. jp, literally. */
double or_j_P(double alpha, double nu, double bt, double n0) {
  if (bt <= 0.0) return 0.0;
  const double pre = sqrt(3.0) * pow(OR_QE, 3) * bt * n0 / (8.0 * OR_PI * OR_ME * OR_C * OR_C);
  const double brk = pow(4.0 * OR_PI * nu * OR_ME * OR_C / (3.0 * OR_QE * bt), (1.0 - alpha) / 2.0);
  return pre * brk * pow(2.0, (alpha - 3.0) / 2.0) * tgamma(alpha / 4.0 - 1.0 / 12.0) *
         tgamma(alpha / 4.0 + 7.0 / 12.0);
}

/* ========================================================================== */
/* Broken power-law CR spectrum (Sec. 2.1 leaves spectra beyond one power    */
/* law to future work; this is a reading)                                    */
/* ========================================================================== */
/*
 * N(gamma) = C gamma^-a1 below the Lorentz factor gamma_b and
 * C gamma_b^(a2 - a1) gamma^-a2 above it (continuous at gamma_b; C = N0 as in
 * Eq. ji).  The emissivity is the single-electron spectrum integrated over the
 * electrons, j = (1 / 4 pi) int N(gamma) P(nu, gamma) dgamma, with
 * P = sqrt(3) q^3 B / (m c^2) F(nu / nu_c), nu_c = 3 gamma^2 q B / (4 pi m c)
 * (and G in place of F for the polarised part).  In x = nu / nu_c, gamma^2 =
 * x0 / x with x0 = 4 pi nu m c / (3 q B): electrons below the break emit at
 * x > xb = x0 / gamma_b^2.  For one power law of index a the integral is the
 * complete x-moment of F of order mu = (a - 3) / 2, which gives Eq. ji (and
 * Eq. jp for G).  For the broken law each segment is an incomplete moment:
 *
 *   j_I = j_I(a1) T_F(a1, xb) + gamma_b^(a2 - a1) j_I(a2) (1 - T_F(a2, xb)),
 *   j_P = the same with j_P and T_G,
 *
 * T(a, xb) = int_xb^inf x^mu F(x) dx / int_0^inf x^mu F(x) dx, the share of the
 * moment above xb.  With F(x) = x int_0^inf e^{-x cosh s} cosh(5s/3)/cosh s ds
 * and G(x) = x K_2/3(x) = x int_0^inf e^{-x cosh s} cosh(2s/3) ds, the x-integral
 * over [xb, inf) of x^(mu+1) e^{-x cosh s} is Gamma(mu + 2, xb cosh s) /
 * cosh^(mu+2) s, so
 *
 *   int_xb^inf x^mu F = int_0^inf cosh(5s/3) cosh^-(mu+3) s Gamma(mu+2, xb cosh s) ds
 *   int_xb^inf x^mu G = int_0^inf cosh(2s/3) cosh^-(mu+2) s Gamma(mu+2, xb cosh s) ds,
 *
 * taken by the trapezoidal rule in s (the integrands are even and analytic in
 * the strip |Im s| < pi/2, so the rule converges geometrically), while the
 * complete moments are the closed forms behind Eqs. ji and jp.
 */

/* Upper incomplete gamma function Gamma(a, y), a > 0, y >= 0: Gamma(a) less
   the power series of the lower function for y < a + 1, else Legendre's
   continued fraction in its even form, evaluated by the modified Lentz
   method. */
double or_gamma_upper(double a, double y) {
  if (y <= 0.0) return tgamma(a);
  if (y < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int k = 1; k < 2000; ++k) {
      term *= y / (a + k);
      sum += term;
      if (term < 1e-17 * sum) break;
    }
    return tgamma(a) - sum * exp(a * log(y) - y);
  }
  const double tiny = 1e-300;
  double b = y + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 2000; ++i) {
    const double an = -(double)i * ((double)i - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return exp(a * log(y) - y) * h;
}

/* Trapezoidal step in s and the cut: terms with x (cosh s - 1) > 60 are below
   e^-60 of the first and are dropped. */
static const double OR_S_STEP = 0.125;
static const double OR_S_CUT = 60.0;

/* Synchrotron functions F(x) = x int_x^inf K_5/3 and G(x) = x K_2/3(x). */
double or_synch_F(double x) {
  if (!(x > 0.0)) return 0.0;
  double sum = 0.0;
  for (int k = 0;; ++k) {
    const double s = k * OR_S_STEP, ch = cosh(s);
    if (x * (ch - 1.0) > OR_S_CUT) break;
    const double t = exp(-x * ch) * cosh(5.0 * s / 3.0) / ch;
    sum += (k == 0 ? 0.5 : 1.0) * t;
  }
  return x * OR_S_STEP * sum;
}

double or_synch_G(double x) {
  if (!(x > 0.0)) return 0.0;
  double sum = 0.0;
  for (int k = 0;; ++k) {
    const double s = k * OR_S_STEP, ch = cosh(s);
    if (x * (ch - 1.0) > OR_S_CUT) break;
    sum += (k == 0 ? 0.5 : 1.0) * exp(-x * ch) * cosh(2.0 * s / 3.0);
  }
  return x * OR_S_STEP * sum;
}

/* Complete moments int_0^inf x^mu F(x) dx and int_0^inf x^mu G(x) dx, the
   Gamma-function factors of Eqs. ji and jp at mu = (alpha - 3) / 2. */
double or_moment_F(double mu) {
  return pow(2.0, mu + 1.0) / (mu + 2.0) * tgamma(mu / 2.0 + 7.0 / 3.0) * tgamma(mu / 2.0 + 2.0 / 3.0);
}
double or_moment_G(double mu) {
  return pow(2.0, mu) * tgamma(mu / 2.0 + 4.0 / 3.0) * tgamma(mu / 2.0 + 2.0 / 3.0);
}

/* Shares of the x-moments of order mu = (alpha - 3) / 2 of F and G that lie
   above xb: tF, tG in [0, 1] (1 at xb = 0, 0 as xb -> inf). */
void or_moment_tails(double alpha, double xb, double* tF, double* tG) {
  if (!(xb > 0.0)) {
    *tF = *tG = 1.0;
    return;
  }
  if (isinf(xb)) {
    *tF = *tG = 0.0;
    return;
  }
  const double mu = 0.5 * (alpha - 3.0), a = mu + 2.0;
  double sF = 0.0, sG = 0.0;
  for (int k = 0;; ++k) {
    const double s = k * OR_S_STEP, ch = cosh(s);
    if (xb * (ch - 1.0) > OR_S_CUT) break;
    const double w = (k == 0 ? 0.5 : 1.0) * or_gamma_upper(a, xb * ch) * pow(ch, -a);
    sF += w * cosh(5.0 * s / 3.0) / ch;
    sG += w * cosh(2.0 * s / 3.0);
  }
  *tF = OR_S_STEP * sF / or_moment_F(mu);
  *tG = OR_S_STEP * sG / or_moment_G(mu);
}

/* Emissivities of the broken power law (a1 below the break Lorentz factor gb,
   a2 above it) at B_trans bt [gauss], N0 [cm^-3], nu [Hz]:
   out = {j_I, j_P, d j_I / d bt, d j_P / d bt}. */
void or_j_broken(double a1, double a2, double gb, double nu, double bt, double n0, double out[4]) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  if (bt <= 0.0) return;
  const double xb = 4.0 * OR_PI * nu * OR_ME * OR_C / (3.0 * OR_QE * bt * gb * gb);
  const double norm2 = pow(gb, a2 - a1);
  const double jI1 = or_j_I(a1, nu, bt, n0), jP1 = or_j_P(a1, nu, bt, n0);
  const double jI2 = norm2 * or_j_I(a2, nu, bt, n0), jP2 = norm2 * or_j_P(a2, nu, bt, n0);
  double tF1, tG1, tF2, tG2;
  or_moment_tails(a1, xb, &tF1, &tG1);
  or_moment_tails(a2, xb, &tF2, &tG2);
  out[0] = jI1 * tF1 + jI2 * (1.0 - tF2);
  out[1] = jP1 * tG1 + jP2 * (1.0 - tG2);
  /* each j(a) grows as bt^((a+1)/2); xb falls as 1/bt, and the tail share
     above xb changes by -xb^mu F(xb) / moment per unit xb */
  const double mu1 = 0.5 * (a1 - 3.0), mu2 = 0.5 * (a2 - 3.0);
  const double FF = or_synch_F(xb), GG = or_synch_G(xb);
  const double dtF1 = pow(xb, mu1 + 1.0) * FF / (or_moment_F(mu1) * bt);
  const double dtG1 = pow(xb, mu1 + 1.0) * GG / (or_moment_G(mu1) * bt);
  const double dtF2 = pow(xb, mu2 + 1.0) * FF / (or_moment_F(mu2) * bt);
  const double dtG2 = pow(xb, mu2 + 1.0) * GG / (or_moment_G(mu2) * bt);
  out[2] = jI1 * ((a1 + 1.0) / (2.0 * bt) * tF1 + dtF1) +
           jI2 * ((a2 + 1.0) / (2.0 * bt) * (1.0 - tF2) - dtF2);
  out[3] = jP1 * ((a1 + 1.0) / (2.0 * bt) * tG1 + dtG1) +
           jP2 * ((a2 + 1.0) / (2.0 * bt) * (1.0 - tG2) - dtG2);
}

/* Derivatives of (j_I, j_P) of the broken power law with respect to its
   parameters (a1, a2, ln gb): dI[3], dP[3].  The shares' dependence on the
   indices has no elementary form, so all three are taken numerically:
   central differences at steps h and h/2 combined by Richardson
   extrapolation, (4 D(h/2) - D(h)) / 3, error O(h^4). */
void or_dj_broken(double a1, double a2, double gb, double nu, double bt, double n0, double dI[3],
                  double dP[3]) {
  const double h = 1e-3;
  for (int k = 0; k < 3; ++k) {
    double d[2][2];
    for (int r = 0; r < 2; ++r) {
      const double hh = r == 0 ? h : 0.5 * h;
      double jp[4], jm[4];
      const double pa[3] = {k == 0 ? hh : 0.0, k == 1 ? hh : 0.0, k == 2 ? hh : 0.0};
      or_j_broken(a1 + pa[0], a2 + pa[1], gb * exp(pa[2]), nu, bt, n0, jp);
      or_j_broken(a1 - pa[0], a2 - pa[1], gb * exp(-pa[2]), nu, bt, n0, jm);
      d[r][0] = (jp[0] - jm[0]) / (2.0 * hh);
      d[r][1] = (jp[1] - jm[1]) / (2.0 * hh);
    }
    dI[k] = (4.0 * d[1][0] - d[0][0]) / 3.0;
    dP[k] = (4.0 * d[1][1] - d[0][1]) / 3.0;
  }
}

/* Emissivities of the spectrum of f (NULL: one power law) at index alpha
   (theta[12] or the local gridded index): out as for or_j_broken. */
static void or_emissivity(const or_field* f, double alpha, double nu, double bt, double n0,
                          double out[4]) {
  if (f != NULL && f->spectrum == OR_SPEC_BROKEN) {
    or_j_broken(alpha, f->alpha_hi, f->gamma_break, nu, bt, n0, out);
    return;
  }
  out[0] = or_j_I(alpha, nu, bt, n0);
  out[1] = or_j_P(alpha, nu, bt, n0);
  out[2] = bt > 0.0 ? out[0] * (alpha + 1.0) / (2.0 * bt) : 0.0;
  out[3] = bt > 0.0 ? out[1] * (alpha + 1.0) / (2.0 * bt) : 0.0;
}

/* Digamma by upward recurrence to x >= 12 and the asymptotic series
   psi(x) = ln x - 1/(2x) - sum_k B_2k / (2k x^2k) (Abramowitz & Stegun 6.3.18). */
double or_digamma(double x) {
  double acc = 0.0;
  while (x < 12.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double x2 = 1.0 / (x * x);
  const double series =
      x2 * (1.0 / 12.0 - x2 * (1.0 / 120.0 - x2 * (1.0 / 252.0 - x2 * (1.0 / 240.0 - x2 * (1.0 / 132.0)))));
  return acc + log(x) - 0.5 / x - series;
}

/* d ln j_I / d alpha and d ln j_P / d alpha at fixed B_trans [gauss]; the
   bracket of Eqs. ji/jp already holds B_trans, so no separate ln B term. */
static void or_dlnj_dalpha(double alpha, double nu, double bt, double* dI, double* dP) {
  const double lb = log(4.0 * OR_PI * nu * OR_ME * OR_C / (3.0 * OR_QE * bt));
  const double common = -0.5 * lb + 0.25 * or_digamma(alpha / 4.0 - 1.0 / 12.0);
  *dI = common + 0.5 * log(2.0) - 1.0 / (alpha + 1.0) + 0.25 * or_digamma(alpha / 4.0 + 19.0 / 12.0);
  *dP = common + 0.5 * log(2.0) + 0.25 * or_digamma(alpha / 4.0 + 7.0 / 12.0);
}

/* Rotation-measure constant of Eq. rm, q^3 / (2 pi m^2 c^4), cgs. */
double or_k_rm(void) { return pow(OR_QE, 3) / (2.0 * OR_PI * OR_ME * OR_ME * pow(OR_C, 4)); }

/* Rayleigh-Jeans conversion of a specific intensity to Kelvin. */
double or_rj(double nu) { return OR_C * OR_C / (2.0 * OR_KB * nu * nu); }

/* Free-free optical depth per pc per (n_e / cm^-3)^2 at frequency nu [Hz] and
   electron temperature te [K] (Mezger & Henderson 1967 approximation). */
double or_kff(double nu, double te) { return 0.08235 * pow(te, -1.35) * pow(nu / 1e9, -2.1); }

/* ========================================================================== */
/* One sightline                                                              */
/* ========================================================================== */

typedef struct {
  double nhat[3], el[3], eb[3];
  double L, dkpc, dcm;
} or_ray;

static void or_make_ray(const or_geom* g, int64_t p, or_ray* ray) {
  double l, b;
  or_pixel_lb(g->nside, p, &l, &b);
  ray->nhat[0] = cos(b) * cos(l);
  ray->nhat[1] = cos(b) * sin(l);
  ray->nhat[2] = sin(b);
  ray->el[0] = -sin(l);
  ray->el[1] = cos(l);
  ray->el[2] = 0.0;
  ray->eb[0] = -sin(b) * cos(l);
  ray->eb[1] = -sin(b) * sin(l);
  ray->eb[2] = cos(b);
  ray->L = or_path_length(g, ray->nhat);
  ray->dkpc = ray->L / (double)g->n_steps;
  ray->dcm = ray->dkpc * 1e3 * OR_PC;
}

static void or_midpoint(const or_geom* g, const or_ray* ray, int n, double r[3]) {
  const double s = ((double)n + 0.5) * ray->dkpc; /* n is 0-based here */
  for (int k = 0; k < 3; ++k) r[k] = g->r_obs[k] + s * ray->nhat[k];
}

/* Per-step local quantities the sums need. */
typedef struct {
  double Bt;     /* |B_trans| [gauss]                      */
  double num;    /* B . e_b [gauss]  (numerator of Eq. chi) */
  double den;    /* -B . e_l [gauss] (denominator, reading) */
  double blos;   /* -B . n [gauss]                          */
  double ne, n0; /* [cm^-3]                                 */
  double chi0;
} or_local;

/* Field values at midpoint n of a sightline: either a field model evaluated at
   the midpoint r, or a table of samples given by the caller. */
typedef struct {
  const or_field* f;       /* field model, or NULL for a table */
  const double* table;     /* [n_steps][5] = Bx, By, Bz [uG], n_e, N0 */
} or_source;

static void or_source_eval(const or_source* src, int n, const double r[3], double B[3], double* ne,
                           double* n0) {
  if (src->f != NULL) {
    or_fields(src->f, r, B, ne, n0);
  } else {
    const double* v = src->table + 5 * (int64_t)n;
    B[0] = v[0];
    B[1] = v[1];
    B[2] = v[2];
    *ne = v[3];
    *n0 = v[4];
  }
}

static void or_local_from(const or_ray* ray, const double B[3], double ne, double n0, or_local* q) {
  double bl = 0, bb = 0, bn = 0;
  for (int k = 0; k < 3; ++k) {
    bl += B[k] * ray->el[k];
    bb += B[k] * ray->eb[k];
    bn += B[k] * ray->nhat[k];
  }
  q->num = 1e-6 * bb;
  q->den = -1e-6 * bl;
  q->blos = -1e-6 * bn;
  q->Bt = sqrt(q->num * q->num + q->den * q->den);
  q->ne = ne;
  q->n0 = n0;
  q->chi0 = atan2(q->num, q->den);
}

static void or_local_eval(const or_field* f, const or_ray* ray, const double r[3], or_local* q) {
  double B[3], ne, n0;
  or_fields(f, r, B, &ne, &n0);
  or_local_from(ray, B, ne, n0, q);
}

/* Forward march of one pixel: out[f][3] = T_I, T_Q, T_U [K]; returns the
   total Faraday depth sum of the segment increments [rad cm^-2]. */
static double or_march_source(const or_geom* g, const or_source* src, double alpha, double te,
                              int64_t p, double* out) {
  or_ray ray;
  or_make_ray(g, p, &ray);
  const double krm = or_k_rm();
  const double dpc = ray.dkpc * 1e3;
  double I[OR_MAX_FREQ] = {0}, Q[OR_MAX_FREQ] = {0}, U[OR_MAX_FREQ] = {0};
  double F[OR_MAX_FREQ] = {0}; /* free-free: sum of e^-tau n_e^2 dl */
  double rm_before = 0.0;      /* integral of n_e B_LOS over all earlier segments */
  double em_before = 0.0;      /* emission measure of all earlier segments [pc cm^-6] */
  for (int n = 0; n < g->n_steps; ++n) {
    double r[3];
    or_midpoint(g, &ray, n, r);
    double B[3], ne, n0;
    or_source_eval(src, n, r, B, &ne, &n0);
    or_local q;
    or_local_from(&ray, B, ne, n0, &q);
    const double seg = q.ne * q.blos * ray.dcm;
    const double RM = krm * (rm_before + 0.5 * seg);
    rm_before += seg;
    const double em_seg = te > 0.0 ? q.ne * q.ne * dpc : 0.0;
    const double EM = em_before + 0.5 * em_seg;
    em_before += em_seg;
    const double a_n = src->f != NULL ? or_alpha_at(src->f, r) : alpha;
    for (int k = 0; k < g->n_freq; ++k) {
      const double nu = g->freq_hz[k];
      const double lam = OR_C / nu;
      const double att = te > 0.0 ? exp(-or_kff(nu, te) * EM) : 1.0;
      double j[4];
      or_emissivity(src->f, a_n, nu, q.Bt, q.n0, j);
      const double jI = j[0], jP = j[1];
      const double chi = RM * lam * lam + q.chi0;
      I[k] += att * jI * ray.dcm;
      Q[k] += att * jP * cos(2.0 * chi) * ray.dcm;
      U[k] += att * jP * sin(2.0 * chi) * ray.dcm;
      F[k] += att * em_seg;
    }
  }
  for (int k = 0; k < g->n_freq; ++k) {
    const double rj = or_rj(g->freq_hz[k]);
    const double tff = te > 0.0 ? te * or_kff(g->freq_hz[k], te) * F[k] : 0.0;
    out[3 * k + 0] = rj * I[k] + tff;
    out[3 * k + 1] = rj * Q[k];
    out[3 * k + 2] = rj * U[k];
  }
  return krm * rm_before;
}

static double or_march_pixel(const or_geom* g, const or_field* f, int64_t p, double* out) {
  const or_source src = {f, NULL};
  return or_march_source(g, &src, f->theta[12], f->te_k, p, out);
}

static int or_check(const or_geom* g, const or_field* f) {
  if (g->nside < 1 || g->n_steps < 1 || g->n_freq < 1 || g->n_freq > OR_MAX_FREQ) return -1;
  if (f->kind != OR_MODEL16 && f->kind != OR_GRID && f->kind != OR_SPHERE && f->kind != OR_WMAP)
    return -1;
  if (f->kind == OR_GRID && (f->grid_bn == NULL || f->grid_n[0] < 2 || f->grid_n[1] < 2 ||
                             f->grid_n[2] < 2))
    return -1;
  if (!(f->te_k >= 0.0) || isinf(f->te_k)) return -1;
  if (f->grid_alpha != NULL && f->kind != OR_GRID) return -1;
  if (f->spectrum != OR_SPEC_POWER && f->spectrum != OR_SPEC_BROKEN) return -1;
  if (f->spectrum == OR_SPEC_BROKEN) {
    /* the moments exist for indices above 1/3; one index per side of the break */
    if (f->grid_alpha != NULL || !(f->theta[12] > 1.0 / 3.0) || !(f->alpha_hi > 1.0 / 3.0) ||
        !(f->gamma_break > 0.0) || isinf(f->gamma_break) || isinf(f->alpha_hi) ||
        isinf(f->theta[12]))
      return -1;
  }
  return 0;
}

/* Full RING map: maps[f][3][npix] in K (double). */
int or_forward(const or_geom* g, const or_field* f, double* maps) {
  if (or_check(g, f)) return -1;
  const int64_t npix = 12LL * g->nside * g->nside;
  const int nf = g->n_freq;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < npix; ++p) {
    double out[3 * OR_MAX_FREQ];
    or_march_pixel(g, f, p, out);
    for (int k = 0; k < nf; ++k)
      for (int s = 0; s < 3; ++s) maps[((int64_t)k * 3 + s) * npix + p] = out[3 * k + s];
  }
  return 0;
}

/* Selected pixels: out[i][f][3] for pixel pix[i]; phi_end[i] may be NULL. */
int or_forward_pixels(const or_geom* g, const or_field* f, const int64_t* pix, int64_t n,
                      double* out, double* phi_end) {
  if (or_check(g, f)) return -1;
  const int64_t npix = 12LL * g->nside * g->nside;
  for (int64_t i = 0; i < n; ++i)
    if (pix[i] < 0 || pix[i] >= npix) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    double ph = or_march_pixel(g, f, pix[i], out + i * 3 * g->n_freq);
    if (phi_end) phi_end[i] = ph;
  }
  return 0;
}

/* Midpoints of the given pixels' sightlines: out[i][n][3] (kpc). */
int or_midpoints(const or_geom* g, const int64_t* pix, int64_t n, double* out) {
  if (g->nside < 1 || g->n_steps < 1) return -1;
  const int64_t npix = 12LL * g->nside * g->nside;
  for (int64_t i = 0; i < n; ++i) {
    if (pix[i] < 0 || pix[i] >= npix) return -1;
    or_ray ray;
    or_make_ray(g, pix[i], &ray);
    for (int k = 0; k < g->n_steps; ++k) or_midpoint(g, &ray, k, out + (i * g->n_steps + k) * 3);
  }
  return 0;
}

/* The march over tabulated field samples: fields[i][n][5] = (Bx, By, Bz [uG],
   n_e, N0) at midpoint n of pixel pix[i]; out[i][f][3] in K. */
int or_forward_tabulated(const or_geom* g, double alpha, const int64_t* pix, int64_t n,
                         const double* fields, double* out) {
  if (g->nside < 1 || g->n_steps < 1 || g->n_freq < 1 || g->n_freq > OR_MAX_FREQ) return -1;
  const int64_t npix = 12LL * g->nside * g->nside;
  for (int64_t i = 0; i < n; ++i)
    if (pix[i] < 0 || pix[i] >= npix) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    const or_source src = {NULL, fields + i * (int64_t)g->n_steps * 5};
    or_march_source(g, &src, alpha, 0.0, pix[i], out + i * 3 * g->n_freq);
  }
  return 0;
}

/* ========================================================================== */
/* Reverse pass: gradient of L = sum(dmaps * maps)                           */
/* ========================================================================== */

/* Adds the gradient of one pixel's contribution.  dm[f][3] are the cotangents
   of (T_I, T_Q, T_U) at this pixel.  Grid gradients go to gbn ([v][4]) and gc
   ([v]) when non-NULL; theta gradients to tb[16]. */
static void or_adjoint_pixel(const or_geom* g, const or_field* f, int64_t p, const double* dm,
                             double* tb, double* gbn, double* gc, int want_spec) {
  or_ray ray;
  or_make_ray(g, p, &ray);
  const int N = g->n_steps;
  const int alpha_gridded = f->kind == OR_GRID && f->grid_alpha != NULL;
  const double krm = or_k_rm();
  const double te = f->te_k;
  const double dpc = ray.dkpc * 1e3;
  or_local* q = (or_local*)malloc(sizeof(or_local) * (size_t)N);
  double* RM = (double*)malloc(sizeof(double) * (size_t)N);
  double* rmb = (double*)malloc(sizeof(double) * (size_t)N); /* dL/dRM_n */
  double* EM = (double*)malloc(sizeof(double) * (size_t)N);  /* emission measure to midpoint n */
  double* emb = (double*)malloc(sizeof(double) * (size_t)N); /* dL/dEM_n */
  double* ffb = (double*)malloc(sizeof(double) * (size_t)N); /* dL/d(n_e^2 dl) of its own emission */
  double* al = (double*)malloc(sizeof(double) * (size_t)N);  /* spectral index at midpoint n */
  /* forward sweep, keeping the per-step quantities */
  double before = 0.0, em_before = 0.0;
  for (int n = 0; n < N; ++n) {
    double r[3];
    or_midpoint(g, &ray, n, r);
    or_local_eval(f, &ray, r, &q[n]);
    al[n] = or_alpha_at(f, r);
    const double seg = q[n].ne * q[n].blos * ray.dcm;
    RM[n] = krm * (before + 0.5 * seg);
    before += seg;
    const double em_seg = te > 0.0 ? q[n].ne * q[n].ne * dpc : 0.0;
    EM[n] = em_before + 0.5 * em_seg;
    em_before += em_seg;
  }
  /* local cotangents of j_I, j_P, chi at every step; dL/dRM_n, dL/dEM_n */
  double* jIb = (double*)calloc((size_t)N * OR_MAX_FREQ, sizeof(double));
  double* jPb = (double*)calloc((size_t)N * OR_MAX_FREQ, sizeof(double));
  double* chi0b = (double*)calloc((size_t)N, sizeof(double));
  for (int n = 0; n < N; ++n) {
    rmb[n] = 0.0;
    emb[n] = 0.0;
    ffb[n] = 0.0;
    const double em_seg = te > 0.0 ? q[n].ne * q[n].ne * dpc : 0.0;
    const double alpha = al[n];
    for (int k = 0; k < g->n_freq; ++k) {
      const double nu = g->freq_hz[k];
      const double lam = OR_C / nu;
      const double rj = or_rj(nu);
      const double kff = te > 0.0 ? or_kff(nu, te) : 0.0;
      const double att = te > 0.0 ? exp(-kff * EM[n]) : 1.0;
      double j[4];
      or_emissivity(f, alpha, nu, q[n].Bt, q[n].n0, j);
      const double jI = j[0], jP = j[1];
      const double chi = RM[n] * lam * lam + q[n].chi0;
      const double gI = dm[3 * k + 0] * rj * ray.dcm;
      const double gQ = dm[3 * k + 1] * rj * ray.dcm;
      const double gU = dm[3 * k + 2] * rj * ray.dcm;
      const double pol = gQ * cos(2.0 * chi) + gU * sin(2.0 * chi);
      jIb[n * OR_MAX_FREQ + k] = gI * att;
      jPb[n * OR_MAX_FREQ + k] = pol * att;
      const double chib = att * jP * (-2.0 * gQ * sin(2.0 * chi) + 2.0 * gU * cos(2.0 * chi));
      chi0b[n] += chib;
      rmb[n] += chib * lam * lam;
      if (te > 0.0) {
        /* term_k = att (gI jI + jP pol + dI te kff em_seg); d att / d EM = -kff att */
        const double ffI = dm[3 * k + 0] * te * kff;
        emb[n] += -kff * att * (gI * jI + jP * pol + ffI * em_seg);
        ffb[n] += ffI * att;
      }
    }
  }
  /* RM_n = krm (sum_{m<n} seg_m + seg_n / 2): dL/dseg_m; the same for EM */
  double suffix = 0.0;    /* sum over n > m of dL/dRM_n */
  double em_suffix = 0.0; /* sum over n > m of dL/dEM_n */
  for (int n = N - 1; n >= 0; --n) {
    const double segb = krm * (suffix + 0.5 * rmb[n]);
    suffix += rmb[n];
    const double em_segb = ffb[n] + em_suffix + 0.5 * emb[n];
    em_suffix += emb[n];
    /* seg = ne * blos * dcm; em_seg = ne^2 dpc */
    const double neb_seg = segb * q[n].blos * ray.dcm + (te > 0.0 ? em_segb * 2.0 * q[n].ne * dpc : 0.0);
    const double blosb = segb * q[n].ne * ray.dcm;
    /* j_I, j_P depend on Bt, n0 (and alpha); chi0 = atan2(num, den) */
    const double alpha = al[n];
    double Btb = 0.0, n0b = 0.0, ab = 0.0;
    for (int k = 0; k < g->n_freq; ++k) {
      const double nu = g->freq_hz[k];
      if (q[n].Bt <= 0.0) continue;
      double j[4];
      or_emissivity(f, alpha, nu, q[n].Bt, q[n].n0, j);
      const double jI = j[0], jP = j[1];
      const double gI = jIb[n * OR_MAX_FREQ + k], gP = jPb[n * OR_MAX_FREQ + k];
      /* j is linear in n0; its B_trans slope comes with the emissivity */
      Btb += gI * j[2] + gP * j[3];
      if (q[n].n0 != 0.0) {
        n0b += (gI * jI + gP * jP) / q[n].n0;
      } else {
        double j1[4];
        or_emissivity(f, alpha, nu, q[n].Bt, 1.0, j1);
        n0b += gI * j1[0] + gP * j1[1];
      }
      if (f->spectrum == OR_SPEC_POWER) {
        double dI, dP;
        or_dlnj_dalpha(alpha, nu, q[n].Bt, &dI, &dP);
        ab += gI * jI * dI + gP * jP * dP;
      } else if (want_spec) {
        /* (a1, a2, ln gamma_b): theta[12], then the two entries after theta */
        double dI[3], dP[3];
        or_dj_broken(alpha, f->alpha_hi, f->gamma_break, nu, q[n].Bt, q[n].n0, dI, dP);
        ab += gI * dI[0] + gP * dP[0];
        tb[OR_NPARAM] += gI * dI[1] + gP * dP[1];
        tb[OR_NPARAM + 1] += gI * dI[2] + gP * dP[2];
      }
    }
    double numb = 0.0, denb = 0.0;
    if (q[n].Bt > 0.0) {
      const double bt2 = q[n].Bt * q[n].Bt;
      numb = Btb * q[n].num / q[n].Bt + chi0b[n] * q[n].den / bt2;
      denb = Btb * q[n].den / q[n].Bt - chi0b[n] * q[n].num / bt2;
    }
    /* a gridded index is an input without a gradient */
    if (!alpha_gridded) tb[12] += ab;
    /* num = 1e-6 B.e_b, den = -1e-6 B.e_l, blos = -1e-6 B.n  (B in uG) */
    double Bb[3];
    for (int k = 0; k < 3; ++k)
      Bb[k] = 1e-6 * (numb * ray.eb[k] - denb * ray.el[k] - blosb * ray.nhat[k]);
    double r[3];
    or_midpoint(g, &ray, n, r);
    if (f->kind == OR_MODEL16) {
      or_model16_vjp(f->theta, r, Bb, neb_seg, n0b, tb);
    } else if (f->kind == OR_WMAP) {
      or_wmap_vjp(f->theta, r, Bb, neb_seg, n0b, tb);
    } else if (f->kind == OR_GRID) {
      if (f->grid_c == NULL) {
        const double zero3[3] = {0, 0, 0};
        or_model16_vjp(f->theta, r, zero3, 0.0, n0b, tb);
      }
      int64_t base, s[3];
      double w[8];
      if (or_grid_cell(f, r, &base, s, w)) {
        for (int c = 0; c < 8; ++c) {
          const int64_t v = or_corner(base, s, c);
          if (gbn) {
            for (int k = 0; k < 3; ++k) {
#pragma omp atomic
              gbn[4 * v + k] += w[c] * Bb[k];
            }
#pragma omp atomic
            gbn[4 * v + 3] += w[c] * neb_seg;
          }
          if (gc && f->grid_c != NULL) {
#pragma omp atomic
            gc[v] += w[c] * n0b;
          }
        }
      }
    }
  }
  free(q);
  free(RM);
  free(rmb);
  free(EM);
  free(emb);
  free(ffb);
  free(al);
  free(jIb);
  free(jPb);
  free(chi0b);
}

/*
 * Gradient of L = sum_{f,s,p} dmaps[f][s][p] * maps[f][s][p] (maps from
 * or_forward) with respect to theta (dtheta[16], may be NULL; for a broken
 * power-law spectrum dtheta[18]: theta[12] is the index below the break and
 * dtheta[16], dtheta[17] are the derivatives in alpha_hi and ln gamma_break) and, for grid
 * fields, the grid values (dgrid_bn [nz][ny][nx][4], dgrid_c [nz][ny][nx]; each
 * may be NULL).  Pixels run in parallel; each thread keeps its own theta sums
 * and grid contributions are added atomically.
 */
int or_adjoint(const or_geom* g, const or_field* f, const double* dmaps, double* dtheta,
               double* dgrid_bn, double* dgrid_c) {
  if (or_check(g, f)) return -1;
  const int64_t npix = 12LL * g->nside * g->nside;
  const int nf = g->n_freq;
  double tb[OR_NPARAM + 2] = {0};
  const int nt = f->spectrum == OR_SPEC_BROKEN ? OR_NPARAM + 2 : OR_NPARAM;
  int64_t nv = 0;
  if (f->kind == OR_GRID) nv = (int64_t)f->grid_n[0] * f->grid_n[1] * f->grid_n[2];
  if (dgrid_bn) memset(dgrid_bn, 0, sizeof(double) * 4 * (size_t)nv);
  if (dgrid_c) memset(dgrid_c, 0, sizeof(double) * (size_t)nv);
#pragma omp parallel
  {
    double tl[OR_NPARAM + 2] = {0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
      double dm[3 * OR_MAX_FREQ];
      int any = 0;
      for (int k = 0; k < nf; ++k)
        for (int s = 0; s < 3; ++s) {
          dm[3 * k + s] = dmaps[((int64_t)k * 3 + s) * npix + p];
          any |= dm[3 * k + s] != 0.0;
        }
      if (any) or_adjoint_pixel(g, f, p, dm, tl, dgrid_bn, dgrid_c, dtheta != NULL);
    }
#pragma omp critical
    for (int k = 0; k < nt; ++k) tb[k] += tl[k];
  }
  if (dtheta)
    for (int k = 0; k < nt; ++k) dtheta[k] = tb[k];
  return 0;
}

/* The analytic 16-parameter model sampled on the nodes of a grid:
   out_bn [nz][ny][nx][4], out_c [nz][ny][nx] (either may be NULL). */
int or_sample_model16(const double* theta, const int32_t n[3], const double lo[3],
                      const double hi[3], float* out_bn, float* out_c) {
  if (n[0] < 2 || n[1] < 2 || n[2] < 2) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t iz = 0; iz < n[2]; ++iz)
    for (int64_t iy = 0; iy < n[1]; ++iy)
      for (int64_t ix = 0; ix < n[0]; ++ix) {
        const double r[3] = {lo[0] + (hi[0] - lo[0]) * (double)ix / (double)(n[0] - 1),
                             lo[1] + (hi[1] - lo[1]) * (double)iy / (double)(n[1] - 1),
                             lo[2] + (hi[2] - lo[2]) * (double)iz / (double)(n[2] - 1)};
        double B[3], ne, n0;
        or_model16(theta, r, B, &ne, &n0);
        const int64_t v = ix + n[0] * (iy + n[1] * iz);
        if (out_bn) {
          for (int k = 0; k < 3; ++k) out_bn[4 * v + k] = (float)B[k];
          out_bn[4 * v + 3] = (float)ne;
        }
        if (out_c) out_c[v] = (float)n0;
      }
  return 0;
}

/* Any field kind sampled on the nodes of a grid (node i of an axis at
   lo + i (hi - lo) / (n - 1)), as the grid field generators of Sec. 2.3 are
   built from a field: out_bn [nz][ny][nx][4] = (Bx, By, Bz, n_e), out_c
   [nz][ny][nx] = N0 (either may be NULL). */
int or_sample_field(const or_field* f, const int32_t n[3], const double lo[3], const double hi[3],
                    float* out_bn, float* out_c) {
  if (n[0] < 2 || n[1] < 2 || n[2] < 2) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t iz = 0; iz < n[2]; ++iz)
    for (int64_t iy = 0; iy < n[1]; ++iy)
      for (int64_t ix = 0; ix < n[0]; ++ix) {
        const double r[3] = {lo[0] + (hi[0] - lo[0]) * (double)ix / (double)(n[0] - 1),
                             lo[1] + (hi[1] - lo[1]) * (double)iy / (double)(n[1] - 1),
                             lo[2] + (hi[2] - lo[2]) * (double)iz / (double)(n[2] - 1)};
        double B[3], ne, n0;
        or_fields(f, r, B, &ne, &n0);
        const int64_t v = ix + n[0] * (iy + n[1] * iz);
        if (out_bn) {
          for (int k = 0; k < 3; ++k) out_bn[4 * v + k] = (float)B[k];
          out_bn[4 * v + 3] = (float)ne;
        }
        if (out_c) out_c[v] = (float)n0;
      }
  return 0;
}

/* Thread count of the OpenMP loops over pixels (for timing on a given number
   of host cores). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
