/*
 * synmarch -- MI355X (gfx950) sightline march for Galactic synchrotron maps.
 *
 * C ABI of the hot path of Diao et al., "synax: a differentiable and
 * GPU-accelerated synchrotron simulation package" (arXiv:2410.01136):
 * for every HEALPix pixel a sightline from the observer is cut into N equal
 * segments sampled at their midpoints (Sec. 2.3); the fields B, n_e and the
 * cosmic-ray normalisation N0 are evaluated there, analytically or by trilinear
 * interpolation of a regular grid (Sec. 2.3); the emissivities of Eqs. ji and
 * jp (Sec. 2.1-2.2), the rotation measure of Eq. rm as a running sum and the
 * angle chi = RM lambda^2 + chi_0 of Eq. chi give the sums of Eq. int, which
 * are returned as Rayleigh-Jeans brightness temperatures in K.
 *
 * Conventions shared by every entry point
 *  - Pointers marked (device) are HIP device pointers; everything else is host.
 *    The caller owns every buffer.  Only syn_batch_create allocates device
 *    memory (freed by syn_batch_destroy).
 *  - Calls are ordered on the given stream and return before the GPU work
 *    ends.  All argument checks run on the host before any launch; on a
 *    non-OK status nothing has been launched and no output was written.
 *  - No C++ exception crosses the ABI.  syn_last_error() returns a
 *    thread-local description of the last failing call.
 *  - Positions are Galactocentric Cartesian in kpc: x from the Sun toward the
 *    Galactic centre, y toward l = 90 deg, z toward b = 90 deg.  B is in
 *    micro-gauss, n_e and N0 in cm^-3, frequencies in Hz.
 *  - Maps are float [n_freq][3][npix], Stokes (I, Q, U) in K, HEALPix RING
 *    order.  Q and U follow Eq. int with chi_0 measured from Galactic north
 *    toward increasing l (tan chi_0 = B.e_b / (-B.e_l)); B_LOS is signed,
 *    -B.n, positive toward the observer; the RM at a midpoint includes half of
 *    its own segment.
 */
#ifndef SYNMARCH_H
#define SYNMARCH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SYN_OK = 0,
  SYN_EINVAL = -1,        /* an argument failed validation                 */
  SYN_EUNSUPPORTED = -2,  /* valid request the library does not implement  */
  SYN_ENOMEM = -3,        /* device allocation failed (batch plans only)   */
  SYN_EHIP = -4,          /* a HIP runtime call failed                     */
  SYN_EWORKSPACE = -5     /* workspace missing or too small                */
} syn_status;

enum {
  SYN_FIELD_MODEL16 = 0, /* 16-parameter analytic spiral-disk model         */
  SYN_FIELD_GRID = 1,    /* trilinear interpolation of node-centred grids   */
  SYN_FIELD_SPHERE = 2,  /* homogeneous sphere (Sec. 2.4 test)              */
  SYN_FIELD_MLP = 3,     /* coordinate-MLP surrogate of the fields          */
  SYN_FIELD_WMAP = 4     /* WMAP field and CR density of Sec. 3.1           */
};

enum { SYN_NPARAM = 16, SYN_MAX_FREQ = 16, SYN_MAX_NSIDE = 8192 };

enum {
  SYN_SPEC_POWER_LAW = 0, /* one power law of index theta[12] (Eqs. ji, jp) */
  SYN_SPEC_BROKEN = 1     /* broken power law, see syn_spectrum_table        */
};

/* Geometry and step schedule (Sec. 2.3).  The sightline of every pixel runs
   from r_obs to the first box face it meets, capped at r_max, and is cut into
   n_steps equal segments sampled at their midpoints. */
typedef struct syn_geom {
  int32_t nside;                /* power of two, 1 .. SYN_MAX_NSIDE          */
  int32_t n_steps;              /* >= 1                                      */
  double r_obs_kpc[3];          /* observer, strictly inside the box         */
  double r_max_kpc;             /* > 0; +inf: box only                       */
  double box_lo_kpc[3];         /* box faces; +-inf allowed, but every       */
  double box_hi_kpc[3];         /* sightline must end at a finite length     */
  int32_t n_freq;               /* 1 .. SYN_MAX_FREQ                         */
  double freq_hz[SYN_MAX_FREQ]; /* > 0                                       */
} syn_geom;

/* Field-model descriptor (Sec. 2.3: a callable field generator, analytic or
   gridded).  theta[12] is the CR power-law index alpha (> 1/3, the pole of
   Gamma(alpha/4 - 1/12) in Eq. ji) for every kind.
   MODEL16 theta: 0 B0[uG] 1 psi0 2 psi1 3 chiB0 [rad] 4 R_B 5 z_B [kpc]
     6 BH0[uG] 7 z_H 8 R_H [kpc] 9 C0[cm^-3] 10 hr_CR 11 hz_CR [kpc] 12 alpha
     13 n0[cm^-3] 14 hz_ne[kpc] 15 kappa_ne[1/kpc]; Sun at R = 8.5 kpc.
       B = B0 e^{-(R-8.5)/R_B - |z|/z_B} (sin psi cos chi rho^ + cos psi cos chi
           phi^ + sin chi z^), psi = psi0 + psi1 ln(R/8.5), chi = chiB0 tanh(z)
         + BH0 (z/z_H) e^{-|z|/z_H - (R-8.5)/R_H} phi^,
       N0 = C0 e^{-(R-8.5)/hr - |z|/hz},  n_e = n0 e^{-|z|/hz_ne - kappa (R-8.5)}.
   GRID: grid_bn (device) float [nz][ny][nx][4] = (Bx, By, Bz, n_e); grid_c
     (device) float [nz][ny][nx] = N0, or NULL for N0 from the MODEL16 formula
     with theta[9..11].  Node i of an axis sits at lo + i (hi - lo) / (n - 1);
     outside [lo, hi] every gridded field is zero.  At least 2 nodes per axis.
   SPHERE theta: 0-2 B[uG] 3 n_e 4 N0 5 radius[kpc] (<= 0: everywhere)
     6-8 centre[kpc]; fields are uniform inside, zero outside.
   MLP: mlp (device) packed weights from syn_mlp_pack; grid_lo/hi give the box
     the network's input coordinates are normalised to.
   WMAP theta (Sec. 3.1, after Page et al. 2007): 0 b0[uG] 1 psi0 2 psi1
     3 chi0 [rad] 4 rho_in 5 rho_out [kpc] 9 C0[cm^-3] 10 h_r 11 h_z [kpc]
     12 alpha 13 n0[cm^-3] 14 hz_ne[kpc] 15 kappa_ne[1/kpc]; 6-8 unused.
       B = b0 (cos psi cos chi rho^ + sin psi cos chi phi^ + sin chi z^) for
           rho_in <= R <= rho_out, zero elsewhere; psi = psi0 + psi1 ln(R/8),
           chi = chi0 tanh(z),
       N0 = C0 e^{-R/h_r} sech^2(z/h_z),  n_e as for MODEL16 (an exponential
       disk standing in for the paper's YMW16).  theta-gradients of every
       entry but the ring radii. */
typedef struct syn_field {
  int32_t kind;
  double theta[SYN_NPARAM];
  int32_t grid_n[3];            /* nx, ny, nz                                 */
  double grid_lo_kpc[3];
  double grid_hi_kpc[3];
  const float* grid_bn;         /* (device)                                   */
  const float* grid_c;          /* (device) or NULL                           */
  const void* mlp;              /* (device)                                   */
  double te_k;                  /* thermal electron temperature [K]; 0 = off  */
  const float* grid_alpha;      /* (device) GRID: CR spectral index per node,
                                   float [nz][ny][nx], or NULL for theta[12]   */
  int32_t spectrum;             /* SYN_SPEC_*; 0 (power law) when zeroed       */
  double alpha_hi;              /* SYN_SPEC_BROKEN: index above the break      */
  double gamma_break;           /* SYN_SPEC_BROKEN: Lorentz factor of the break */
  const void* spectrum_table;   /* (device) SYN_SPEC_BROKEN: from
                                   syn_spectrum_table(theta[12], alpha_hi)     */
} syn_field;
/* Gridded spectral index (grid_alpha != NULL, GRID fields only; a first step
   toward the full CR spectrum the paper leaves to future work, Sec. 2.1):
   Eqs. ji and jp are evaluated at each midpoint with alpha interpolated
   trilinearly from the nodes like the other gridded fields.  Values must
   exceed 1/3 (the pole of Gamma(alpha/4 - 1/12)); they are not checked on the
   host.  theta[12] then only sets the reference point of the prefactors and
   receives no gradient (dtheta[12] = 0); the index itself gets no gradient.
   SYN_EINVAL for a non-GRID field or a pointer not 4-byte aligned. */
/* Free-free emission and absorption (te_k > 0; the paper names both as future
   work in Sec. 5 and gives no formulas, so this follows the textbook radio
   treatment): the thermal electrons n_e, taken as a fully ionised hydrogen
   plasma at temperature te_k, have the optical depth
     d tau = 0.08235 te_k^-1.35 (nu / GHz)^-2.1 n_e^2 dl   (dl in pc; Mezger &
   Henderson 1967), emit d T_I = te_k d tau (Rayleigh-Jeans source function),
   and attenuate everything a segment emits (I, Q, U) by e^-tau, tau being the
   depth from the observer to the segment's midpoint (earlier segments plus
   half of its own, as for the rotation measure).  Not available for the MLP
   surrogate (SYN_EUNSUPPORTED) or in batch plans; te_k must be finite and
   >= 0 (SYN_EINVAL).  Gradients flow through n_e; te_k itself gets none. */

/* Broken power-law CR spectrum (spectrum = SYN_SPEC_BROKEN; the paper models
   the CR electrons with one power law and names fuller spectra as future work,
   Sec. 2.1): N(gamma) = N0 gamma^-a1 below the Lorentz factor gamma_break and
   N0 gamma_break^(a2 - a1) gamma^-a2 above it (continuous at the break), with
   a1 = theta[12] and a2 = alpha_hi.  The emissivities are the single-electron
   synchrotron spectrum integrated over this N(gamma), which for one index is
   Eqs. ji and jp; for the broken law each side of the break contributes the
   part of its x-moment (x = nu / nu_c) on its side of
   xb = 4 pi nu m c / (3 q B_perp gamma_break^2):
     j_I = j_I(a1) (1 - S_F(a1, xb)) + gamma_break^(a2 - a1) j_I(a2) S_F(a2, xb),
   and the same for j_P with the shares S_G of G(x) = x K_2/3(x), S being the
   share of the moment below xb.  The kernels interpolate S from a table that
   syn_spectrum_table builds for (a1, a2) once; gamma_break and the frequencies
   enter per call.  Ranges: 1/3 < a1, a2 <= 6, 1 <= gamma_break <= 1e12, and
   the break within reach of the FP32 arithmetic at every frequency of the
   geometry (for B_perp from 2^-20 to 2^20 uG the powers of xb the kernels form
   stay finite; else SYN_EUNSUPPORTED naming the frequency).  Not with
   grid_alpha (SYN_EINVAL), the MLP surrogate or batch plans
   (SYN_EUNSUPPORTED).  syn_adjoint differentiates the spectrum too: dtheta
   then holds 18 doubles, dtheta[12] = dL/d alpha_lo (theta[12]), dtheta[16] =
   dL/d alpha_hi and dtheta[17] = dL/d ln gamma_break (the index derivatives of
   the moment shares come from a second part of the table). */

/* Bytes of a broken power-law table (device memory the caller allocates). */
size_t syn_spectrum_table_bytes(void);

/* Builds the table of moment shares for indices alpha_lo (the field's
   theta[12]) and alpha_hi on the host and copies it into table (device,
   table_bytes >= syn_spectrum_table_bytes(), 16-byte aligned) on stream,
   which it then synchronises.  The library records the pair of indices with
   the table's address; syn_forward and syn_adjoint accept a broken-spectrum
   field only with a table recorded for its theta[12] and alpha_hi (else
   SYN_EINVAL).  The caller keeps the table alive and unmodified while fields
   use it.  SYN_EINVAL for indices out of range, a small or misaligned table;
   SYN_EHIP if the copy fails. */
syn_status syn_spectrum_table(double alpha_lo, double alpha_hi, void* table, size_t table_bytes,
                              hipStream_t stream);

/* The same table built into host memory (table (host) float, table_bytes >=
   syn_spectrum_table_bytes()), for inspection: two parts of 753 nodes x 8
   floats, node k at t = log2 xb = -40 + k / 16 holding (g_F(lo), g_G(lo),
   g_F(hi), g_G(hi)) and h dg/dt of each, g = S 2^(-p t), p = a / 2 - 1/6; the
   second part the same for the derivatives in each function's own index.
   Fields accept only tables that syn_spectrum_table wrote.  SYN_EINVAL as
   syn_spectrum_table. */
syn_status syn_spectrum_table_host(double alpha_lo, double alpha_hi, float* table,
                                   size_t table_bytes);

/* Bytes of workspace syn_forward needs; with_adjoint != 0 adds what the
   matching syn_adjoint reads (the Faraday sum of every sightline, 8 B per
   pixel, with free-free also its emission measure, 8 B per pixel, plus
   per-block gradient partials) and, for fields with a reverse pass (GRID;
   MODEL16 and WMAP unless under a broken power law, whose theta-only reverse
   pass interleaves steps instead), the piece snapshots: the running sums the
   forward leaves at the ends of the reverse pass's S contiguous pieces per
   sightline (S its lane count; 1 + 2 n_freq doubles, with free-free
   2 + 4 n_freq, per piece end and pixel), from which the reverse pass starts
   each piece.  Returns 0 for invalid input. */
size_t syn_workspace_bytes(const syn_geom* geom, const syn_field* field, int32_t with_adjoint);

/* Forward march: maps (device) float [n_freq][3][npix] in K.  ws (device) may
   be NULL (ws_bytes 0) when no adjoint will follow; otherwise it must hold
   syn_workspace_bytes(geom, field, 1) bytes and is read by syn_adjoint. */
syn_status syn_forward(const syn_geom* geom, const syn_field* field, float* maps, void* ws,
                       size_t ws_bytes, hipStream_t stream);

/* Reverse pass of syn_forward -- the gradient of the maps with respect to the
   field model's inputs that the paper obtains by automatic differentiation of
   the forward (Sec. 1 and Sec. 2.4; a gradient costs a few forwards, Sec. 2.4
   and Sec. 4.2) and uses for gradient-based inference (Sec. 3.1-3.2) and for
   optimising gridded fields (Sec. 3.3).  Given dmaps (device) = dL/dmaps, float
   [n_freq][3][npix], returns dL/dtheta in dtheta (device, double[16], or
   double[18] for a broken power-law spectrum (see above); written, not
   accumulated; may be NULL) and, for GRID fields, ADDS dL/dgrid into
   dgrid_bn (device, float [nz][ny][nx][4]) and dgrid_c (device, float
   [nz][ny][nx]) when non-NULL (atomic float adds: bitwise order may vary).
   ws must be the workspace of the syn_forward call with the same geom and
   field: the library records, per workspace address, a hash of the geometry
   and field (parameters and grid pointers included) of the last syn_forward
   that wrote it, and returns SYN_EWORKSPACE for a workspace no forward wrote
   or one written under another geometry or field.  Sightlines are
   recomputed in reverse step order; the Faraday sum is rebuilt from its
   stored total, so no per-step state is stored. */
syn_status syn_adjoint(const syn_geom* geom, const syn_field* field, const float* dmaps,
                       void* ws, size_t ws_bytes, double* dtheta, float* dgrid_bn,
                       float* dgrid_c, hipStream_t stream);

/* Gaussian chi^2 of Sec. 3.1 extended to I, Q and U:
   chi2 = sum_m inv_sigma2[m] sum_p (maps[m][p] - target[m][p])^2 over n_maps
   maps of n_pix values, and dmaps = d chi2 / d maps (device, float; may be
   NULL).  chi2 is a device double[1], summed in FP64 in a fixed order.
   inv_sigma2 is host, double[n_maps] (finite, >= 0).  ws (device) holds
   syn_chi2_workspace_bytes(n_pix, n_maps) bytes of partial sums. */
size_t syn_chi2_workspace_bytes(int64_t n_pix, int32_t n_maps);
syn_status syn_chi2(int64_t n_pix, int32_t n_maps, const float* maps, const float* target,
                    const double* inv_sigma2, float* dmaps, double* chi2, void* ws,
                    size_t ws_bytes, hipStream_t stream);

/* syn_chi2 for callers that cannot allocate device memory (code under HIP
   graph capture, serving loops, harnesses that forbid hipMalloc): the same
   arguments, kernels and results (bit for bit), without the workspace; the
   FP64 partial sums live in a static 32 KiB device array of the library, one
   per GPU, kept until the process ends.  The call allocates nothing.  Calls
   that overlap on one GPU (on different streams, or from several threads)
   share that array and race: order them.  n_pix * n_maps may be at most
   SYN_CHI2_MAX_VALUES; beyond it, and for the arguments syn_chi2 rejects,
   SYN_EINVAL; a failing HIP call, SYN_EHIP. */
#define SYN_CHI2_MAX_VALUES ((int64_t)1 << 36)
syn_status syn_chi2_cotangent(int64_t n_pix, int32_t n_maps, const float* maps,
                              const float* target, const double* inv_sigma2, float* dmaps,
                              double* chi2, hipStream_t stream);

/* One step of the Adam optimiser (Kingma & Ba 2015, arXiv:1412.6980,
   Algorithm 1) in place on n FP32 parameters, as used to fit a gridded field
   to observed maps in Sec. 3.3 (the gradient comes from syn_adjoint):
     m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
     params -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
   params, m, v (device, FP32, n each) are updated in place; grads (device)
   is read; m and v start at zero and t counts updates from 1.  Element i
   takes part iff bit (i % period) of mask is set (period in [1, 32]; e.g.
   period 4, mask 0x7 updates the B components of a (B_x, B_y, B_z, n_e)
   grid and leaves n_e alone); the others are not touched.  Arithmetic in
   FP32, bias corrections on the host in FP64.  SYN_EINVAL for n < 0,
   t < 1, betas outside [0, 1), eps < 0, a non-finite lr, a period outside
   [1, 32] or NULL/misaligned pointers; no launch for n = 0. */
syn_status syn_adam_step(int64_t n, int32_t period, uint32_t mask, float* params,
                         const float* grads, float* m, float* v, int32_t t, double lr,
                         double beta1, double beta2, double eps, hipStream_t stream);

/* The MODEL16 fields sampled on the nodes of a grid: out_bn (device) float
   [nz][ny][nx][4] = (Bx, By, Bz, n_e) and out_c (device) float [nz][ny][nx]
   = N0 (either may be NULL).  n = (nx, ny, nz), each >= 2. */
syn_status syn_sample_model16(const double* theta, const int32_t n[3], const double lo[3],
                              const double hi[3], float* out_bn, float* out_c,
                              hipStream_t stream);

/* Field values at n points (device float [n][3], kpc): out (device) float
   [n][5] = (Bx, By, Bz, n_e, N0).  Any field kind. */
syn_status syn_eval_fields(const syn_field* field, int64_t n, const float* xyz, float* out,
                           hipStream_t stream);

/* ---- coordinate-MLP surrogate of the fields ------------------------------ */
/* Network: x^ = 2 (r - lo) / (hi - lo) - 1; features sin(2 pi b_k . x^),
   cos(2 pi b_k . x^) for 16 frequency vectors b_k; 4 hidden layers of width
   128 with the cubic-gated unit x S(s), s = clamp(x / 4 + 1/2, 0, 1),
   S = s^2 (3 - 2 s); a linear output of 5 = (Bx, By, Bz [uG], ln n_e, ln N0).
   Weights and layer inputs are FP16, biases FP32; products accumulate in FP32
   on the matrix cores and the gate is evaluated in FP16.  syn_mlp_pack converts host FP32 arrays
   (w_in [128][32], b_in [128], w_h [3][128][128], b_h [3][128], w_out
   [5][128], b_out [5], fourier [16][3]) into the packed device layout;
   syn_mlp_packed_bytes gives its size. */
size_t syn_mlp_packed_bytes(void);
syn_status syn_mlp_pack(const float* fourier, const float* w_in, const float* b_in,
                        const float* w_h, const float* b_h, const float* w_out,
                        const float* b_out, void* packed_host);

/* ---- many parameter sets in one persistent launch ------------------------ */
/* The batched evaluation the paper gets from vectorising the forward and its
   gradient over parameter sets (Sec. 1 and Sec. 3.2: many sampler chains, or
   leapfrog states, evaluated together), with the chi^2 likelihood of
   Sec. 3.1.  A batch is n_sets MODEL16 or WMAP parameter vectors, each with its
   own N_side, sharing one geometry (steps, observer, cap, box, frequency).  One
   plan runs forward, chi^2 against per-set targets and the adjoint for every
   set in a single captured HIP graph of persistent work-queue kernels. */
typedef struct syn_batch_desc {
  int32_t n_sets;              /* 1 .. 65536                                    */
  const int32_t* nside;        /* [n_sets], powers of two                       */
  const double* theta;         /* [n_sets][16]                                  */
  syn_geom geom;               /* nside ignored; exactly one frequency          */
  int32_t use_graph;           /* 1: capture the launch sequence once as a HIP
                                  graph and replay it; 0: launch directly     */
  int32_t kind;                /* field of every set: SYN_FIELD_MODEL16 (0) or
                                  SYN_FIELD_WMAP; theta as for syn_field       */
} syn_batch_desc;

typedef struct syn_batch syn_batch;

/* Creates a plan; allocates its device tables.  Pixel p of set s lives at
   offset syn_batch_offset(plan, s) + p of the ragged map arrays, which hold
   syn_batch_total_pixels(plan) pixels per Stokes map ([3][total]). */
syn_status syn_batch_create(const syn_batch_desc* desc, syn_batch** plan);
int64_t syn_batch_total_pixels(const syn_batch* plan);
int64_t syn_batch_offset(const syn_batch* plan, int32_t set);
/* Runs forward, chi^2 with inv_sigma2 (host double[3], one weight per Stokes
   map, shared by all sets) against target (device float [3][total]) and the
   adjoint.  Outputs (device): maps float [3][total], dmaps float [3][total]
   (= d chi2 / d maps), chi2 double [n_sets], dtheta double [n_sets][16]
   (= d chi2_s / d theta_s).  With use_graph the first call captures the
   sequence (on a private stream) and every call launches the graph on
   `stream`; a call with different pointers or weights captures again.  Calls
   on one plan must not overlap (they share the plan's work counters).  The
   plan is bound to the device current at creation. */
/* Replaces the parameters of every set (host double [n_sets][16], same kind
   and checks as at creation) for the following runs -- the sampler's case,
   where chains move every step.  Waits for earlier work on `stream` (which
   may still read the set table), then copies the new table synchronously; a
   captured graph stays valid.  On an error nothing changes. */
syn_status syn_batch_set_theta(syn_batch* plan, const double* theta, hipStream_t stream);

syn_status syn_batch_run(syn_batch* plan, const float* target, const double* inv_sigma2,
                         float* maps, float* dmaps, double* chi2, double* dtheta,
                         hipStream_t stream);
void syn_batch_destroy(syn_batch* plan);

/* ---- launch shapes --------------------------------------------------------- */
/* Kernel families tuned by the autotuner. */
enum { SYN_KERNEL_FORWARD = 0, SYN_KERNEL_ADJOINT = 1, SYN_KERNEL_BATCH = 2 };

/* Lanes per sightline S (1, 4, 8, 16 or 64; the batch kernels take 1, 4, 16
   or 64): consecutive steps of one sightline
   are spread over S lanes and their Faraday sums are combined with a
   wavefront prefix scan.  The adjoint instead gives each of the S lanes a
   contiguous piece of ceil(n_steps / S) steps (the pieces are joined by
   group scans of their Faraday sums and phase cotangents); when the forward
   stored piece snapshots for S pieces, syn_adjoint uses that S.  0 restores the built-in choice.  Applies to the given
   (kernel, field kind) pair on the calling process. */
syn_status syn_set_lanes_per_ray(int32_t kernel, int32_t field_kind, int32_t lanes);
int32_t syn_get_lanes_per_ray(int32_t kernel, int32_t field_kind, int64_t npix);

/* Grid reads of the forward march over a GRID field.
   Grids under 4 GiB whose cell indices along every sightline of the geometry
   fit in 30 bits can be read through buffer resources with 32-bit byte offsets,
   either each lane reading its own cell or each distinct cell of a wavefront
   loaded once into LDS and shared by the lanes in it; other grids are read
   through 64-bit addresses.
   0 (default) = automatic: shared reads from 2^18 sightlines on, per-lane
     buffer reads below;
   1 = always 64-bit addresses, each lane reading its own cell;
   2 = buffer reads, each lane its own cell (where allowed);
   3 = buffer reads shared through LDS (where allowed).
   All read the same node values and agree to FP32 rounding (the compiler may
   fuse the interpolation sums differently per variant).  Process-wide;
   SYN_EINVAL for any other mode. */
syn_status syn_set_grid_addressing(int32_t mode);
int32_t syn_get_grid_addressing(void);

/* Autotuned launch shapes (the project's tuner, which times every lane count
   and grid read mode on the workload at hand and caches the fastest).
   syn_autotune_load reads the tuner's cache file (path: host string): a JSON
   object whose keys are
     "<device name>|<build id>|k<kernel>|f<field kind>|p<npix>|n<n_steps>|q<n_freq>"
   (with a trailing "|g" when the value carries a grid read mode) and whose
   values are a lane count (1, 4, 8, 16, 64; 8 not for batch entries) or
   [lane count, grid read mode 2|3].
   Entries whose build id is not this library's (syn_build_id: a hash of the
   sources it was built from) are stale and skipped; the rest replace the
   table.  From then on a syn_forward, syn_adjoint or syn_batch_create whose
   kernel family, field kind, N_side, step count and frequency count (1 for
   batch plans, whose npix is the plan's total) match an entry for the current
   device (name "*": any device) uses its lane count -- unless one was set
   with syn_set_lanes_per_ray -- and, for gridded forwards under automatic
   grid addressing, its read mode.  A missing or unreadable file, malformed
   JSON, a malformed key or a value out of range returns SYN_EINVAL and leaves
   the table as it was (calls then keep their previous or built-in shapes).
   Process-wide. */
syn_status syn_autotune_load(const char* path);
void syn_autotune_clear(void);
int32_t syn_autotune_entries(void);
/* 1 and the table's lane count and grid read mode (0: none) if an entry
   applies to this shape on the current device, else 0. */
int32_t syn_autotune_lookup(int32_t kernel, int32_t field_kind, int64_t npix, int32_t n_steps,
                            int32_t n_freq, int32_t* lanes, int32_t* grid_mode);
const char* syn_build_id(void);

const char* syn_last_error(void);
int32_t syn_version(void);

/* Host-side copy of the pixel ordering the kernels use, for checks without a
   GPU: the RING index, z = cos(colatitude) and longitude of NESTED pixel q. */
syn_status syn_host_nest_pixel(int32_t nside, int64_t q, int64_t* ring, double* z, double* phi);

#ifdef __cplusplus
}
#endif

#endif /* SYNMARCH_H */
