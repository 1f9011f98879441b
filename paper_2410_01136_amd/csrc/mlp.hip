// Coordinate-MLP surrogate of the fields, evaluated on the matrix cores and
// fused into the sightline march.
//
// Network: x^ = 2 (r - lo) / (hi - lo) - 1; 32 Fourier features sin(2 pi b_f.x^),
// cos(2 pi b_f.x^) (f < 16); 4 hidden layers of width 128 with a GELU-shaped gate;
// a linear output of 5 = (Bx, By, Bz [uG], ln n_e, ln N0).  The activation is a
// cubic-gated linear unit, x S((x + 2) / 4) with S(s) = 3 s^2 - 2 s^3 on [0, 1]
// (clamped): the shape of GELU (its gate approximates the normal CDF, slope 3/8
// against 0.40 at 0) in six full-rate instructions, where the tanh form of GELU
// costs an exp and a reciprocal at a quarter of the rate.  FP16 weights and
// layer inputs, FP32 accumulation (v_mfma_f32_32x32x16_f16, the same dense rate
// as BF16 on this chip); the FP32 bias is the addend of each row block's first
// product, and the gate runs on packed FP16 pairs (v_pk_fma_f16,
// v_pk_mul_f16), two activations per instruction.
//
// Tiling.  One wavefront evaluates 64 points as two blocks of 32 (A: points
// 0..31, B: points 32..63), both at once: each weight fragment read from LDS
// feeds the two blocks' products, two independent accumulation chains.  Every
// layer is computed transposed, features on
// the rows and points on the columns: D[128 x 32] = W[128 x K] X[K x 32].  With
// that orientation the accumulator a lane holds after a layer (16 rows of one
// column per 32-row block) is exactly the B operand the next layer needs, once
// the next layer's weight columns are permuted to the order in which the rows
// sit in the lanes -- so activations never leave the registers.  The weights
// (117 KB packed) are staged once per workgroup in LDS; A-operand fragments
// are read with one 16-byte LDS load each, once per 64-point tile.  A layer's
// outputs go to a second operand buffer, so each 32-row block is activated as
// soon as its products are done.
// The output layer places the 5 outputs twice, at rows {0,1,2,3,8} (held by
// lanes 0..31 for block A) and {4,5,6,7,12} (lanes 32..63 for block B), so
// afterwards every lane holds the 5 fields of its own point.
//
// In the fused march a wavefront owns one sightline; point p of a tile is step
// 64 c + p, so the Faraday prefix of Eq. rm is a full-wavefront scan.
#include <string.h>

#include <cmath>

#include "../../include/synmarch.h"
#include "march_body.h"
#include "mlp_layout.h"
#include "sm_launch.h"

namespace sm {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline f32x16 mfma(f16x8 a, f16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// sin and cos of 2 pi t in FP32: reduced to [-1/2, 1/2] turn, then the
// hardware sine and cosine (argument in turns).
__device__ inline void sincos_turns_f(float t, float* sn, float* cs) {
  const float r = t - rintf(t);
  *sn = __builtin_amdgcn_sinf(r);
  *cs = __builtin_amdgcn_cosf(r);
}

// Copies the packed network from global memory into LDS (whole workgroup).
__device__ inline void stage_weights(const void* packed, unsigned char* lds, int nthreads) {
  const uint4* src = reinterpret_cast<const uint4*>(packed);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  for (int i = threadIdx.x; i < kMlpBytes / 16; i += nthreads) dst[i] = src[i];
  __syncthreads();
}

// Fourier-feature B operands of one point for this lane's half: the lane
// supplies features k = 16 t + 8 h + i, i.e. sin (t = 0) and cos (t = 1) of
// frequencies 8 h + i.
__device__ inline void fourier_operand(const float* fq, float x, float y, float z, int h,
                                       f16x8* op) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float* b = fq + 3 * (8 * h + i);
    const float t = fmaf(b[0], x, fmaf(b[1], y, b[2] * z));
    float s, c;
    sincos_turns_f(t, &s, &c);
    op[0][i] = (_Float16)s;
    op[1][i] = (_Float16)c;
  }
}

// Activation of a 32-row accumulator block (bias included), converted into the
// next layer's B operands (two k-steps per row block): the accumulator rounded
// to FP16 and the gate applied on packed pairs.  The gate runs stage by stage
// over the block's 8 pairs, so that consecutive instructions are independent;
// pair by pair, each packed FP16 instruction would read the one before it, a
// dependence this chip makes wait a cycle.
__device__ inline void activate(const f32x16& acc, f16x8* op2) {
  h2v x[8], s[8], t[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    x[p].x = (_Float16)acc[2 * p];
    x[p].y = (_Float16)acc[2 * p + 1];
  }
  // cubic-gated linear unit x S(s), s = clamp(x / 4 + 1/2, 0, 1), S = s^2 (3 - 2 s);
  // each operation rounds to FP16 (x / 4 and 2 s are exact, so the fused forms
  // round once like the separate ones)
#pragma unroll
  for (int p = 0; p < 8; ++p)
    s[p] = __builtin_elementwise_min(
        __builtin_elementwise_max(x[p] * (h2v)(0.25f16) + (h2v)(0.5f16), (h2v)(0.0f16)),
        (h2v)(1.0f16));
#pragma unroll
  for (int p = 0; p < 8; ++p) t[p] = (h2v)(3.0f16) - (h2v)(2.0f16) * s[p];
#pragma unroll
  for (int p = 0; p < 8; ++p) s[p] = s[p] * s[p];
#pragma unroll
  for (int p = 0; p < 8; ++p) t[p] = s[p] * t[p];
  // pair p is accumulator registers 2p, 2p + 1: elements 2 (p % 4), +1 of k-step p / 4
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const h2v y = x[p] * t[p];
    op2[p >> 2][2 * (p & 3)] = y.x;
    op2[p >> 2][2 * (p & 3) + 1] = y.y;
  }
}

// One layer for both point blocks: X (block A) and XB (block B) in, YA and YB
// out, one 32-row block at a time; each weight fragment feeds both blocks.
// Fragments are loaded kPrefetch k-steps ahead of their products; the
// scheduling barriers hold that order (at its register limit the compiler
// would otherwise load each fragment just before its products and wait out
// the LDS latency) and keep the next row block's loads below the activation.
constexpr int kPrefetch = 2;

template <int KS>
__device__ inline void pair_layer(const f16x8* W, const f32x16* bias, int lane, int h,
                                  const f16x8* XA, const f16x8* XB, f16x8* YA, f16x8* YB) {
  constexpr int D = KS < kPrefetch ? KS : kPrefetch;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const f16x8* Wr = W + rb * KS * 64 + lane;
    // the bias enters as the first product's addend (FP32, no vector instruction)
    const f32x16 c = bias[rb * 2 + h];
    f16x8 w[KS];
#pragma unroll
    for (int t = 0; t <= D && t < KS; ++t) w[t] = Wr[t * 64];
    f32x16 a = mfma(w[0], XA[0], c), b = mfma(w[0], XB[0], c);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 1; t < KS; ++t) {
      if (t + D < KS) w[t + D] = Wr[(t + D) * 64];
      a = mfma(w[t], XA[t], a);
      b = mfma(w[t], XB[t], b);
      __builtin_amdgcn_sched_barrier(0);
    }
    activate(a, &YA[2 * rb]);
    activate(b, &YB[2 * rb]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The 64 points of a tile: block A = points 0..31, block B = points 32..63.
// (xa, ya, za) / (xb, yb, zb): normalised coordinates of points l % 32 and
// 32 + l % 32 (every lane supplies both); returns the 5 outputs of point l.
__device__ inline void mlp_tile(const unsigned char* lds, int lane, float xa, float ya, float za,
                                float xb, float yb, float zb, float out[5]) {
  const int h = lane >> 5;
  const float* fq = reinterpret_cast<const float*>(lds + kMlpOffFourier);
  f16x8 XA[8], XB[8], YA[8], YB[8];
  fourier_operand(fq, xa, ya, za, h, XA);
  fourier_operand(fq, xb, yb, zb, h, XB);
  const f32x16* bias = reinterpret_cast<const f32x16*>(lds + kMlpOffBias);  // [layer][rb][h]
  constexpr int kBlk = kMlpBiasPerLayer / 16;
  pair_layer<2>(reinterpret_cast<const f16x8*>(lds + kMlpOffW0), bias, lane, h, XA, XB, YA, YB);
  pair_layer<8>(reinterpret_cast<const f16x8*>(lds + kMlpOffW1), bias + kBlk, lane, h, YA, YB,
                XA, XB);
  pair_layer<8>(reinterpret_cast<const f16x8*>(lds + kMlpOffW1 + kMlpHiddenBytes),
                bias + 2 * kBlk, lane, h, XA, XB, YA, YB);
  pair_layer<8>(reinterpret_cast<const f16x8*>(lds + kMlpOffW1 + 2 * kMlpHiddenBytes),
                bias + 3 * kBlk, lane, h, YA, YB, XA, XB);
  // output layer: registers 0..4 hold the 5 outputs in the lanes of the
  // block's half (see the file comment)
  const f16x8* W = reinterpret_cast<const f16x8*>(lds + kMlpOffWout);
  f32x16 oa = {}, ob = {};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const f16x8 w = W[t * 64 + lane];
    oa = mfma(w, XA[t], oa);
    ob = mfma(w, XB[t], ob);
  }
  const float* bout = reinterpret_cast<const float*>(lds + kMlpOffBout);
  const bool lo_half = lane < 32;
#pragma unroll
  for (int k = 0; k < 5; ++k) out[k] = (lo_half ? oa[k] : ob[k]) + bout[k];
}

// ---------------------------------------------------------------------------
// Fused march with MLP fields.  A wavefront owns a sightline; the pixel loop
// is wavefront-uniform (the matrix instructions need the whole wavefront).
// ---------------------------------------------------------------------------
template <int MF>
__global__ __launch_bounds__(512) void k_forward_mlp(GeomArgs g, FreqArgs fa, EmitArgs ea,
                                                     MlpArgs m, float* __restrict__ maps,
                                                     double* __restrict__ phi_end) {
  extern __shared__ __align__(16) unsigned char lds[];
  stage_weights(m.packed, lds, 512);
  const int lane = threadIdx.x & 63;
  const int n32 = lane & 31;
  const int64_t nwaves = (int64_t)gridDim.x * 8;
  for (int64_t q = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 6); q < g.npix; q += nwaves) {
    const Ray ray = make_ray(g, q);
    double carry = 0.0, accI = 0.0, accQ[MF], accU[MF];
#pragma unroll
    for (int f = 0; f < MF; ++f) accQ[f] = accU[f] = 0.0;
    for (int c0 = 0; c0 < g.n_steps; c0 += 64) {
      // normalised coordinates of the two points this lane feeds
      float cx[2], cy[2], cz[2];
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) {
        const double s = ((double)(c0 + 32 * pb + n32) + 0.5) * ray.dkpc;
        cx[pb] = ((float)(g.r_obs[0] + s * ray.nx) - m.lo[0]) * m.scale[0] - 1.0f;
        cy[pb] = ((float)(g.r_obs[1] + s * ray.ny) - m.lo[1]) * m.scale[1] - 1.0f;
        cz[pb] = ((float)(g.r_obs[2] + s * ray.nz) - m.lo[2]) * m.scale[2] - 1.0f;
      }
      float o[5];
      mlp_tile(lds, lane, cx[0], cy[0], cz[0], cx[1], cy[1], cz[1], o);
      // this lane's own step
      const int n = c0 + lane;
      const bool act = n < g.n_steps;
      FV v;
      v.bx = o[0];
      v.by = o[1];
      v.bz = o[2];
      v.ne = fexp2(o[3] * kLog2e);
      v.n0 = fexp2(o[4] * kLog2e);
      const float bl = v.bx * ray.elx + v.by * ray.ely;
      const float bb = v.bx * ray.ebx + v.by * ray.eby + v.bz * ray.ebz;
      const double bpar = -((double)v.bx * ray.nx + (double)v.by * ray.ny + (double)v.bz * ray.nz);
      const double cn = act ? (double)v.ne * bpar : 0.0;
      const double incl = group_inclusive_scan<64>(cn, lane);
      const double psi = carry + incl - 0.5 * cn;
      carry += group_last<64>(incl);
      Emit e = emission(v.n0, bl, bb, ea.alpha3 != 0, ea.eI);
      if (!act) e.u = e.zr = e.zi = 0.0f;
      accI += (double)e.u;
      const double psid = psi * ray.dkpc;
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < fa.n_freq) {
          float sn, cs;
          sincos_turns(psid * fa.kappa[f], &sn, &cs);
          accQ[f] += (double)(e.zr * cs - e.zi * sn);
          accU[f] += (double)(e.zr * sn + e.zi * cs);
        }
      }
    }
    accI = group_sum<64>(accI);
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      accQ[f] = group_sum<64>(accQ[f]);
      accU[f] = group_sum<64>(accU[f]);
    }
    if (lane == 0) {
      const MapAddr ma{g.npix, 0};
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < fa.n_freq) {
          maps[ma.at(f, 0, ray.ring)] = (float)(fa.sI[f] * ray.dkpc * accI);
          maps[ma.at(f, 1, ray.ring)] = (float)(fa.sP[f] * ray.dkpc * accQ[f]);
          maps[ma.at(f, 2, ray.ring)] = (float)(fa.sP[f] * ray.dkpc * accU[f]);
        }
      }
      if (phi_end != nullptr) phi_end[ray.ring] = carry;
    }
  }
}

// Point evaluation through the same tile code: out[n][5] = (Bx, By, Bz, n_e, N0).
__global__ __launch_bounds__(512) void k_eval_mlp(MlpArgs m, int64_t n, const float* __restrict__ xyz,
                                                  float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char lds[];
  stage_weights(m.packed, lds, 512);
  const int lane = threadIdx.x & 63;
  const int n32 = lane & 31;
  const int64_t ntiles = (n + 63) / 64;
  for (int64_t tile = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 6); tile < ntiles;
       tile += (int64_t)gridDim.x * 8) {
    float cx[2], cy[2], cz[2];
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
      int64_t i = tile * 64 + 32 * pb + n32;
      i = i < n ? i : n - 1;
      cx[pb] = (xyz[3 * i + 0] - m.lo[0]) * m.scale[0] - 1.0f;
      cy[pb] = (xyz[3 * i + 1] - m.lo[1]) * m.scale[1] - 1.0f;
      cz[pb] = (xyz[3 * i + 2] - m.lo[2]) * m.scale[2] - 1.0f;
    }
    float o[5];
    mlp_tile(lds, lane, cx[0], cy[0], cz[0], cx[1], cy[1], cz[1], o);
    const int64_t i = tile * 64 + lane;
    if (i < n) {
      out[5 * i + 0] = o[0];
      out[5 * i + 1] = o[1];
      out[5 * i + 2] = o[2];
      out[5 * i + 3] = fexp2(o[3] * kLog2e);
      out[5 * i + 4] = fexp2(o[4] * kLog2e);
    }
  }
}

static int mlp_grid_blocks() {
  int cus = 256;
  if (device_cus(&cus) != hipSuccess) cus = 256;
  return cus;
}

// Lifts a kernel's dynamic LDS limit to the packed weights, once per device.
static hipError_t mlp_lds_attr(const void* fn, PerDevice& done) {
  int one = 0;
  return done.get(&one, [fn](int* out) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMlpBytes);
    *out = 1;
    return e;
  });
}

template <int MF>
static hipError_t fwd_mlp_go(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const MlpArgs& m, float* maps, double* phi_end, hipStream_t st) {
  static PerDevice attr_done;
  hipError_t e = mlp_lds_attr(reinterpret_cast<const void*>(k_forward_mlp<MF>), attr_done);
  if (e != hipSuccess) return e;
  int64_t blocks = mlp_grid_blocks();
  const int64_t need = (g.npix + 7) / 8;
  if (blocks > need) blocks = need;
  k_forward_mlp<MF><<<dim3((unsigned)blocks), dim3(512), kMlpBytes, st>>>(g, fa, ea, m, maps, phi_end);
  return hipGetLastError();
}

hipError_t launch_forward_mlp(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                              const MlpArgs& m, float* maps, double* phi_end, hipStream_t st) {
  if (fa.n_freq <= 1) return fwd_mlp_go<1>(g, fa, ea, m, maps, phi_end, st);
  if (fa.n_freq <= 4) return fwd_mlp_go<4>(g, fa, ea, m, maps, phi_end, st);
  return fwd_mlp_go<16>(g, fa, ea, m, maps, phi_end, st);
}

hipError_t launch_eval_mlp(const MlpArgs& m, int64_t n, const float* xyz, float* out,
                           hipStream_t st) {
  static PerDevice attr_done;
  hipError_t e = mlp_lds_attr(reinterpret_cast<const void*>(k_eval_mlp), attr_done);
  if (e != hipSuccess) return e;
  int64_t blocks = mlp_grid_blocks();
  const int64_t need = ((n + 63) / 64 + 7) / 8;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  k_eval_mlp<<<dim3((unsigned)blocks), dim3(512), kMlpBytes, st>>>(m, n, xyz, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host-side packing.
// ---------------------------------------------------------------------------

// float -> IEEE binary16 bits, round to nearest even: overflow to +-inf, NaN
// kept quiet, subnormals rounded on the 2^-24 grid.
static uint16_t to_f16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  const uint32_t sign = (u >> 16) & 0x8000u, a = u & 0x7fffffffu;
  if (a >= 0x7f800000u) return (uint16_t)(sign | (a > 0x7f800000u ? 0x7e00u : 0x7c00u));
  if (a >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // 65520 and up round to inf
  if (a < 0x38800000u) {  // below 2^-14: a multiple of 2^-24 (the product is exact)
    float v;
    memcpy(&v, &a, 4);
    return (uint16_t)(sign | (uint32_t)std::nearbyint(v * 16777216.0f));
  }
  uint32_t h = (((a >> 23) - 112u) << 10) | ((a & 0x7fffffu) >> 13);
  const uint32_t rem = a & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;  // a carry into the exponent is right
  return (uint16_t)(sign | h);
}

// Input feature held in element i of the B operand of k-step t by lane half h,
// for layers fed by a previous layer's accumulator (see the file comment).
int mlp_feature_of_k(int t, int h, int i) {
  return 32 * (t / 2) + 16 * (t % 2) + 8 * (i / 4) + 4 * h + (i % 4);
}

// Row of a 32-row accumulator block held in register r by lane half h.
static int acc_row(int r, int h) { return (r % 4) + 8 * (r / 4) + 4 * h; }

}  // namespace sm

extern "C" {

size_t syn_mlp_packed_bytes(void) { return (size_t)sm::kMlpBytes; }

syn_status syn_mlp_pack(const float* fourier, const float* w_in, const float* b_in,
                        const float* w_h, const float* b_h, const float* w_out,
                        const float* b_out, void* packed_host) {
  using namespace sm;
  if (!fourier || !w_in || !b_in || !w_h || !b_h || !w_out || !b_out || !packed_host)
    return SYN_EINVAL;
  unsigned char* P = static_cast<unsigned char*>(packed_host);
  memset(P, 0, kMlpBytes);
  float* fq = reinterpret_cast<float*>(P + kMlpOffFourier);
  for (int i = 0; i < kMlpFourier * 3; ++i) fq[i] = fourier[i];
  // layer 0: A[m][k] = w_in[m][k], features in natural order k = 16 t + 8 h + i
  uint16_t* W0 = reinterpret_cast<uint16_t*>(P + kMlpOffW0);
  for (int rb = 0; rb < 4; ++rb)
    for (int t = 0; t < 2; ++t)
      for (int l = 0; l < 64; ++l)
        for (int i = 0; i < 8; ++i) {
          const int mrow = 32 * rb + (l % 32), k = 16 * t + 8 * (l / 32) + i;
          W0[(((rb * 2 + t) * 64) + l) * 8 + i] = to_f16(w_in[mrow * 32 + k]);
        }
  // hidden layers: A[m][k] = W[m][feature(k)]
  for (int layer = 0; layer < 3; ++layer) {
    uint16_t* W = reinterpret_cast<uint16_t*>(P + kMlpOffW1 + layer * kMlpHiddenBytes);
    const float* src = w_h + (size_t)layer * 128 * 128;
    for (int rb = 0; rb < 4; ++rb)
      for (int t = 0; t < 8; ++t)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < 8; ++i) {
            const int mrow = 32 * rb + (l % 32);
            W[(((rb * 8 + t) * 64) + l) * 8 + i] =
                to_f16(src[mrow * 128 + mlp_feature_of_k(t, l / 32, i)]);
          }
  }
  // output layer: outputs 0..4 at rows {0,1,2,3,8} and again at {4,5,6,7,12}
  static const int rowA[5] = {0, 1, 2, 3, 8}, rowB[5] = {4, 5, 6, 7, 12};
  uint16_t* WO = reinterpret_cast<uint16_t*>(P + kMlpOffWout);
  for (int t = 0; t < 8; ++t)
    for (int l = 0; l < 64; ++l)
      for (int i = 0; i < 8; ++i) {
        const int mrow = l % 32;
        int o = -1;
        for (int k = 0; k < 5; ++k)
          if (rowA[k] == mrow || rowB[k] == mrow) o = k;
        const float v = o >= 0 ? w_out[o * 128 + mlp_feature_of_k(t, l / 32, i)] : 0.0f;
        WO[((t * 64) + l) * 8 + i] = to_f16(v);
      }
  // biases in accumulator order: [layer][rb][h][r]
  float* bias = reinterpret_cast<float*>(P + kMlpOffBias);
  for (int layer = 0; layer < 4; ++layer) {
    const float* bsrc = layer == 0 ? b_in : b_h + (layer - 1) * 128;
    for (int rb = 0; rb < 4; ++rb)
      for (int h = 0; h < 2; ++h)
        for (int r = 0; r < 16; ++r)
          bias[layer * kMlpBiasPerLayer + (rb * 2 + h) * 16 + r] = bsrc[32 * rb + acc_row(r, h)];
  }
  float* bo = reinterpret_cast<float*>(P + kMlpOffBout);
  for (int k = 0; k < 5; ++k) bo[k] = b_out[k];
  return SYN_OK;
}

}  // extern "C"
