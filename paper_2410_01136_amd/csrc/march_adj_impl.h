// Reverse-march kernels and their launch-shape dispatch, templated on free-free
// (FF) and the spectral model (SP).  Included by one march_adj*.hip file per
// (FF, SP) pair so that the sets of kernels compile in parallel.
#pragma once

#include <algorithm>
#include <type_traits>

#include "march_body.h"
#include "sm_launch.h"

namespace sm {

// Reaches (kpc from the observer) tried for a workgroup's LDS box: 64 / 2^c.
constexpr int kBoxReaches = 10;

// The LDS accumulation box of one workgroup of the grid adjoint: the bounding
// box of the first D kpc of all its sightlines (every sightline starts at the
// observer, and a workgroup's sightlines form a compact sky patch, so this cone
// section is where its gradients pile up), for the largest D = 64 / 2^c whose
// box holds at most `cap` nodes.  Collective over the workgroup; zeroes the box.
template <class F>
__device__ inline AdjBox workgroup_box(const GeomArgs& g, const F& fld, int64_t q, float* lds,
                                       int cap) {
  __shared__ int s_rng[kBoxReaches][6];  // per reach: lowest node, highest node + 1 per axis
  __shared__ int s_box[7];               // b0[3], d[3], in use
  for (int j = threadIdx.x; j < kBoxReaches * 6; j += blockDim.x)
    (&s_rng[0][0])[j] = (j % 6) < 3 ? INT_MAX : INT_MIN;
  __syncthreads();
  const Ray r = make_ray(g, q);
  const double L = r.dkpc * (double)g.n_steps;
  const double n3[3] = {r.nx, r.ny, r.nz};
  for (int c = 0; c < kBoxReaches; ++c) {
    const double D = fmin(64.0 / (double)(1 << c), L);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double u0 = (g.r_obs[k] - fld.p.lo[k]) * fld.p.inv_h[k];
      const double u1 = u0 + D * n3[k] * fld.p.inv_h[k];
      // clamped to just outside the grid, so the conversions are defined
      const double a = fmax(fmin(u0, u1), -1.0), b = fmin(fmax(u0, u1), fld.p.umax[k] + 1.0);
      atomicMin(&s_rng[c][k], (int)floor(a));
      atomicMax(&s_rng[c][3 + k], (int)floor(b) + 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_box[6] = 0;
    for (int c = 0; c < kBoxReaches; ++c) {
      int lo[3], d[3];
      int64_t cnt = 1;
      for (int k = 0; k < 3; ++k) {
        lo[k] = min(max(s_rng[c][k], 0), fld.p.n[k] - 1);
        const int hi = min(s_rng[c][3 + k], fld.p.n[k] - 1);
        d[k] = max(hi - lo[k] + 1, 1);
        cnt *= d[k];
      }
      if (cnt <= cap) {
        for (int k = 0; k < 3; ++k) {
          s_box[k] = lo[k];
          s_box[3 + k] = d[k];
        }
        s_box[6] = 1;
        break;
      }
    }
  }
  __syncthreads();
  AdjBox B;
  if (s_box[6]) {
    for (int k = 0; k < 3; ++k) {
      B.b0[k] = s_box[k];
      B.d[k] = s_box[3 + k];
    }
    B.lds = lds;
    const int nf = 5 * B.d[0] * B.d[1] * B.d[2];
    for (int j = threadIdx.x; j < nf; j += blockDim.x) lds[j] = 0.0f;
  }
  __syncthreads();
  return B;
}

template <class F, int S, int MF, bool THETA, bool GRID, bool FF, int SP>
__global__ __launch_bounds__(256) void k_adjoint(GeomArgs g, FreqArgs fa, EmitArgs ea, F fld,
                                                 const float* __restrict__ dmaps,
                                                 const double* __restrict__ phi_end,
                                                 const double* __restrict__ em_end,
                                                 double* __restrict__ partials, float* gbn,
                                                 float* gc, int box_cap) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t tid = blk * 256 + threadIdx.x;
  const int sub = (int)(threadIdx.x & (S - 1));
  int64_t q = tid / S;
  const bool valid = q < g.npix;
  if (!valid) q = g.npix - 1;
  // theta partials; a broken spectrum adds its two parameters after theta
  constexpr int NPT = THETA ? (SP == kSpecBroken ? kNParam + 2 : kNParam) : 1;
  double tb[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) tb[k] = 0.0;
  AdjBox box;
  float* stage = nullptr;
  if constexpr (GRID) {
    // box_cap nodes x 5 floats, then kStageRecs records per wavefront
    extern __shared__ float lds_dyn[];
    box = workgroup_box(g, fld, q, lds_dyn, box_cap);
    stage = lds_dyn + 5 * box_cap + (threadIdx.x >> 6) * (kStageRecs * kStageFloats);
  }
  // a theta-only pass walks contiguous pieces too (from the forward's piece
  // snapshots, or a pre-pass without them), except under a broken power law,
  // whose reverse pass measured faster with interleaved steps
  constexpr bool PIECES = THETA && SP != kSpecBroken;
  adj_lane<F, S, MF, THETA, GRID, FF, SP, PIECES>(g, fa, ea, fld, q, sub, valid, dmaps,
                                          MapAddr{g.npix, 0}, phi_end, tb, gbn, gc, &box, stage,
                                          em_end);
  if constexpr (GRID) {
    __syncthreads();
    fld.flush_box(box, gbn, gc, threadIdx.x, 256);
  }
  if constexpr (THETA) {
    const double r = block_reduce<NPT>(tb, threadIdx.x);
    if (threadIdx.x < NPT) partials[blk * NPT + threadIdx.x] = r;
  }
}

// Sums the per-block partials (NP per block) in a fixed order: G strided
// groups of lanes per parameter, then a fixed sum over the groups.
template <class T, int NP = kNParam>
__global__ __launch_bounds__(256) void k_reduce_partials(const T* __restrict__ partials,
                                                         int64_t nblk, T* __restrict__ out) {
  constexpr int L = NP <= 16 ? 16 : 32;  // lanes per group (>= NP)
  constexpr int G = 256 / L;
  static_assert(NP <= 32, "at most 32 parameters");
  __shared__ T red[G][L + 1];
  const int k = threadIdx.x & (L - 1), j = threadIdx.x / L;
  T acc = 0.0;
  if (k < NP)
    for (int64_t b = j; b < nblk; b += G) acc += partials[b * NP + k];
  red[j][k] = acc;
  __syncthreads();
  if (threadIdx.x < NP) {
    T s = 0.0;
    for (int jj = 0; jj < G; ++jj) s += red[jj][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

template <bool FF, int SP, class F, int S, int MF, bool TH, bool GR>
static hipError_t adj_go(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         const float* dm, const double* pe, const double* ee, double* part,
                         double* dth, float* gbn, float* gc, hipStream_t st) {
  const int64_t nb = march_blocks(g.npix, S);
  int cap = 0;
  size_t lds = 0;
  if (GR) {
    // the LDS of a CU is shared by the workgroups it runs at once (at most four
    // here, fewer when registers or the grid size allow no more)
    int n_cu = 0;
    hipError_t e0 = device_cus(&n_cu);
    if (e0 != hipSuccess) return e0;
    // workgroups one CU can hold with the smallest box (registers permitting);
    // the first call on a device also lifts the kernel's dynamic LDS limit there
    static PerDevice regs_cache;
    int by_regs = 0;
    e0 = regs_cache.get(&by_regs, [](int* out) {
      const void* fn = reinterpret_cast<const void*>(&k_adjoint<F, S, MF, TH, GR, FF, SP>);
      hipError_t e = hipFuncSetAttribute(
          fn, hipFuncAttributeMaxDynamicSharedMemorySize,
          (int)((size_t)kAdjBoxNodesMax * 5 * sizeof(float) + kStageBytesPerBlock));
      if (e != hipSuccess) return e;
      int nblk = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nblk, fn, 256, (size_t)adj_box_cap(4) * 5 * sizeof(float) + kStageBytesPerBlock);
      if (e != hipSuccess) return e;
      *out = std::min(std::max(nblk, 1), 4);
      return hipSuccess;
    });
    if (e0 != hipSuccess) return e0;
    // the box takes the LDS share of one of the workgroups that run on a CU at once
    const int per_cu = (int)std::min<int64_t>(by_regs, (nb + n_cu - 1) / n_cu);
    cap = adj_box_cap(per_cu);
    lds = (size_t)cap * 5 * sizeof(float) + kStageBytesPerBlock;
  }
  k_adjoint<F, S, MF, TH, GR, FF, SP><<<dim3((unsigned)nb), dim3(256), lds, st>>>(
      g, fa, ea, f, dm, pe, ee, part, gbn, gc, cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (TH) {
    constexpr int NPT = SP == kSpecBroken ? kNParam + 2 : kNParam;
    k_reduce_partials<double, NPT><<<dim3(1), dim3(256), 0, st>>>(part, nb, dth);
    e = hipGetLastError();
  }
  return e;
}

template <bool FF, int SP, class F, int S, int MF>
static hipError_t adj_flags(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                            const float* dm, const double* pe, const double* ee, double* part,
                            double* dth, float* gbn, float* gc, hipStream_t st) {
  const bool th = dth != nullptr, gr = (gbn != nullptr || gc != nullptr);
  if constexpr (std::is_same_v<F, Grid>) {
    if (th && gr)
      return adj_go<FF, SP, F, S, MF, true, true>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
    if (gr) return adj_go<FF, SP, F, S, MF, false, true>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
  } else {
    if (gr) return hipErrorInvalidValue;  // only gridded fields have grid gradients
  }
  if (th) return adj_go<FF, SP, F, S, MF, true, false>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
  return hipSuccess;
}

template <bool FF, int SP, class F, int S>
static hipError_t adj_mf(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                         const float* dm, const double* pe, const double* ee, double* part,
                         double* dth, float* gbn, float* gc, hipStream_t st) {
  if (fa.n_freq <= 1) return adj_flags<FF, SP, F, S, 1>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
  if (fa.n_freq <= 4) return adj_flags<FF, SP, F, S, 4>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
  return adj_flags<FF, SP, F, S, 16>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
}

template <bool FF, int SP, class F>
static hipError_t adj_s(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea, const F& f,
                        int S, const float* dm, const double* pe, const double* ee, double* part,
                        double* dth, float* gbn, float* gc, hipStream_t st) {
  switch (S) {
    case 1: return adj_mf<FF, SP, F, 1>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
    case 4: return adj_mf<FF, SP, F, 4>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
    case 8: return adj_mf<FF, SP, F, 8>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
    case 16: return adj_mf<FF, SP, F, 16>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
    case 64: return adj_mf<FF, SP, F, 64>(g, fa, ea, f, dm, pe, ee, part, dth, gbn, gc, st);
    default: return hipErrorInvalidValue;
  }
}

// Model16 fields have no grid to scatter into.
struct Model16NoGrid : Model16 {
  struct Acc {
    AdjBox box;
  };
};

// The WMAP field has no grid to scatter into either.
struct WmapNoGrid : Wmap {
  struct Acc {
    AdjBox box;
  };
};

// SP: spectral model (kSpecPower, kSpecGridAlpha: gridded index, grid fields
// only; kSpecBroken: broken power law).
template <bool FF, int SP>
static hipError_t launch_adjoint_t(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                   const FieldPack& fp, int S, const float* dmaps,
                                   const double* phi_end, const double* em_end, double* partials,
                                   double* dtheta, float* gbn, float* gc, hipStream_t st) {
  if (fp.kind == kGrid)
    return adj_s<FF, SP>(g, fa, ea, Grid{fp.grid, Model16{fp.m16}}, S, dmaps, phi_end, em_end,
                         partials, dtheta, gbn, gc, st);
  if constexpr (SP != kSpecGridAlpha) {
    switch (fp.kind) {
      case kModel16:
        return adj_s<FF, SP>(g, fa, ea, Model16NoGrid{Model16{fp.m16, fp.snap}}, S, dmaps, phi_end, em_end,
                             partials, dtheta, nullptr, nullptr, st);
      case kWmap:
        return adj_s<FF, SP>(g, fa, ea, WmapNoGrid{Wmap{fp.wmap, fp.snap}}, S, dmaps, phi_end, em_end,
                             partials, dtheta, nullptr, nullptr, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace sm
