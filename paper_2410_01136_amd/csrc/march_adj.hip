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
#include "march_body.h"
#include "sm_launch.h"

namespace sm {

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
  double tb[THETA ? kNParam : 1];
#pragma unroll
  for (int k = 0; k < (THETA ? kNParam : 1); ++k) tb[k] = 0.0;
  float* box = nullptr;
  if constexpr (GRID) {
    __shared__ float lds_box[kAdjBoxFloats];
    for (int j = threadIdx.x; j < kAdjBoxFloats; j += 256) lds_box[j] = 0.0f;
    __syncthreads();
    box = lds_box;
  }
  adj_lane<F, S, MF, THETA, GRID>(g, fa, ea, fld, q, sub, valid, dmaps, MapAddr{g.npix, 0}, phi_end,
                                  tb, gbn, gc, box);
  if constexpr (GRID) {
    __syncthreads();
    fld.flush_box(box, gbn, gc, threadIdx.x, 256);
  }
  if constexpr (THETA) {
    const double r = block_reduce16(tb, threadIdx.x);
    if (threadIdx.x < kNParam) partials[blk * kNParam + threadIdx.x] = r;
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
  struct Acc {
    float* lds = nullptr;
  };
  __device__ inline void accumulate_at(const GeomArgs&, const Ray&, double, const FV&, Acc&, float*,
                                       float*) const {}
  __device__ inline void flush(Acc&, float*, float*) const {}
  __device__ inline void flush_box(const float*, float*, float*, int, int) const {}
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
