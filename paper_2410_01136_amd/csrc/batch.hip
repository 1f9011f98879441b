// Many parameter sets in one launch: persistent work-queue kernels.
//
// Work item = one block's worth of sightlines (256 / S pixels) of one set.
// Items of all sets are numbered consecutively (set s owns items
// [item0_s, item0_s + n_items_s)); a block takes the next item from a global
// counter until the counter passes the last item, so sets with different
// N_side balance by item count.  Each set carries its own geometry, field
// parameters and frequency prefactors (alpha differs between sets).
#include "batch.h"
#include "march_body.h"

namespace sm {

// Largest set index s with sets[s].item0 <= item (sets sorted by item0).
__device__ inline int find_set(const BatchSet* __restrict__ sets, int n_sets, int item) {
  int lo = 0, hi = n_sets - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sets[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Takes the next work item for the whole block; every thread gets the same value.
__device__ inline int next_item(unsigned int* counter) {
  __shared__ int s_item;
  if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(s_item);
  __syncthreads();
  return item;
}

__global__ void k_batch_reset(unsigned int* counters) {
  if (threadIdx.x < 2) counters[threadIdx.x] = 0u;
}

// Analytic fields of the sets, without a grid to scatter gradients into.
struct Model16NoScatter : Model16 {
  struct Acc {
    AdjBox box;
  };
};
struct WmapNoScatter : Wmap {
  struct Acc {
    AdjBox box;
  };
};

// The field of set B in a plan of the given kind.
template <bool WM>
__device__ inline auto set_field(const BatchSet& B) {
  if constexpr (WM)
    return WmapNoScatter{Wmap{B.w}};
  else
    return Model16NoScatter{Model16{B.m}};
}

template <int S, bool WM>
__global__ __launch_bounds__(256) void k_batch_fwd(const BatchSet* __restrict__ sets, int n_sets,
                                                   int n_items, unsigned int* counter,
                                                   int64_t total, float* __restrict__ maps,
                                                   double* __restrict__ phi_end) {
  using F = decltype(set_field<WM>(sets[0]));
  for (;;) {
    const int item = next_item(counter);
    if (item >= n_items) return;
    const BatchSet& B = sets[find_set(sets, n_sets, item)];
    const int sub = (int)(threadIdx.x & (S - 1));
    int64_t q = (int64_t)(item - B.item0) * (256 / S) + threadIdx.x / S;
    const bool valid = q < B.g.npix;
    if (!valid) q = B.g.npix - 1;
    fwd_lane<F, S, 1>(B.g, B.fa, B.ea, set_field<WM>(B), q, sub, valid, maps,
                      MapAddr{total, B.map_off}, phi_end);
  }
}

// (one lane per sightline, the plans' shape: held to 128 VGPRs, 4 wavefronts
// per SIMD, which it fits without spilling)
template <int S, bool WM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == 1 ? 4 : 1))) void
k_batch_adj(const BatchSet* __restrict__ sets, int n_sets, int n_items, unsigned int* counter,
            int64_t total, const float* __restrict__ dmaps, const double* __restrict__ phi_end,
            double* __restrict__ partials) {
  using F = decltype(set_field<WM>(sets[0]));
  for (;;) {
    const int item = next_item(counter);
    if (item >= n_items) return;
    const BatchSet& B = sets[find_set(sets, n_sets, item)];
    const int sub = (int)(threadIdx.x & (S - 1));
    int64_t q = (int64_t)(item - B.item0) * (256 / S) + threadIdx.x / S;
    const bool valid = q < B.g.npix;
    if (!valid) q = B.g.npix - 1;
    double tb[kNParam];
#pragma unroll
    for (int k = 0; k < kNParam; ++k) tb[k] = 0.0;
    adj_lane<F, S, 1, true, false>(B.g, B.fa, B.ea, set_field<WM>(B), q, sub, valid, dmaps,
                                   MapAddr{total, B.map_off}, phi_end, tb, nullptr, nullptr);
    const double r = block_reduce16(tb, threadIdx.x);
    if (threadIdx.x < kNParam) partials[(int64_t)item * kNParam + threadIdx.x] = r;
  }
}

// chi^2 of every set against its target (one block per set, fixed order).
__global__ __launch_bounds__(256) void k_batch_chi2(const BatchSet* __restrict__ sets,
                                                    int64_t total, const float* __restrict__ maps,
                                                    const float* __restrict__ target,
                                                    BatchChi2Args a, float* __restrict__ dmaps,
                                                    double* __restrict__ chi2) {
  const BatchSet& B = sets[blockIdx.x];
  const int64_t np = B.g.npix;
  double acc = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double w = a.inv_s2[k];
    for (int64_t p = threadIdx.x; p < np; p += 256) {
      const int64_t i = k * total + B.map_off + p;
      const double r = (double)maps[i] - (double)target[i];
      acc += w * r * r;
      dmaps[i] = (float)(2.0 * w * r);
    }
  }
  __shared__ double red[4];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) chi2[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dtheta of every set from its items' partials (one block per set, fixed order).
__global__ __launch_bounds__(256) void k_batch_reduce(const BatchSet* __restrict__ sets,
                                                      const double* __restrict__ partials,
                                                      double* __restrict__ dtheta) {
  const BatchSet& B = sets[blockIdx.x];
  __shared__ double red[16][17];
  const int k = threadIdx.x & 15, j = threadIdx.x >> 4;
  double acc = 0.0;
  for (int64_t it = j; it < B.n_items; it += 16) acc += partials[(B.item0 + it) * kNParam + k];
  red[j][k] = acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    double s = 0.0;
    for (int jj = 0; jj < 16; ++jj) s += red[jj][threadIdx.x];
    dtheta[(int64_t)blockIdx.x * kNParam + threadIdx.x] = s;
  }
}

template <int S, bool WM>
static int occupancy_blocks(bool adjoint) {
  int per_cu = 0;
  hipError_t e =
      adjoint ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_adj<S, WM>, 256, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_fwd<S, WM>, 256, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu;
}

template <bool WM>
static int blocks_per_cu(int S, bool adjoint) {
  switch (S) {
    case 1: return occupancy_blocks<1, WM>(adjoint);
    case 4: return occupancy_blocks<4, WM>(adjoint);
    case 16: return occupancy_blocks<16, WM>(adjoint);
    case 64: return occupancy_blocks<64, WM>(adjoint);
    default: return 1;
  }
}

int batch_blocks_per_cu(int S, bool adjoint, bool wmap) {
  return wmap ? blocks_per_cu<true>(S, adjoint) : blocks_per_cu<false>(S, adjoint);
}

template <int S, bool WM>
static hipError_t batch_go(const BatchLaunch& L, hipStream_t st) {
  k_batch_reset<<<1, 64, 0, st>>>(L.counters);
  k_batch_fwd<S, WM><<<L.blocks_fwd, 256, 0, st>>>(L.sets, L.n_sets, L.n_items, L.counters,
                                                   L.total, L.maps, L.phi);
  k_batch_chi2<<<L.n_sets, 256, 0, st>>>(L.sets, L.total, L.maps, L.target, L.chi2_args, L.dmaps,
                                         L.chi2);
  k_batch_adj<S, WM><<<L.blocks_adj, 256, 0, st>>>(L.sets, L.n_sets, L.n_items, L.counters + 1,
                                                   L.total, L.dmaps, L.phi, L.partials);
  k_batch_reduce<<<L.n_sets, 256, 0, st>>>(L.sets, L.partials, L.dtheta);
  return hipGetLastError();
}

template <bool WM>
static hipError_t batch_s(const BatchLaunch& L, hipStream_t st) {
  switch (L.S) {
    case 1: return batch_go<1, WM>(L, st);
    case 4: return batch_go<4, WM>(L, st);
    case 16: return batch_go<16, WM>(L, st);
    case 64: return batch_go<64, WM>(L, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch(const BatchLaunch& L, hipStream_t st) {
  return L.wmap ? batch_s<true>(L, st) : batch_s<false>(L, st);
}

}  // namespace sm
