// Small kernels around the march: the chi^2 cotangent, sampling the analytic
// model onto grid nodes, and point evaluation of any field kind.
#include <atomic>
#include <mutex>

#include "sm_device.h"
#include "sm_launch.h"

namespace sm {

constexpr int kMaxMaps = 3 * kMaxFreq;

struct Chi2Args {
  double inv_s2[kMaxMaps];
};

// Gaussian chi^2 of the maps against a target (log-likelihood of Sec. 3.1 with
// one noise level per Stokes map) and its gradient.  Each block owns a fixed
// strided slice, so the FP64 partial sums do not depend on timing.
__global__ __launch_bounds__(256) void k_chi2(int64_t n_pix, int n_maps, const float* __restrict__ m,
                                              const float* __restrict__ t, Chi2Args a,
                                              float* __restrict__ dm, double* __restrict__ part) {
  const int64_t total = n_pix * n_maps;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += stride) {
    const int mi = (int)(i / n_pix);
    const double r = (double)m[i] - (double)t[i];
    acc += a.inv_s2[mi] * r * r;
    if (dm != nullptr) dm[i] = (float)(2.0 * a.inv_s2[mi] * r);
  }
  __shared__ double red[4];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_sum_fixed(const double* __restrict__ part, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

int64_t chi2_partials(int64_t n_pix, int n_maps) {
  const int64_t total = n_pix * n_maps;
  int64_t nb = (total + 256 * 8 - 1) / (256 * 8);
  if (nb < 1) nb = 1;
  if (nb > kChi2MaxPartials) nb = kChi2MaxPartials;
  return nb;
}

// Scratch of the chi^2 entry point that allocates nothing: its per-block FP64
// partial sums live in this file-scope device array (32 KiB; every GPU the
// library runs on holds its own copy until the process ends).  k_chi2 writes
// every partial that k_sum_fixed then reads, so nothing needs clearing between
// calls; calls that overlap on one GPU share the array and race.
static __device__ __align__(256) double scratch[kChi2MaxPartials];

namespace {
constexpr int kMaxScratchDevices = 64;
std::atomic<double*> g_scratch_ptr[kMaxScratchDevices];
std::mutex g_scratch_mu;
}  // namespace

// Device address of the current GPU's copy of the chi^2 scratch array, looked up
// once per device (with that device current) and kept.
hipError_t chi2_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  double* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p == nullptr) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (p == nullptr) {
      void* a = nullptr;
      e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      p = static_cast<double*>(a);
      g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return hipSuccess;
}

hipError_t launch_chi2(int64_t n_pix, int n_maps, const float* maps, const float* target,
                       const double* inv_s2, float* dmaps, double* chi2, double* partials,
                       int64_t n_partials, hipStream_t st) {
  Chi2Args a{};
  for (int i = 0; i < n_maps; ++i) a.inv_s2[i] = inv_s2[i];
  k_chi2<<<dim3((unsigned)n_partials), dim3(256), 0, st>>>(n_pix, n_maps, maps, target, a, dmaps,
                                                          partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (chi2 != nullptr) {
    k_sum_fixed<<<dim3(1), dim3(256), 0, st>>>(partials, n_partials, chi2);
    e = hipGetLastError();
  }
  return e;
}

// One Adam update (Kingma & Ba 2015, Algorithm 1), elementwise; the bias
// corrections c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) come from the host.
// Element i takes part iff bit (i % period) of mask is set.  The float4 form
// takes four consecutive elements per thread (period divides 4, arrays 16-byte
// aligned, n a multiple of 4); the scalar form takes any layout.
struct AdamArgs {
  float b1, b2, omb1, omb2;  // beta1, beta2, 1 - beta1, 1 - beta2
  float c1, c2, lr, eps;
  int period;
  uint32_t mask;
};

__device__ inline void adam_one(const AdamArgs& a, float& p, float g, float& m, float& v) {
  m = a.b1 * m + a.omb1 * g;
  v = a.b2 * v + a.omb2 * (g * g);
  p = p - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

__global__ __launch_bounds__(256) void k_adam4(int64_t n4, AdamArgs a, float4* __restrict__ p,
                                               const float4* __restrict__ g, float4* __restrict__ m,
                                               float4* __restrict__ v) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const bool on0 = (a.mask >> (0 % a.period)) & 1u, on1 = (a.mask >> (1 % a.period)) & 1u;
  const bool on2 = (a.mask >> (2 % a.period)) & 1u, on3 = (a.mask >> (3 % a.period)) & 1u;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
    float4 pp = p[i], mm = m[i], vv = v[i];
    const float4 gg = g[i];
    if (on0) adam_one(a, pp.x, gg.x, mm.x, vv.x);
    if (on1) adam_one(a, pp.y, gg.y, mm.y, vv.y);
    if (on2) adam_one(a, pp.z, gg.z, mm.z, vv.z);
    if (on3) adam_one(a, pp.w, gg.w, mm.w, vv.w);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

__global__ __launch_bounds__(256) void k_adam1(int64_t n, AdamArgs a, float* __restrict__ p,
                                               const float* __restrict__ g, float* __restrict__ m,
                                               float* __restrict__ v) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    if (!((a.mask >> (int)(i % a.period)) & 1u)) continue;
    float pp = p[i], mm = m[i], vv = v[i];
    adam_one(a, pp, g[i], mm, vv);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

hipError_t launch_adam(int64_t n, int period, uint32_t mask, float* p, const float* g, float* m,
                       float* v, int t, double lr, double b1, double b2, double eps,
                       hipStream_t st) {
  AdamArgs a;
  a.b1 = (float)b1;
  a.b2 = (float)b2;
  a.omb1 = (float)(1.0 - b1);
  a.omb2 = (float)(1.0 - b2);
  a.c1 = (float)(1.0 / (1.0 - pow(b1, (double)t)));
  a.c2 = (float)(1.0 / (1.0 - pow(b2, (double)t)));
  a.lr = (float)lr;
  a.eps = (float)eps;
  a.period = period;
  a.mask = mask;
  const bool vec = (n % 4 == 0) && (4 % period == 0) &&
                   ((((uintptr_t)p | (uintptr_t)g | (uintptr_t)m | (uintptr_t)v) & 15) == 0);
  const int64_t work = vec ? n / 4 : n;
  int64_t nb = (work + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  if (vec)
    k_adam4<<<dim3((unsigned)nb), dim3(256), 0, st>>>(n / 4, a, reinterpret_cast<float4*>(p),
                                                      reinterpret_cast<const float4*>(g),
                                                      reinterpret_cast<float4*>(m),
                                                      reinterpret_cast<float4*>(v));
  else
    k_adam1<<<dim3((unsigned)nb), dim3(256), 0, st>>>(n, a, p, g, m, v);
  return hipGetLastError();
}

struct NodeGrid {
  int32_t n[3];
  double lo[3], h[3];
};

__global__ __launch_bounds__(256) void k_sample_model16(Model16 m, NodeGrid ng, float* out_bn,
                                                        float* out_c) {
  const int64_t nv = (int64_t)ng.n[0] * ng.n[1] * ng.n[2];
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nv) return;
  const int64_t ix = v % ng.n[0];
  const int64_t iy = (v / ng.n[0]) % ng.n[1];
  const int64_t iz = v / ((int64_t)ng.n[0] * ng.n[1]);
  const float x = (float)(ng.lo[0] + ng.h[0] * (double)ix);
  const float y = (float)(ng.lo[1] + ng.h[1] * (double)iy);
  const float z = (float)(ng.lo[2] + ng.h[2] * (double)iz);
  const FV f = m.eval(x, y, z);
  if (out_bn != nullptr) reinterpret_cast<float4*>(out_bn)[v] = make_float4(f.bx, f.by, f.bz, f.ne);
  if (out_c != nullptr) out_c[v] = f.n0;
}

hipError_t launch_sample_model16(const M16Args& m, const int32_t n[3], const double lo[3],
                                 const double hi[3], float* out_bn, float* out_c,
                                 hipStream_t st) {
  NodeGrid ng;
  for (int k = 0; k < 3; ++k) {
    ng.n[k] = n[k];
    ng.lo[k] = lo[k];
    ng.h[k] = (hi[k] - lo[k]) / (double)(n[k] - 1);
  }
  const int64_t nv = (int64_t)n[0] * n[1] * n[2];
  k_sample_model16<<<dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st>>>(Model16{m}, ng, out_bn,
                                                                            out_c);
  return hipGetLastError();
}

template <class F>
__global__ __launch_bounds__(256) void k_eval_fields(F fld, int64_t n, const float* __restrict__ xyz,
                                                     float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const FV f = fld.eval_point(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
  out[5 * i + 0] = f.bx;
  out[5 * i + 1] = f.by;
  out[5 * i + 2] = f.bz;
  out[5 * i + 3] = f.ne;
  out[5 * i + 4] = f.n0;
}

hipError_t launch_eval_fields(const FieldPack& fp, int64_t n, const float* xyz, float* out,
                              hipStream_t st) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (fp.kind) {
    case kModel16: k_eval_fields<<<grid, block, 0, st>>>(Model16{fp.m16}, n, xyz, out); break;
    case kGrid:
      k_eval_fields<<<grid, block, 0, st>>>(Grid{fp.grid, Model16{fp.m16}}, n, xyz, out);
      break;
    case kSphere: k_eval_fields<<<grid, block, 0, st>>>(Sphere{fp.sph}, n, xyz, out); break;
    case kWmap: k_eval_fields<<<grid, block, 0, st>>>(Wmap{fp.wmap}, n, xyz, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sm
