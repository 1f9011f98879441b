// Host-side launchers of the march kernels (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>

#include "sm_params.h"

namespace sm {

// A value computed once per device on first use (a kernel attribute set, an
// occupancy or CU count), safe to read from several host threads; 0 means not
// yet computed.  The calling thread's current device is the one meant.
struct PerDevice {
  static constexpr int kMaxDevices = 64;
  std::atomic<int> v[kMaxDevices] = {};
  template <class Fn>  // Fn: hipError_t(int* out)
  hipError_t get(int* out, Fn&& compute) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return compute(out);
    const int have = v[dev].load(std::memory_order_acquire);
    if (have != 0) {
      *out = have;
      return hipSuccess;
    }
    e = compute(out);
    if (e == hipSuccess) v[dev].store(*out, std::memory_order_release);
    return e;
  }
};

// Multiprocessor (CU) count of the current device.
inline hipError_t device_cus(int* out) {
  static PerDevice cache;
  return cache.get(out, [](int* o) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(o, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && *o < 1) *o = 1;
    return e;
  });
}

enum FieldKind { kModel16 = 0, kGrid = 1, kSphere = 2, kMlp = 3, kWmap = 4 };

// How the gridded forward reads the grid: 64-bit addresses, 32-bit buffer
// offsets per lane, or buffer reads of each distinct cell shared through LDS.
enum GridPath { kGridGlobal = 0, kGridBuffer = 1, kGridShared = 2 };

struct MlpArgs {
  const void* packed;     // device, layout of mlp_layout.h
  float lo[3], scale[3];  // x^ = (r - lo) * scale - 1, scale = 2 / (hi - lo)
};

struct FieldPack {
  int kind;
  M16Args m16;
  GridArgs grid;
  int grid_path = 0;  // forward's grid reads: GridPath
  SphereArgs sph;
  MlpArgs mlp;
  WmapArgs wmap;
  SnapArgs snap;  // piece snapshots of the analytic and WMAP fields (grids: in grid)
  bool ff = false;  // free-free emission and absorption (constants in FreqArgs)
  int spec = kSpecPower;  // kSpecBroken: broken power law (table and constants in EmitArgs, FreqArgs)
};

// Number of 256-thread blocks a launch with S lanes per sightline uses.
inline int64_t march_blocks(int64_t npix, int S) { return (npix * S + 255) / 256; }

// phi_end, em_end: per-sightline Faraday sum and (free-free) emission-measure
// sum the adjoint starts from, or nullptr when no adjoint follows
hipError_t launch_forward(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                          const FieldPack& fp, int S, float* maps, double* phi_end,
                          double* em_end, hipStream_t st);
hipError_t launch_forward_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, float* maps, double* phi_end,
                             double* em_end, hipStream_t st);
hipError_t launch_forward_va(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, float* maps, double* phi_end,
                             double* em_end, hipStream_t st);
hipError_t launch_forward_va_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                const FieldPack& fp, int S, float* maps, double* phi_end,
                                double* em_end, hipStream_t st);
hipError_t launch_forward_bp(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, float* maps, double* phi_end,
                             double* em_end, hipStream_t st);
hipError_t launch_forward_bp_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                const FieldPack& fp, int S, float* maps, double* phi_end,
                                double* em_end, hipStream_t st);

// partials: [march_blocks(npix, S)][16] doubles; dtheta: device double[16]
hipError_t launch_adjoint(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                          const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                          const double* em_end, double* partials, double* dtheta, float* gbn,
                          float* gc, hipStream_t st);
hipError_t launch_adjoint_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                             const double* em_end, double* partials, double* dtheta, float* gbn,
                             float* gc, hipStream_t st);
hipError_t launch_adjoint_va(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                             const double* em_end, double* partials, double* dtheta, float* gbn,
                             float* gc, hipStream_t st);
hipError_t launch_adjoint_va_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                const FieldPack& fp, int S, const float* dmaps,
                                const double* phi_end, const double* em_end, double* partials,
                                double* dtheta, float* gbn, float* gc, hipStream_t st);
hipError_t launch_adjoint_bp(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                             const FieldPack& fp, int S, const float* dmaps, const double* phi_end,
                             const double* em_end, double* partials, double* dtheta, float* gbn,
                             float* gc, hipStream_t st);
hipError_t launch_adjoint_bp_ff(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                                const FieldPack& fp, int S, const float* dmaps,
                                const double* phi_end, const double* em_end, double* partials,
                                double* dtheta, float* gbn, float* gc, hipStream_t st);

hipError_t launch_chi2(int64_t n_pix, int n_maps, const float* maps, const float* target,
                       const double* inv_s2, float* dmaps, double* chi2, double* partials,
                       int64_t n_partials, hipStream_t st);
int64_t chi2_partials(int64_t n_pix, int n_maps);
// Largest number of chi^2 partial sums (the block count is capped here), and
// the device address of the current GPU's static scratch array that holds
// that many for the entry point that allocates nothing.
constexpr int64_t kChi2MaxPartials = 4096;
hipError_t chi2_scratch(double** out);

hipError_t launch_adam(int64_t n, int period, uint32_t mask, float* p, const float* g, float* m,
                       float* v, int t, double lr, double b1, double b2, double eps,
                       hipStream_t st);

hipError_t launch_sample_model16(const M16Args& m, const int32_t n[3], const double lo[3],
                                 const double hi[3], float* out_bn, float* out_c, hipStream_t st);

hipError_t launch_eval_fields(const FieldPack& fp, int64_t n, const float* xyz, float* out,
                              hipStream_t st);

hipError_t launch_forward_mlp(const GeomArgs& g, const FreqArgs& fa, const EmitArgs& ea,
                              const MlpArgs& m, float* maps, double* phi_end, hipStream_t st);
hipError_t launch_eval_mlp(const MlpArgs& m, int64_t n, const float* xyz, float* out,
                           hipStream_t st);

}  // namespace sm
