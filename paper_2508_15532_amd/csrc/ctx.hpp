// Library context and the internal launch interface between the C ABI
// (api.cpp) and the HIP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "../../include/rt.h"
#include "grid.hpp"

struct rt_ctx {
  rt_grid_desc desc{};
  int device = 0;
  rt::GeodesicGrid grid;
  int ns = 0;
  int n[3] = {0, 0, 0};
  long long nc = 0;
  bool fp32 = false;
  size_t elem = 8;  // bytes per intensity element

  // metric / geometry (flat: identity tetrad)
  bool metric_set = false;
  int metric_kind = RT_FLAT;
  double dx[3] = {1, 1, 1};
  double dt_max = 0;

  // device grid tables
  double* d_dir = nullptr;    // [3][ns] n-hat components, component-major
  float* d_dir_f = nullptr;   // same in float (FP32 transport)
  double* d_w = nullptr;      // [ns] weights
  double* d_W16 = nullptr;    // [ns4][16] moment weights w n^a n^b, padded

  // fluid and opacity model (library-owned copies)
  bool opac_set = false;
  rt_opacity_desc opac{};
  bool moving = false;
  double* d_rho = nullptr;
  double* d_uhat = nullptr;   // [4][nc] tetrad-frame fluid 4-velocity
  double* d_v = nullptr;      // [3][nc] coordinate 3-velocity u^a/u^0
  double* d_ka = nullptr;
  double* d_ks = nullptr;
  double* d_j = nullptr;

  // per-stage scratch
  double* d_abar_a = nullptr;  // [nc] fluid-frame absorption at T_coef
  double* d_abar_s = nullptr;  // [nc] scattering
  double* d_ahat = nullptr;    // [nc] u-hat^0 (abar_a + abar_s)
  double* d_Tstar = nullptr;   // [nc]
  void* d_face[3] = {nullptr, nullptr, nullptr};  // per axis [5][nfaces]
  long long nface[3] = {0, 0, 0};
  void* d_Itil = nullptr;      // [ns][nc] transported, pre-interaction intensity
  void* d_Istar = nullptr;     // [ns][nc] half-step intensity
  void* d_gA = nullptr;        // adjoint scratch [ns][nc] x 3
  void* d_gB = nullptr;
  void* d_gC = nullptr;
  double* d_gcell = nullptr;   // adjoint per-cell scratch [4][nc]
  unsigned long long* d_count = nullptr;  // [0] interaction failures, [1] non-finite
  int debug = 0;
  // kernel timing (debug bit 1): events recorded around launches
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
};

namespace rt {

void set_error(const std::string& msg);

// all launchers enqueue on `st` and return the launch status
hipError_t launch_fluid(rt_ctx* c, const double* u, hipStream_t st);
hipError_t launch_opacity(rt_ctx* c, const double* T_coef, hipStream_t st);
hipError_t launch_faces(rt_ctx* c, double dt, hipStream_t st);
hipError_t launch_transport(rt_ctx* c, const void* I_flux, const void* I_base, void* I_out,
                            double h, hipStream_t st);
hipError_t launch_source(rt_ctx* c, const void* I_til, void* I_out, const double* T_start,
                         const double* T_coef, double* T_out, double h, double* G,
                         hipStream_t st);
hipError_t launch_moments(rt_ctx* c, const void* I, double* R, double* J, hipStream_t st);
hipError_t launch_nonfinite(rt_ctx* c, const void* I, const double* T, hipStream_t st);
hipError_t launch_adjoint_step(rt_ctx* c, const void* I_n, double dt, const void* gI_np1,
                               void* gI_n, double* g_ka, double* g_j, hipStream_t st);

}  // namespace rt
