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
  // Kerr-Schild tables on the device (curved geometry; NULL when flat)
  bool curved = false;
  int ks_ninc = 0, ks_zin_stride = 0, ks_cw = 64;
  bool ks_lco = true;  // angular kernel: coefficient rows staged in LDS
  void* d_rec_r = nullptr;       // [ns][(N1+1) N2][4] transport type
  void* d_rec_t = nullptr;       // [ns][N1 (N2+1)][4]
  void* d_rec_p = nullptr;       // [ns][N1 N2][4]
  unsigned char* d_zin = nullptr;
  void* d_acoef = nullptr;       // [N1 N2][ns][KS_ROW] angular coefficients, transport type
  double* d_nu0 = nullptr;       // [N1 N2]
  double* d_e = nullptr;         // [N1 N2][16] e^mu_a
  double* d_einv = nullptr;      // [N1 N2][16] e^a_mu
  int* d_inc = nullptr;          // [ns][KS_ROW] the direction, then its neighbours (padded)
  // patches of directions for the angular kernel with many directions
  int ks_npatch = 0;
  int* d_plist = nullptr;        // load lists, concatenated: the patch's directions, then its halo
  int* d_poff = nullptr;         // [npatch + 1] offsets into d_plist
  int* d_pnout = nullptr;        // [npatch] directions owned by the patch (the list's head)
  int* d_plnb = nullptr;         // [ns][KS_ROW] positions of a direction's row set in its patch's list
  void* d_angD = nullptr;        // [ns][nc] angular divergence scratch
  // MAPR edge states (angular_recon = RT_AREC_MAPR), transport type unless noted
  bool mapr = false;
  int* d_mp_ring = nullptr;      // [ns][KS_ROW] neighbour count, neighbours in cyclic order
  void* d_mp_minv = nullptr;     // [ns][KS_DEG][4] inverse of the pair's gnomonic coordinates
  void* d_mp_pq = nullptr;       // [ns][KS_ROW][4] per neighbour slot: the edge midpoint in the
                                 // direction's and in the neighbour's gnomonic coordinates
  void* d_mp_coef = nullptr;     // [N1 N2][ns][KS_ROW] edge flux coefficient per slot
  unsigned char* d_mp_self = nullptr;  // [N1 N2][ns] bit j: slot j's upwind side is the direction
  void* d_mp_grad = nullptr;     // [ns][2][nc] slope per direction and cell

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
  double* d_Tstar = nullptr;   // [nc]
  void* d_Itil = nullptr;      // [ns][nc] stage-1 output (I~ of the half step)
  double* d_mapA = nullptr;    // [3][nc] lazy interaction map of the state buffer
  double* d_mapB = nullptr;    // [3][nc] lazy interaction map of d_Itil
  // frequency bins (rt_set_groups; 0: gray).  With bins the intensity and the
  // per-stage scratch hold ng bin-major copies: d_Itil [ng][ns][nc], the lazy
  // maps [ng][2][nc] (alpha, beta per bin; at least 3 nc), d_Emg [ng][nc] the
  // per-bin E_- of the current stage
  int ng = 0;
  std::vector<double> nu_edges;  // [ng + 1]
  double* d_ka_g = nullptr;      // [ng][nc] kappa_a per bin
  double* d_Emg = nullptr;       // [ng][nc]
  double W0 = 0.0;             // sum of the weights
  double Wsum[10] = {0};       // sum_s w_s n^a n^b
  void* d_gA = nullptr;        // adjoint scratch [ns][nc] x 3
  void* d_gB = nullptr;
  void* d_gC = nullptr;
  void* d_gD = nullptr;
  double* d_gcell = nullptr;   // adjoint per-face tau gradients [groups][3][2][nc]
  double* d_gT = nullptr;      // adjoint: dL/dT* and a stage-2 temperature scratch [2][nc]
  unsigned long long* d_count = nullptr;  // [0] interaction failures, [1] non-finite
  // launch order of the stage kernel's tiles (bricks of tiles that run together),
  // cached per (tiles per axis, tile shape, resident workgroups)
  unsigned* d_tile_order = nullptr;
  long long tile_order_key = -1;
  int debug = 0;
  std::string noalloc_error;  // why the static scratch could not be resolved, if it could not
  // kernel timing (debug bit 1): events recorded around launches
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
};

namespace rt {

// angular coupling of the curved geometry: a direction of the geodesic grid
// has at most KS_DEG neighbours; its coefficient row holds KS_ROW entries
constexpr int KS_DEG = 6, KS_ROW = 8;
// rows (directions) one workgroup of the patched angular kernel stages: 40 KiB
// of 256-byte rows, plus the patch's coefficient rows (three workgroups per
// compute unit)
constexpr int KS_PATCH_LOADS = 160;
// LDS of the angular kernel for a run of cw cells: intensities and, when lco,
// the coefficient rows and 16-bit neighbour lists
inline size_t angular_lds_bytes(int ns, int cw, size_t elem, bool lco) {
  return (size_t)ns * cw * elem + (lco ? (size_t)ns * KS_ROW * (elem + 2) : 0);
}

void set_error(const std::string& msg);

// Device scratch of one rt_step call: the half-step intensity (stage-1
// output), the two lazy interaction maps, the half-step temperature and, in
// curved space, the angular flux divergence and the MAPR slopes.  rt_step takes
// them from the context's own allocations; the allocation-free entry point
// carves them from the library's static scratch array.
struct StepScratch {
  void* Itil;       // [ns][nc] transport type
  double* mapA;     // [3][nc]
  double* mapB;     // [3][nc]
  double* Tstar;    // [nc]
  void* angD;       // [ns][nc] transport type (curved only, else NULL)
  void* mp_grad;    // [ns][2][nc] transport type (MAPR only, else NULL)
  double* Emg;      // [ng][nc] per-bin E_- (frequency bins only, else NULL)
};
// bytes of a context's step scratch laid out as 256-byte aligned parts, and
// that layout carved from one base pointer
size_t step_scratch_bytes(const rt_ctx* c);
StepScratch carve_step_scratch(const rt_ctx* c, void* base);

// The allocation-free entry point's scratch (noalloc.hip): a file-scope static
// device array of kNoallocScratchBytes, one per device, held until the process
// ends.  noalloc_scratch_init resolves its device address once per device (the
// device must be current) and must run before noalloc_scratch_ptr returns it.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch_ptr(int device);
// n 64-bit words at p set to v, by a kernel (no memset node in a captured graph)
hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st);

// all launchers enqueue on `st` and return the launch status
hipError_t launch_fluid(rt_ctx* c, const double* u, hipStream_t st);
hipError_t launch_moments(rt_ctx* c, const void* I, double* R, double* J, hipStream_t st);
// R^(ab) (tetrad) -> R^(mu nu) = e^mu_a e^nu_b R^(ab) in place (curved geometry)
hipError_t launch_to_coord(rt_ctx* c, double* R, hipStream_t st);
hipError_t launch_nonfinite(rt_ctx* c, const void* I, const double* T, hipStream_t st);
// multi-group temperature solve and per-bin interaction maps of one stage
// (multigroup.hip): from the per-bin E_- in `Emg` [ng][nc], writes T_out and
// map [ng][2][nc] (alpha, beta per bin); Newton starts from T_guess (may alias
// T_start or T_out)
hipError_t launch_mg_solve(rt_ctx* c, double h, const double* Emg, const double* T_start,
                           const double* T_guess, double* T_out, double* map, hipStream_t st);
// direction groups of the transport adjoint (its per-face scratch holds
// groups x 6 nc doubles)
int adjoint_dir_groups(const rt_ctx* c);
// one reverse step; gT_np1 (may be NULL) and gT_n are used by the
// bremsstrahlung model only (gT_n is written, not accumulated)
hipError_t launch_adjoint_step(rt_ctx* c, const void* I_n, const double* T_n, double dt,
                               const void* gI_np1, const double* gT_np1, void* gI_n, double* gT_n,
                               double* g_ka, double* g_j, hipStream_t st);

}  // namespace rt
