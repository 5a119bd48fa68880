// Arguments of the fused stage kernel and the materialisation pass.
#pragma once
#include <hip/hip_runtime_api.h>

struct rt_ctx;

namespace rt {

struct StageArgs {
  int n1, n2, n3;
  long long nc;
  int ns;
  int bc_lo[3], bc_hi[3];
  double inv_dx[3];
  double h;     // length of this stage's transport and interaction step
  double dt;    // full step (enters tau)
  double abar;
  int limiter;
  int model;
  double gamma, C_a, C_s, rho_floor;
  int max_iter;
  double rtol;
  double W0;        // sum of the quadrature weights
  double Wsum[10];  // sum_s w_s n^a n^b (moments of a unit isotropic field)
  int tiles_x, tiles_y, tiles_z, ntiles, tiles_per_xcd;
  // curved (Kerr-Schild) geometry
  int curved;       // 0: flat Cartesian, 1: per-(r, theta) geometry tables
  int zin_stride;   // bytes per direction of the boundary incoming flags
  int pole_rows;    // theta rows next to each axis whose intensity is zeroed
};

struct StagePtrs {
  const void* Iflux_v;
  const double* mapF;   // lazy map (alpha, beta) of Iflux, [2][nc]; NULL = identity
  const void* Ibase_v;  // stage 2: intensity of the step start (centre only)
  const double* mapB;   // its lazy map; NULL = identity
  void* Iout_v;         // transported intensity I~ (may alias Ibase)
  double* mapO;         // out: (alpha, beta) at rest; (Q, abar, use) with a moving fluid
  const double* Tstart;
  const double* Tcoef;
  double* Tout;
  const double* rho;
  const double* ka;
  const double* ks;
  const double* jv;
  const double* uhat;
  const double* vel;
  const void* dirF_v;   // [3][ns] directions in the transport type
  const double* dirD;   // [3][ns] directions in double
  const double* w;      // [ns]
  const double* W16;    // [ns][16] moment weights
  unsigned long long* fail;
  // curved geometry (NULL when flat): face records {gP, gN, gA, x} in the
  // transport type, [ns][faces][4] for faces normal to x1, theta and phi
  // (the phi records carry the centre factor x), boundary incoming flags,
  // the angular flux divergence of Iflux already scaled to the update
  // (transport type, [ns][nc]) and n^0 = 1/lapse per (r, theta)
  const void* rec_r_v;
  const void* rec_t_v;
  const void* rec_p_v;
  const unsigned char* zin;
  const void* angD_v;
  const double* nu0;
  // tile launch order: code = tx | ty << 10 | tz << 21 per position in the
  // order (NULL: x fastest, then y, then z)
  const unsigned* tile_order;
  // at rest only: when set, the kernel writes each cell's E_- = sum_s w_s I~_s
  // here ([nc]) instead of solving the interaction (Tout and mapO untouched);
  // the multi-group solve then combines the bins
  double* sumE;
};

// may_alloc = false: the call allocates nothing (the tile launch order is taken
// from the context's cache when it matches, else tiles run in natural order)
hipError_t launch_stage(rt_ctx* c, const StageArgs& a, const StagePtrs& p, bool stage2,
                        hipStream_t st, bool may_alloc = true);
// acc: add the moments and the 4-force to R and G instead of overwriting them
// (the bins of a multi-group step; at rest only)
hipError_t launch_materialize(rt_ctx* c, void* I, const double* map, double h, double* R,
                              double* G, hipStream_t st, bool acc = false);
// angular flux divergence of I (curved geometry) into angD; MAPR keeps its
// per-direction slopes in grad ([ns][2][nc])
hipError_t launch_angular(rt_ctx* c, const void* I, void* angD, void* grad, hipStream_t st);

}  // namespace rt
