// Fused stage kernel of the flat-metric step: per-face flux coefficients,
// PLI transport of every direction, and the per-cell sums and implicit
// temperature solve of the interaction, in one pass over the intensities.
//
// Work decomposition.  A workgroup owns a tile of 64 (i3) x TY (i2) x TZ (i1)
// cells and loops over all directions.  Thread (tx, ty) owns the column of TZ
// cells at (i2 = y0 + ty, i3 = x0 + tx).  For each direction the tile and a
// two-cell halo (the PLI stencil) are staged in LDS; the i1 faces of a column
// are computed once per face (column march), the i2 and i3 faces from LDS.
//
// Lazy interaction.  At rest the implicit update of a cell is affine in the
// transported intensity, I_out = alpha I~ + beta for every direction, with
// alpha = 1/(1 + abar h) and beta = h Q / (4 pi (1 + abar h)) (see the
// interaction section below).  The stage therefore writes I~ and the per-cell
// pair (alpha, beta); whoever reads the intensity next (the next stage's
// stencil, the base term of stage 2, the final materialisation) applies the
// pair on load.  Each stage thus reads and writes every intensity once.  With
// a moving fluid the update is not affine in a direction-independent way and a
// separate materialisation pass follows each stage.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "ctx.hpp"
#include "stage.hpp"

namespace rt {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int TX = 64;

__device__ __forceinline__ int wrap_clamp(int i, int n, bool periodic) {
  if (periodic) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <typename T>
__device__ __forceinline__ T lim_slope(T p, T q, int limiter) {
  if (!(p * q > T(0))) return T(0);
  T ap = fabs(p), aq = fabs(q);
  T m = limiter == RT_LIM_MC ? fmin(fmin(T(2) * ap, T(2) * aq), T(0.5) * fabs(p + q)) : fmin(ap, aq);
  return p > T(0) ? m : -m;
}

// minmod(a, b) = median(a, b, 0): zero for opposite signs, else the argument
// closer to zero.  MC(p, q) = minmod(2p, 2q, (p+q)/2) = med(2 med(p, q, 0), (p+q)/2, 0).
__device__ __forceinline__ float med0(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double med0(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}
// half of the limited slope (the factor 2 is folded into the flux coefficients)
template <int LIM, typename T>
__device__ __forceinline__ T half_slope(T p, T q) {
  if (LIM == RT_LIM_MC) return med0(med0(p, q), T(0.25) * (p + q));
  return T(0.5) * med0(p, q);
}

// fluid-frame opacities of one cell at temperature T (Sec. 3.6.2)
__device__ __forceinline__ void opac(const StageArgs& a, const double* __restrict__ rho,
                                     const double* __restrict__ T, const double* __restrict__ ka,
                                     const double* __restrict__ ks, long long c, double& aa,
                                     double& as) {
  double r = rho[c];
  if (a.model == RT_OPAC_BREMS) {
    aa = a.C_a * r * r * pow(T[c], -3.5);
    as = a.C_s * r;
  } else {
    aa = ka ? r * ka[c] : 0.0;
    as = ks ? r * ks[c] : 0.0;
  }
  if (!(r >= a.rho_floor)) aa = as = 0.0;
}

// Face coefficients for F = nu (P IcL + Q IcR + U dL - V dR) (nu > 0) and
// F = nu (Q IcL + P IcR + V dL - U dR) (nu < 0): the modified signal-speed flux
// of Sec. 3.5 written in the cell-centre values and PLI slopes either side of
// the face, with E = exp(-tau), Wu = f2/(f2+f4), Wd = f4/(f2+f4),
// Dc = f2 f4/(f2+f4): P = E Wu + Dc, Q = E Wd - Dc, U = E Wu/2, V = E Wd/2.
// With a moving fluid the advection term (1-E)(max(vL,0) I_L + min(vR,0) I_R)
// adds aL = (1-E) max(vL,0), aR = (1-E) min(vR,0).
template <typename F>
struct FaceC {
  F P, Q, U, V;
};

__device__ __forceinline__ void face_coefs(double tau, double& P, double& Q, double& U, double& V,
                                           double& E) {
  E = exp(-tau);
  double fa, fb;
  if (tau < 1e-4) {
    double t2 = tau * tau;
    fa = 1.0 - 0.25 * t2;
    fb = tau * (1.0 - 0.25 * t2 * t2);
  } else {
    double t2 = tau * tau;
    fa = sqrt(-expm1(-t2)) / tau;
    fb = sqrt(-expm1(-t2 * t2)) / tau;
  }
  double Wu = fa / (fa + fb), Wd = fb / (fa + fb), Dc = fa * fb / (fa + fb);
  P = E * Wu + Dc;
  Q = E * Wd - Dc;
  U = 0.5 * E * Wu;
  V = 0.5 * E * Wd;
}

// Positive root machinery of the temperature equations (Sec. 3.6.2).
struct Solve {
  double T, Q;  // T_+, and Q = S_+ + alpha^s E_+
  bool ok;
};

__device__ Solve solve_cell(const StageArgs& a, double r, double T0, double aa, double as,
                            double Em, double A1, double A2, double jc) {
  const double Y = r / (a.gamma - 1.0);
  const double q = 1.0 - A2 * as;
  const double K = A1 - Y * q * T0 - q * Em;
  Solve o{T0, 0.0, true};
  if (a.model == RT_OPAC_FIXED_EMISSIVITY) {
    double Sp = 4.0 * kPi * jc;
    double Ep = (A1 + A2 * Sp) / q;
    o.Q = Sp + as * Ep;
    return o;
  }
  if (!((K < 0.0) && (q > 0.0))) {
    o.ok = false;
    return o;
  }
  const double b = Y * q;
  double Tp, Sp;
  if (a.model == RT_OPAC_BREMS) {
    // Method 2: A2 N sqrt(T) + Y q T + K = 0 is a quadratic in y = sqrt(T)
    const double N = a.C_a * r * r;
    const double B = A2 * N;
    const double y = -2.0 * K / (B + sqrt(B * B - 4.0 * b * K));
    Tp = y * y;
    Sp = N * y;
  } else {
    // Method 1: A2 alpha^a T^4 + Y q T + K = 0, Newton from above the root
    const double A = A2 * aa;
    double T = -K / b;
    if (A > 0.0) T = fmin(T, sqrt(sqrt(-K / A)));
    bool conv = false;
    for (int it = 0; it < a.max_iter; ++it) {
      double T3 = T * T * T;
      double dT = (A * T3 * T + b * T + K) / (4.0 * A * T3 + b);
      T -= dT;
      if (fabs(dT) <= a.rtol * fabs(T)) {
        conv = true;
        break;
      }
    }
    if (!conv) {
      o.ok = false;
      return o;
    }
    Tp = T;
    Sp = aa * T * T * T * T;
  }
  const double Ep = Em - Y * (Tp - T0);
  o.T = Tp;
  o.Q = Sp + as * Ep;
  return o;
}

}  // namespace

// ---------------------------------------------------------------------------
// the fused stage kernel
//
// Per direction s, with two LDS buffers alternating between directions:
//   1. stage the tile's region (cells plus a two-cell cross halo) of the flux
//      intensity, with its lazy map applied and zero-incoming ghosts zeroed;
//   2. compute every face flux of the tile once (face-parallel thread mapping:
//      faces along i3, i2 and i1 are flattened and dealt round-robin to the
//      workgroup's threads) into LDS;
//   3. each thread forms the divergence of its own cells, writes I~ and adds
//      the cell's interaction sums (FP64).
// After the last direction each thread solves the temperature equation of its
// cells and writes the cell's lazy interaction map.
// ---------------------------------------------------------------------------
template <typename S, typename F, int TY, int TZ, bool STAGE2, bool MOVING, int LIM, bool CURVED>
__global__ void __launch_bounds__(TX* TY)
k_stage(StageArgs a, StagePtrs p) {
  constexpr int NT = TX * TY;
  constexpr int RX = TX + 4, RY = TY + 4, RZ = TZ + 4;
  constexpr int NREG = RX * RY * RZ;
  constexpr int NJ = (NREG + NT - 1) / NT;
  // faces of the tile along i3 (x), i2 (y), i1 (z)
  constexpr int NFX = TZ * TY * (TX + 1), NFY = TZ * (TY + 1) * TX, NFZ = (TZ + 1) * TY * TX;
  constexpr int JX = (NFX + NT - 1) / NT, JY = (NFY + NT - 1) / NT, JZ = (NFZ + NT - 1) / NT;
  // every staging slot and every face slot owns an LDS word, so the loops below
  // run without per-slot branches (slots outside the region / face set write
  // words nobody reads)
  constexpr int OFY = JX * NT, OFZ = (JX + JY) * NT;
  __shared__ F reg[2][NJ * NT];
  __shared__ F flx[2][(JX + JY + JZ) * NT];
  // curved geometry: per-direction face records of the tile, {gP, gN, gA, x},
  // for the x1 faces ((TZ+1) x TY), theta faces (TZ x (TY+1)) and phi rows /
  // centres (TZ x TY), staged like the intensity region
  constexpr int NRR = (TZ + 1) * TY, NRT = TZ * (TY + 1), NRP = TZ * TY;
  constexpr int NREC = NRR + NRT + NRP;
  static_assert(!CURVED || NREC * 4 <= NT, "one record word per thread");
  __shared__ F grec[CURVED ? 2 : 1][CURVED ? NREC * 4 : 1];

  // ---- tile of this workgroup (XCD-aware: each XCD gets a contiguous range)
  const int b = blockIdx.x;
  const int tile = (b % 8) * a.tiles_per_xcd + b / 8;
  if (tile >= a.ntiles) return;
  const int bx = tile % a.tiles_x;
  const int by = (tile / a.tiles_x) % a.tiles_y;
  const int bz = tile / (a.tiles_x * a.tiles_y);
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
  const int t = threadIdx.x, tx = t % TX, ty = t / TX;
  const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
  const long long nc = a.nc;
  const S* __restrict__ Iflux = (const S*)p.Iflux_v;
  const S* Ibase = (const S*)p.Ibase_v;  // may alias Iout (same cell, earlier direction)
  S* Iout = (S*)p.Iout_v;
  const F* __restrict__ dirF = (const F*)p.dirF_v;
  const bool per0 = a.bc_lo[0] == RT_BC_PERIODIC, per1 = a.bc_lo[1] == RT_BC_PERIODIC,
             per2 = a.bc_lo[2] == RT_BC_PERIODIC;
  auto gcell = [&](int z, int y, int x) -> long long {
    return ((long long)wrap_clamp(z, n1, per0) * n2 + wrap_clamp(y, n2, per1)) * n3 +
           wrap_clamp(x, n3, per2);
  };

  // ---- region elements this thread stages every direction
  int gidx[NJ];      // global cell (after wrap / clamp); a valid cell for unused slots
  F mA[NJ], mB[NJ];  // lazy interaction map of the staged cell (identity if none)
  // zero-incoming sides the slot lies outside of (6 bits per slot, packed)
  static_assert(NJ * 6 <= 96, "slot flags");
  unsigned zf[(NJ * 6 + 31) / 32];
#pragma unroll
  for (int q = 0; q < (NJ * 6 + 31) / 32; ++q) zf[q] = 0;
  // curved: offset of the slot's boundary face in the incoming flags (-1: none)
  int zoff[CURVED ? NJ : 1];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = t + j * NT;
    int gi = -1;
    F ma = F(1), mb = F(0);
    if (CURVED) zoff[j] = -1;
    if (k < NREG) {
      const int rx = k % RX, ry = (k / RX) % RY, rz = k / (RX * RY);
      const bool hz = rz < 2 || rz >= TZ + 2, hy = ry < 2 || ry >= TY + 2, hx = rx < 2 || rx >= TX + 2;
      if ((int)hz + (int)hy + (int)hx <= 1) {
        const int gz = z0 - 2 + rz, gy = y0 - 2 + ry, gx = x0 - 2 + rx;
        unsigned f = 0;
        if (gz < 0 && a.bc_lo[0] == RT_BC_ZERO_INCOMING) f |= 1u;
        if (gz >= n1 && a.bc_hi[0] == RT_BC_ZERO_INCOMING) f |= 2u;
        if (gy < 0 && a.bc_lo[1] == RT_BC_ZERO_INCOMING) f |= 4u;
        if (gy >= n2 && a.bc_hi[1] == RT_BC_ZERO_INCOMING) f |= 8u;
        if (gx < 0 && a.bc_lo[2] == RT_BC_ZERO_INCOMING) f |= 16u;
        if (gx >= n3 && a.bc_hi[2] == RT_BC_ZERO_INCOMING) f |= 32u;
        if (CURVED) {
          // flags of the boundary face of the slot's line; slots outside two
          // sides at once (tile overhang corners) feed no valid cell and keep -1
          const int b2 = 2 * n2, b1 = 2 * n2 + n1, bp = 2 * n2 + 2 * n1, np = n1 * n2;
          const bool iz = gz >= 0 && gz < n1, iy = gy >= 0 && gy < n2, ix = gx >= 0 && gx < n3;
          zoff[j] = ((f & 1u) && iy && ix) ? gy
                  : ((f & 2u) && iy && ix) ? n2 + gy
                  : ((f & 4u) && iz && ix) ? b2 + gz
                  : ((f & 8u) && iz && ix) ? b1 + gz
                  : ((f & 16u) && iz && iy) ? bp + gz * n2 + gy
                  : ((f & 32u) && iz && iy) ? bp + np + gz * n2 + gy : -1;
        } else {
          zf[(j * 6) / 32] |= f << ((j * 6) % 32);
          if ((j * 6) % 32 > 26) zf[(j * 6) / 32 + 1] |= f >> (32 - (j * 6) % 32);
        }
        gi = (int)gcell(gz, gy, gx);
        if (p.mapF) {
          ma = (F)p.mapF[gi];
          mb = (F)p.mapF[nc + gi];
        }
      }
    }
    gidx[j] = gi >= 0 ? gi : (int)gcell(z0, y0, x0);
    mA[j] = ma;
    mB[j] = mb;
  }
  bool anyzf = false;
#pragma unroll
  for (int q = 0; q < (NJ * 6 + 31) / 32; ++q) anyzf |= zf[q] != 0u;
  if (CURVED) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) anyzf |= zoff[j] >= 0;
  }
  auto slot_flags = [&](int j) -> unsigned {
    const int bit = j * 6, w = bit / 32, o = bit % 32;
    unsigned v = zf[w] >> o;
    if (o > 26) v |= zf[w + 1] << (32 - o);
    return v & 63u;
  };

  // ---- own cells
  long long own[TZ];
  bool valid[TZ];
  const int gx = x0 + tx, gy = y0 + ty;
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    const int gz = z0 + k;
    valid[k] = gx < n3 && gy < n2 && gz < n1;
    own[k] = valid[k] ? ((long long)gz * n2 + gy) * n3 + gx : 0;
  }

  // ---- coefficients of the faces this thread computes (direction independent)
  auto ahat_of = [&](long long c) -> double {
    double aa, as;
    opac(a, p.rho, p.Tcoef, p.ka, p.ks, c, aa, as);
    return (MOVING ? p.uhat[c] : 1.0) * (aa + as);
  };
  auto vel_of = [&](int axis, int z, int y, int x) -> double { return p.vel[axis * nc + gcell(z, y, x)]; };
  constexpr int JF = JX + JY + JZ;
  FaceC<F> fc[JF];
  F adL[MOVING ? JF : 1], adR[MOVING ? JF : 1];
  // face slot q -> (axis, tile-relative z, y, x of the cell on the upper side of the face)
  auto face_of = [&](int q, int& axis, int& fz, int& fy, int& fx) -> bool {
    int i;
    if (q < JX) {
      axis = 2;
      i = t + q * NT;
      if (i >= NFX) return false;
      fx = i % (TX + 1);
      fy = (i / (TX + 1)) % TY;
      fz = i / ((TX + 1) * TY);
    } else if (q < JX + JY) {
      axis = 1;
      i = t + (q - JX) * NT;
      if (i >= NFY) return false;
      fx = i % TX;
      fy = (i / TX) % (TY + 1);
      fz = i / (TX * (TY + 1));
    } else {
      axis = 0;
      i = t + (q - JX - JY) * NT;
      if (i >= NFZ) return false;
      fx = i % TX;
      fy = (i / TX) % TY;
      fz = i / (TX * TY);
    }
    return true;
  };
  int fr0[JF];  // region index of the cell on the upper side of each face slot (-1: none)
  int frec[CURVED ? JF : 1];  // curved: record of each face slot
#pragma unroll
  for (int q = 0; q < JF; ++q) {
    int axis, fz, fy, fx;
    fc[q] = FaceC<F>{F(0), F(0), F(0), F(0)};
    if (MOVING) adL[q] = adR[q] = F(0);
    fr0[q] = ((2 + 0) * RY + 2) * RX + 2;  // any interior word for unused slots
    if (CURVED) frec[q] = 0;
    if (!face_of(q, axis, fz, fy, fx)) continue;
    fr0[q] = ((fz + 2) * RY + fy + 2) * RX + fx + 2;
    if (CURVED)
      frec[q] = axis == 0 ? fz * TY + fy : (axis == 1 ? NRR + fz * (TY + 1) + fy : NRR + NRT + fz * TY + fy);
    const int z = z0 + fz, y = y0 + fy, x = x0 + fx;
    const int dz = axis == 0, dy = axis == 1, dx = axis == 2;
    const double tau =
        a.abar * 0.5 * (ahat_of(gcell(z - dz, y - dy, x - dx)) + ahat_of(gcell(z, y, x))) * a.dt;
    double P, Q, U, V, E;
    face_coefs(tau, P, Q, U, V, E);
    fc[q] = FaceC<F>{(F)P, (F)Q, (F)(2.0 * U), (F)(2.0 * V)};
    if (MOVING) {
      // PLI of the coordinate velocity either side of the face
      const double vm2 = vel_of(axis, z - 2 * dz, y - 2 * dy, x - 2 * dx);
      const double vm1 = vel_of(axis, z - dz, y - dy, x - dx);
      const double v0 = vel_of(axis, z, y, x);
      const double vp1 = vel_of(axis, z + dz, y + dy, x + dx);
      const double vL = vm1 + 0.5 * lim_slope(vm1 - vm2, v0 - vm1, a.limiter);
      const double vR = v0 - 0.5 * lim_slope(v0 - vm1, vp1 - v0, a.limiter);
      adL[q] = (F)((1.0 - E) * fmax(vL, 0.0));
      adR[q] = (F)((1.0 - E) * fmin(vR, 0.0));
    }
  }

  // ---- curved: the record word this thread stages every direction
  const F* gsrc = nullptr;
  long long gstride = 0;
  if (CURVED && t < NREC * 4) {
    const int rec = t >> 2, comp = t & 3;
    if (rec < NRR) {
      const int i1 = z0 + rec / TY, i2 = y0 + rec % TY;
      if (i1 <= n1 && i2 < n2) {
        gsrc = (const F*)p.rec_r_v + ((long long)i1 * n2 + i2) * 4 + comp;
        gstride = (long long)(n1 + 1) * n2 * 4;
      }
    } else if (rec < NRR + NRT) {
      const int r2 = rec - NRR, i1 = z0 + r2 / (TY + 1), i2 = y0 + r2 % (TY + 1);
      if (i1 < n1 && i2 <= n2) {
        gsrc = (const F*)p.rec_t_v + ((long long)i1 * (n2 + 1) + i2) * 4 + comp;
        gstride = (long long)n1 * (n2 + 1) * 4;
      }
    } else {
      const int r3 = rec - NRR - NRT, i1 = z0 + r3 / TY, i2 = y0 + r3 % TY;
      if (i1 < n1 && i2 < n2) {
        gsrc = (const F*)p.rec_p_v + ((long long)i1 * n2 + i2) * 4 + comp;
        gstride = (long long)n1 * n2 * 4;
      }
    }
  }

  // ---- own-cell data used in the direction loop
  F bA[TZ], bB[TZ];                        // lazy map of the stage-2 base intensity
  double u0[TZ], u1[TZ], u2[TZ], u3[TZ];   // moving fluid: tetrad-frame 4-velocity
  double abh[TZ];                          // moving fluid: (alpha^a + alpha^s) h
  double nu0k[TZ];                         // n^0 = 1/lapse (1 when flat)
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    const long long c = own[k];
    bA[k] = F(1);
    bB[k] = F(0);
    if (STAGE2 && p.mapB) {
      bA[k] = (F)p.mapB[c];
      bB[k] = (F)p.mapB[nc + c];
    }
    if (MOVING) {
      u0[k] = p.uhat[c];
      u1[k] = p.uhat[nc + c];
      u2[k] = p.uhat[2 * nc + c];
      u3[k] = p.uhat[3 * nc + c];
      double x1, x2;
      opac(a, p.rho, p.Tcoef, p.ka, p.ks, c, x1, x2);
      abh[k] = (x1 + x2) * a.h;
    }
    nu0k[k] = CURVED ? p.nu0[c / n3] : 1.0;
  }

  // accumulators: at rest E_- = sum w I~; moving E_-, A1, A2
  constexpr int NACC = MOVING ? 3 : 1;
  double acc[TZ][NACC];
#pragma unroll
  for (int k = 0; k < TZ; ++k)
#pragma unroll
    for (int m = 0; m < NACC; ++m) acc[k][m] = 0.0;

  const F h = (F)a.h;
  const F idx0 = (F)a.inv_dx[0], idx1 = (F)a.inv_dx[1], idx2 = (F)a.inv_dx[2];
  const int ns = a.ns;

  // prefetch of direction 0
  S pre[NJ];
  S prb[TZ];
  S pda[CURVED ? TZ : 1];  // curved: angular divergence of the own cells
  F gpre = F(0);
  const S* angD = (const S*)p.angD_v;
#pragma unroll
  for (int j = 0; j < NJ; ++j) pre[j] = Iflux[gidx[j]];
  if (CURVED) {
    if (gsrc) gpre = gsrc[0];
#pragma unroll
    for (int k = 0; k < TZ; ++k) pda[k] = angD[own[k]];
  }
  if (STAGE2) {
#pragma unroll
    for (int k = 0; k < TZ; ++k) prb[k] = Ibase[own[k]];
  }

  for (int s = 0; s < ns; ++s) {
    const int buf = s & 1;
    F* R = reg[buf];
    F* FL = flx[buf];
    // direction components along i1 (z of the tile), i2 (y), i3 (x)
    const F nz = dirF[s], ny = dirF[ns + s], nx = dirF[2 * ns + s];
    // zero-incoming: which outside sides receive zero for this direction
    const unsigned inc = (nz > F(0) ? 1u : 0u) | (nz < F(0) ? 2u : 0u) | (ny > F(0) ? 4u : 0u) |
                         (ny < F(0) ? 8u : 0u) | (nx > F(0) ? 16u : 0u) | (nx < F(0) ? 32u : 0u);
    // 1. stage the region (lazy map applied)
    if (CURVED && anyzf) {
      const unsigned char* zs = p.zin + (long long)s * a.zin_stride;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        R[t + j * NT] = (zoff[j] >= 0 && zs[zoff[j]]) ? F(0) : mA[j] * (F)pre[j] + mB[j];
    } else if (anyzf) {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        R[t + j * NT] = (slot_flags(j) & inc) ? F(0) : mA[j] * (F)pre[j] + mB[j];
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) R[t + j * NT] = mA[j] * (F)pre[j] + mB[j];
    }
    F base[TZ];
    if (STAGE2) {
#pragma unroll
      for (int k = 0; k < TZ; ++k) base[k] = bA[k] * (F)prb[k] + bB[k];
    }
    F dang[CURVED ? TZ : 1];
    F* GR = grec[CURVED ? buf : 0];
    if (CURVED) {
      if (t < NREC * 4) GR[t] = gpre;
#pragma unroll
      for (int k = 0; k < TZ; ++k) dang[k] = (F)pda[k];
    }
    __syncthreads();
    // prefetch the next direction while this one is computed
    if (s + 1 < ns) {
      const S* Is = Iflux + (long long)(s + 1) * nc;
#pragma unroll
      for (int j = 0; j < NJ; ++j) pre[j] = Is[gidx[j]];
      if (STAGE2) {
        const S* Ib = Ibase + (long long)(s + 1) * nc;
#pragma unroll
        for (int k = 0; k < TZ; ++k) prb[k] = Ib[own[k]];
      }
      if (CURVED) {
        if (gsrc) gpre = gsrc[(long long)(s + 1) * gstride];
        const S* As = angD + (long long)(s + 1) * nc;
#pragma unroll
        for (int k = 0; k < TZ; ++k) pda[k] = As[own[k]];
      }
    }
    // 2. face fluxes, each face once; the sign of the direction component is
    // uniform over an axis, so each axis takes one branch per direction
    auto faces = [&](auto axis_tag, F nu) {
      constexpr int AX = decltype(axis_tag)::value;
      constexpr int Q0 = AX == 2 ? 0 : (AX == 1 ? JX : JX + JY);
      constexpr int QN = AX == 2 ? JX : (AX == 1 ? JY : JZ);
      constexpr int ST = AX == 2 ? 1 : (AX == 1 ? RX : RX * RY);
      // F = nu (P I_l + Q I_l+1 + U dL - V dR) for nu > 0, the mirror image for
      // nu < 0; hL, hR are half slopes, so U2 = 2U and V2 = 2V multiply them
      auto one = [&](int q, bool pos) {
        const F* Rq = R + fr0[q];
        const F vm2 = Rq[-2 * ST], vm1 = Rq[-ST], v0 = Rq[0], vp1 = Rq[ST];
        const F d0 = vm1 - vm2, d1 = v0 - vm1, d2 = vp1 - v0;
        const F hL = half_slope<LIM>(d0, d1), hR = half_slope<LIM>(d1, d2);
        const FaceC<F>& c = fc[q];
        F fl = pos ? nu * (c.P * vm1 + c.Q * v0 + c.U * hL - c.V * hR)
                   : nu * (c.Q * vm1 + c.P * v0 + c.V * hL - c.U * hR);
        if (MOVING) fl += adL[q] * (vm1 + hL) + adR[q] * (v0 - hR);
        FL[t + q * NT] = fl;
      };
      if (__builtin_amdgcn_readfirstlane(__float_as_int((float)nu)) > 0) {
#pragma unroll
        for (int qq = 0; qq < QN; ++qq) one(Q0 + qq, true);
      } else {
#pragma unroll
        for (int qq = 0; qq < QN; ++qq) one(Q0 + qq, false);
      }
    };
    if (CURVED) {
      // direction components vary with position: both upwind forms, weighted
      // by the face records (one of gP, gN is zero)
#pragma unroll
      for (int q = 0; q < JF; ++q) {
        const int ST = q < JX ? 1 : (q < JX + JY ? RX : RX * RY);
        const F* Rq = R + fr0[q];
        const F vm2 = Rq[-2 * ST], vm1 = Rq[-ST], v0 = Rq[0], vp1 = Rq[ST];
        const F d0 = vm1 - vm2, d1 = v0 - vm1, d2 = vp1 - v0;
        const F hL = half_slope<LIM>(d0, d1), hR = half_slope<LIM>(d1, d2);
        const F* g = GR + frec[q] * 4;
        const FaceC<F>& c = fc[q];
        F fl = g[0] * (c.P * vm1 + c.Q * v0 + c.U * hL - c.V * hR) +
               g[1] * (c.Q * vm1 + c.P * v0 + c.V * hL - c.U * hR);
        if (MOVING) fl += g[2] * (adL[q] * (vm1 + hL) + adR[q] * (v0 - hR));
        FL[t + q * NT] = fl;
      }
    } else {
      faces(std::integral_constant<int, 2>{}, nx);
      faces(std::integral_constant<int, 1>{}, ny);
      faces(std::integral_constant<int, 0>{}, nz);
    }
    __syncthreads();
    // 3. divergence, update, interaction sums
    const double ws = p.w[s];
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
      const F fxl = FL[(k * TY + ty) * (TX + 1) + tx], fxh = FL[(k * TY + ty) * (TX + 1) + tx + 1];
      const F fyl = FL[OFY + (k * (TY + 1) + ty) * TX + tx];
      const F fyh = FL[OFY + (k * (TY + 1) + ty + 1) * TX + tx];
      const F fzl = FL[OFZ + (k * TY + ty) * TX + tx];
      const F fzh = FL[OFZ + ((k + 1) * TY + ty) * TX + tx];
      const F bse = STAGE2 ? base[k] : R[((k + 2) * RY + ty + 2) * RX + tx + 2];
      F It;
      if (CURVED) {
        // X = n^0 n_0 I updated by the area-weighted face fluxes; x = 1/(dV n^0 n_0),
        // zero where |n_0| is below the cut (I~ = 0 there)
        const F x = GR[(NRR + NRT + k * TY + ty) * 4 + 3];
        const F sum = (fzh - fzl) + (fyh - fyl) + (fxh - fxl);
        It = (x != F(0) ? bse : F(0)) - h * (x * sum + dang[k]);
      } else {
        const F div = (fzh - fzl) * idx0 + (fyh - fyl) * idx1 + (fxh - fxl) * idx2;
        It = bse - h * div;
      }
      if (valid[k]) Iout[(long long)s * nc + own[k]] = (S)It;
      // ---- interaction sums (FP64)
      const double Itd = (double)(S)It;
      if (MOVING) {
        const double nb = u0[k] - (u1[k] * p.dirD[s] + u2[k] * p.dirD[ns + s] + u3[k] * p.dirD[2 * ns + s]);
        const double nb2 = nb * nb;
        const double Ib = Itd * nb2 * nb2, dOb = ws / nb2;
        const double den = nu0k[k] + nb * abh[k];
        acc[k][0] += Ib * dOb;
        acc[k][1] += nu0k[k] * Ib * dOb / den;
        acc[k][2] += nb * a.h / (4.0 * kPi * den) * dOb;
      } else {
        acc[k][0] += ws * Itd;
      }
    }
  }

  // ---- per-cell implicit temperature and the interaction map
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    if (!valid[k]) continue;
    const long long c = own[k];
    double aak, ask;
    opac(a, p.rho, p.Tcoef, p.ka, p.ks, c, aak, ask);
    const double ab = aak + ask, rrk = p.rho[c], T0k = p.Tstart[c];
    const bool live = rrk >= a.rho_floor;
    double Em, A1, A2;
    if (MOVING) {
      Em = acc[k][0];
      A1 = acc[k][1];
      A2 = acc[k][2];
    } else {
      const double cs = 1.0 / (1.0 + ab * a.h);
      Em = acc[k][0];
      A1 = cs * Em;
      A2 = a.h / (4.0 * kPi * (1.0 + ab * a.h)) * a.W0;
    }
    Solve so{T0k, 0.0, false};
    if (live) {
      so = solve_cell(a, rrk, T0k, aak, ask, Em, A1, A2, p.jv ? p.jv[c] : 0.0);
      if (!so.ok && p.fail) atomicAdd(p.fail, 1ull);
    }
    const bool use = live && so.ok;
    p.Tout[c] = use ? so.T : T0k;
    if (MOVING) {
      // parameters of the direction-dependent map, applied by the materialisation
      p.mapO[c] = use ? so.Q : 0.0;
      p.mapO[nc + c] = ab;
      // 1: apply the interaction, 0: keep I~, 2: zero (rows next to the axis)
      const int gyk = (int)((c / n3) % n2);
      const bool pole = CURVED && (gyk < a.pole_rows || gyk >= n2 - a.pole_rows);
      p.mapO[2 * nc + c] = pole ? 2.0 : (use ? 1.0 : 0.0);
    } else {
      const double al = use ? 1.0 / (1.0 + ab * a.h) : 1.0;
      const double be = use ? a.h * so.Q / (4.0 * kPi * (1.0 + ab * a.h)) : 0.0;
      p.mapO[c] = al;
      p.mapO[nc + c] = be;
    }
  }
}

// ---------------------------------------------------------------------------
// materialisation: apply the interaction map to a stored I~ in place
//   at rest:  I = alpha I~ + beta
//   moving:   I = (c_s I~ nbar^4 + d_s Q) / nbar^4 with c_s, d_s of the
//             implicit update (Eq. fluid_interaction_discrete), plus the moments
//             and the 4-force of the new intensity when requested.
// One thread per cell, directions looped (coalesced across cells).
// ---------------------------------------------------------------------------
template <typename S, bool MOVING>
__global__ void __launch_bounds__(256)
k_materialize(long long nc, int ns, double h, const double* __restrict__ map, S* __restrict__ I,
              const double* __restrict__ uhat, const double* __restrict__ dirD,
              const double* __restrict__ w, const double* __restrict__ W16,
              double* __restrict__ Rout, double* __restrict__ Gout,
              const double* __restrict__ nu0, int n3) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  if (!MOVING) {
    const double al = map[c], be = map[nc + c];
    if (!Rout && !Gout) {
      for (int s = 0; s < ns; ++s) {
        S* q = I + (long long)s * nc + c;
        *q = (S)(al * (double)*q + be);
      }
      return;
    }
    // moments of the stored new intensity; 4-force -(R^(0a)(out) - R^(0a)(I~)) / h
    double R[10];
    for (int m = 0; m < 10; ++m) R[m] = 0.0;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
      S* q = I + (long long)s * nc + c;
      const double It = (double)*q;
      const S o = (S)(al * It + be);
      *q = o;
      const double Iq = (double)o;
      const double* Ws = W16 + s * 16;
#pragma unroll
      for (int m = 0; m < 10; ++m) R[m] += Ws[m] * Iq;
#pragma unroll
      for (int m = 0; m < 4; ++m) g[m] += Ws[m] * (Iq - It);
    }
    if (Rout)
      for (int m = 0; m < 10; ++m) Rout[m * nc + c] = R[m];
    if (Gout)
      for (int m = 0; m < 4; ++m) Gout[m * nc + c] = -g[m] / h;
    return;
  }
  const double Q = map[c], ab = map[nc + c];
  const double code = map[2 * nc + c];  // 1: apply, 0: keep, 2: zero
  const bool use = code == 1.0, zero = code == 2.0;
  const double n0c = nu0 ? nu0[c / n3] : 1.0;
  const double u0 = uhat[c], u1 = uhat[nc + c], u2 = uhat[2 * nc + c], u3 = uhat[3 * nc + c];
  double R[10];
  for (int m = 0; m < 10; ++m) R[m] = 0.0;
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < ns; ++s) {
    S* q = I + (long long)s * nc + c;
    const double It = (double)*q;
    double Io = It;
    if (use) {
      double nb = u0 - (u1 * dirD[s] + u2 * dirD[ns + s] + u3 * dirD[2 * ns + s]);
      double nb2 = nb * nb, nb4 = nb2 * nb2;
      double den = n0c + nb * ab * h;
      double cs = n0c / den, ds = nb * h / (4.0 * kPi * den);
      Io = (cs * It * nb4 + ds * Q) / nb4;
      *q = (S)Io;
    } else if (zero) {
      Io = 0.0;
      *q = (S)0;
    }
    const double Iq = (double)(S)Io;
    if (Rout)
      for (int m = 0; m < 10; ++m) R[m] += W16[s * 16 + m] * Iq;
    if (Gout) {
      const double dI = w[s] * (Iq - It);
      g[0] += dI;
      g[1] += dI * dirD[s];
      g[2] += dI * dirD[ns + s];
      g[3] += dI * dirD[2 * ns + s];
    }
  }
  if (Rout)
    for (int m = 0; m < 10; ++m) Rout[m * nc + c] = R[m];
  if (Gout)
    for (int m = 0; m < 4; ++m) Gout[m * nc + c] = -g[m] / h;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
template <typename S, typename F, int TY, int TZ, int LIM>
hipError_t launch_tiled(rt_ctx* c, StageArgs a, const StagePtrs& p, bool stage2, hipStream_t st) {
  a.tiles_x = (c->n[2] + TX - 1) / TX;
  a.tiles_y = (c->n[1] + TY - 1) / TY;
  a.tiles_z = (c->n[0] + TZ - 1) / TZ;
  a.ntiles = a.tiles_x * a.tiles_y * a.tiles_z;
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  dim3 grid(8 * a.tiles_per_xcd), block(TX * TY);
  if (c->curved) {
    // curved geometry always runs the moving-fluid form (direction-dependent map)
    if (stage2)
      hipLaunchKernelGGL((k_stage<S, F, TY, TZ, true, true, LIM, true>), grid, block, 0, st, a, p);
    else
      hipLaunchKernelGGL((k_stage<S, F, TY, TZ, false, true, LIM, true>), grid, block, 0, st, a, p);
  } else if (c->moving) {
    if (stage2)
      hipLaunchKernelGGL((k_stage<S, F, TY, TZ, true, true, LIM, false>), grid, block, 0, st, a, p);
    else
      hipLaunchKernelGGL((k_stage<S, F, TY, TZ, false, true, LIM, false>), grid, block, 0, st, a, p);
  } else {
    if (stage2)
      hipLaunchKernelGGL((k_stage<S, F, TY, TZ, true, false, LIM, false>), grid, block, 0, st, a, p);
    else
      hipLaunchKernelGGL((k_stage<S, F, TY, TZ, false, false, LIM, false>), grid, block, 0, st, a, p);
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_stage(rt_ctx* c, const StageArgs& a, const StagePtrs& p, bool stage2,
                        hipStream_t st) {
  const bool mc = a.limiter == RT_LIM_MC;
  if (c->fp32)
    return mc ? launch_tiled<float, float, 4, 2, RT_LIM_MC>(c, a, p, stage2, st)
              : launch_tiled<float, float, 4, 2, RT_LIM_MINMOD>(c, a, p, stage2, st);
  return mc ? launch_tiled<double, double, 4, 1, RT_LIM_MC>(c, a, p, stage2, st)
            : launch_tiled<double, double, 4, 1, RT_LIM_MINMOD>(c, a, p, stage2, st);
}

hipError_t launch_materialize(rt_ctx* c, void* I, const double* map, double h, double* R,
                              double* G, hipStream_t st) {
  dim3 grid((unsigned)((c->nc + 255) / 256)), block(256);
  if (c->fp32) {
    if (c->moving)
      hipLaunchKernelGGL((k_materialize<float, true>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (float*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2]);
    else
      hipLaunchKernelGGL((k_materialize<float, false>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (float*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2]);
  } else {
    if (c->moving)
      hipLaunchKernelGGL((k_materialize<double, true>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (double*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2]);
    else
      hipLaunchKernelGGL((k_materialize<double, false>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (double*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2]);
  }
  return hipGetLastError();
}

}  // namespace rt
