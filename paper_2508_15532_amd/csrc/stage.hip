// Fused stage kernel of the predictor-corrector step (flat and curved
// metrics): per-face flux coefficients, PLI transport of every direction, and
// the per-cell sums and implicit temperature solve of the interaction, in one
// pass over the intensities.
//
// Work decomposition: see the kernel below (64 x TY x TZ cell tiles, a column
// of TZ cells per thread, all directions looped inside the workgroup).
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

#include <limits>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

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

// 1/d for a positive normal d: the hardware reciprocal refined by two
// Newton-Raphson steps (r <- r + r (1 - d r)), each of which doubles the
// correct bits, to within an ulp of the quotient; cheaper than the IEEE
// division sequence, which also handles scaling and special values that a
// positive normal d does not need
__device__ __forceinline__ double rcp_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
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

// x > 0 and x < 0 for a value every lane holds (a direction component read
// by a scalar load), from its bits: scalar comparisons, no vector compare
template <typename T>
__device__ __forceinline__ bool upos(T x) {
  using B = typename std::conditional<sizeof(T) == 4, int, long long>::type;
  return __builtin_bit_cast(B, x) > 0;
}
template <typename T>
__device__ __forceinline__ bool uneg(T x) {
  using B = typename std::conditional<sizeof(T) == 4, int, long long>::type;
  const B b = __builtin_bit_cast(B, x);
  return b < 0 && b != std::numeric_limits<B>::min();  // negative, not -0
}

// a read-only device array in the constant address space (loads at uniform
// addresses become scalar loads)
template <typename T>
using CPtr = const __attribute__((address_space(4))) T*;

// One direction's plane of nc cells as a buffer resource: loads and stores
// take a uniform base and an unsigned 32-bit byte offset per lane, so the
// direction loop carries no 64-bit address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes) {
  // stride 0, raw dword addressing (the data-format word of the gfx9 family)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// a byte offset at or past the end of any plane (a plane holds fewer than
// 2^29 cells of at most 8 bytes): buffer stores there are dropped by the range check
constexpr unsigned kDropOffset = 0xFFFFFFF8u;
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "dword or dwordx2");
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// stores are marked non-temporal (cache policy bit 1 on this target): the
// kernel never reads back what it writes, so these lines go first when L2
// needs room and the staged planes of the neighbouring tiles stay resident
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 2);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, (int)off, 0, 2);
}

// fluid-frame opacities of one cell at temperature T (Sec. 3.6.2)
__device__ __forceinline__ void opac(const StageArgs& a, const double* __restrict__ rho,
                                     const double* __restrict__ T, const double* __restrict__ ka,
                                     const double* __restrict__ ks, long long c, double& aa,
                                     double& as) {
  double r = rho[c];
  if (a.model == RT_OPAC_BREMS || a.model == RT_OPAC_BREMS_M3) {
    const double t = T[c];
    aa = a.C_a * r * r / (t * t * t * sqrt(t)) * (ka ? ka[c] : 1.0);  // T^-3.5, per-cell factor
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
__device__ __forceinline__ void face_coefs(double tau, double& P, double& Q, double& U, double& V,
                                           double& E) {
  E = exp(-tau);
  // fa = ga / tau, fb = gb / tau: the weights are ratios of ga and gb
  double ga, gb, itau;
  const double t2 = tau * tau;
  if (tau < 1e-4) {
    ga = 1.0 - 0.25 * t2;
    gb = tau * (1.0 - 0.25 * t2 * t2);
    itau = 1.0;
  } else {
    ga = sqrt(-expm1(-t2));
    gb = sqrt(-expm1(-t2 * t2));
    itau = 1.0 / tau;
  }
  const double r = 1.0 / (ga + gb);
  double Wu = ga * r, Wd = gb * r, Dc = ga * gb * r * itau;
  P = E * Wu + Dc;
  Q = E * Wd - Dc;
  U = 0.5 * E * Wu;
  V = 0.5 * E * Wd;
}

// Positive root machinery of the temperature equations (Sec. 3.6.2).
struct Solve {
  double T, Q;  // T_+, and Q = S_+ + alpha^s E_+
  double r;     // alpha_- / alpha_+ (Method 3), else 1
  bool ok;
};

// Method 3 (the total opacity semi-implicit): T_+ is the root in (0, E0/Y) of
//   F(T) = (E0 - Y T)(N T^-3.5 + alpha^s (1 - alpha_- A2)) - alpha_- (A1 + A2 N sqrt T),
// the energy balance E_+ = E0 - Y T_+ with E_+ = r (A1 + A2 S_+),
// r = alpha_-/alpha_+, S_+ = N sqrt(T_+).  F decreases strictly and is convex on
// that interval, so Newton from either side of the root stays in the bracket
// or is replaced by bisection.
__device__ bool method3_root(double Y, double E0, double N, double as, double ab, double A1, double A2,
                             double T0, int max_iter, double rtol, double& T) {
  const double qs = as * (1.0 - ab * A2);
  if (!(E0 > 0.0) || !(Y > 0.0) || !(N > 0.0) || !(A1 >= 0.0) || !(1.0 - ab * A2 > 0.0)) return false;
  double lo = 0.0, hi = E0 / Y;
  double x = (T0 > 0.0 && T0 < hi) ? T0 : 0.5 * hi;
  for (int it = 0; it < max_iter; ++it) {
    const double sx = sqrt(x), ix = 1.0 / x;
    const double p35 = ix * ix * ix / sx;  // x^-3.5
    const double g = N * p35 + qs, e = E0 - Y * x;
    const double F = e * g - ab * (A1 + A2 * N * sx);
    const double dF = -Y * g - 3.5 * e * N * p35 * ix - 0.5 * ab * A2 * N / sx;
    if (F > 0.0) lo = x;
    else hi = x;
    const double step = F / dF;
    double xn = x - step;
    // converged: the Newton step is within the tolerance (tested before the
    // bracket guard, which would replace a step onto the bracket's end)
    if (fabs(step) <= rtol * x) {
      T = (xn >= lo && xn <= hi) ? xn : x;
      return true;
    }
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    x = xn;
    if (hi - lo <= rtol * x) {
      T = x;
      return true;
    }
  }
  return false;
}

// jc: the emissivity (fixed-emissivity model) or the per-cell factor of the
// bremsstrahlung opacity (1 when none is given)
__device__ Solve solve_cell(const StageArgs& a, double r, double T0, double aa, double as,
                            double Em, double A1, double A2, double jc) {
  const double Y = r / (a.gamma - 1.0);
  const double q = 1.0 - A2 * as;
  const double K = A1 - Y * q * T0 - q * Em;
  Solve o{T0, 0.0, 1.0, true};
  if (a.model == RT_OPAC_BREMS_M3) {
    const double N = a.C_a * r * r * jc, E0 = Em + Y * T0, ab = aa + as;
    double Tp = T0;
    // with the Newton cap of Methods 1-2, at least the bisection depth of FP64
    if (!method3_root(Y, E0, N, as, ab, A1, A2, T0, max(a.max_iter, 120), a.rtol, Tp)) {
      o.ok = false;
      return o;
    }
    const double st = sqrt(Tp);
    const double Ep = E0 - Y * Tp;
    o.T = Tp;
    o.Q = N * st + as * Ep;
    o.r = ab / (N / (Tp * Tp * Tp * st) + as);
    return o;
  }
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
    const double N = a.C_a * r * r * jc;
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
// Work decomposition.  A workgroup of 64 TY threads owns a tile of 64 (i3, x) x
// TY (i2, y) x TZ (i1, z) cells and loops over all directions (TY = 8 at rest,
// 4 with a moving fluid, whose threads hold more state).  Wave ty owns row
// y0 + ty, lane tx column x0 + tx, and each thread the TZ cells of its column
// along z.  For each direction:
//   1. the thread's column with a two-cell halo along z lives in registers
//      (the z stencil needs no data movement); the TZ planes of the tile with
//      a two-cell halo in x and y are staged in LDS (lazy map applied,
//      zero-incoming ghosts zeroed); the next direction's loads are issued;
//   2. every thread forms the half slopes of its cells and of their
//      neighbours and both faces of each cell along every axis, from the
//      planes (x, y) and its column (z), with no further exchange; the planes
//      (and the curved face records) alternate between two buffers, so one
//      barrier per direction suffices;
//   3. each thread forms the divergence of its cells, writes I~ and adds the
//      cell's FP64 interaction sums.
// After the last direction each thread solves the temperature equation of its
// cells and writes the cell's interaction map.
// ---------------------------------------------------------------------------
template <typename S, typename F, int TZ, bool STAGE2, bool MOVING, int LIM, bool CURVED>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
k_stage(StageArgs a, StagePtrs p) {
  constexpr int TY = !MOVING ? 8 : 4, NT = TX * TY;  // rows per tile (one per wave), threads
  constexpr int RX = TX + 4, RY = TY + 4;
  constexpr int NW = TZ + 4;  // column window: planes z0-2 .. z0+TZ+1
  static_assert(4 * TZ <= TX, "the x halo takes four lanes per plane");
  // curved geometry: per-direction face records {gP, gN, gA, x} for the x
  // (phi) rows (k, ty) -- x holds the centre factor --, the y (theta) faces
  // (k, 0..TY) and the z (r) faces (0..TZ, ty)
  constexpr int NRX = TZ * TY, NRY = TZ * (TY + 1), NRZ = (TZ + 1) * TY;
  constexpr int NREC = NRX + NRY + NRZ;
  static_assert(!CURVED || NREC * 4 <= NT, "one record word per thread");
  // Every thread evaluates the slopes and both faces of its cells itself, so
  // the planes and the curved records are the only shared data: they
  // alternate between two buffers (a buffer is rewritten two directions later,
  // after a barrier that every reader of it has passed), and one barrier per
  // direction suffices.
  __shared__ F plb[2][TZ][RY][RX];  // planes of the tile with x/y halo
  __shared__ F grec[CURVED ? 2 : 1][CURVED ? NREC * 4 : 1];

  // ---- tile (XCD-aware order)
  const int b = blockIdx.x;
  const int tile = (b % 8) * a.tiles_per_xcd + b / 8;
  if (tile >= a.ntiles) return;
  int bx, by, bz;
  if (p.tile_order) {
    const unsigned code = p.tile_order[tile];
    bx = (int)(code & 1023u);
    by = (int)((code >> 10) & 2047u);
    bz = (int)(code >> 21);
  } else {
    bx = tile % a.tiles_x;
    by = (tile / a.tiles_x) % a.tiles_y;
    bz = tile / (a.tiles_x * a.tiles_y);
  }
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
  const int t = threadIdx.x, tx = t % TX, ty = t / TX;
  const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
  const long long nc = a.nc;
  const S* __restrict__ Iflux = (const S*)p.Iflux_v;
  const S* Ibase = (const S*)p.Ibase_v;  // may alias Iout (same cell, earlier direction)
  S* Iout = (S*)p.Iout_v;
  const bool per0 = a.bc_lo[0] == RT_BC_PERIODIC, per1 = a.bc_lo[1] == RT_BC_PERIODIC,
             per2 = a.bc_lo[2] == RT_BC_PERIODIC;
  auto gcell = [&](int z, int y, int x) -> int {
    return (int)(((long long)wrap_clamp(z, n1, per0) * n2 + wrap_clamp(y, n2, per1)) * n3 +
                 wrap_clamp(x, n3, per2));
  };
  // sides of the domain a position lies outside of, where the boundary is
  // zero-incoming (bits: z lo, z hi, y lo, y hi, x lo, x hi)
  auto zi_flags = [&](int z, int y, int x) -> unsigned {
    unsigned f = 0;
    if (z < 0 && a.bc_lo[0] == RT_BC_ZERO_INCOMING) f |= 1u;
    if (z >= n1 && a.bc_hi[0] == RT_BC_ZERO_INCOMING) f |= 2u;
    if (y < 0 && a.bc_lo[1] == RT_BC_ZERO_INCOMING) f |= 4u;
    if (y >= n2 && a.bc_hi[1] == RT_BC_ZERO_INCOMING) f |= 8u;
    if (x < 0 && a.bc_lo[2] == RT_BC_ZERO_INCOMING) f |= 16u;
    if (x >= n3 && a.bc_hi[2] == RT_BC_ZERO_INCOMING) f |= 32u;
    return f;
  };
  // curved: offset of a position's boundary face in the incoming flags (-1:
  // inside, or outside two sides at once -- such cells feed no valid cell)
  auto zi_offset = [&](unsigned f, int z, int y, int x) -> int {
    const int b2 = 2 * n2, b1 = 2 * n2 + n1, bp = 2 * n2 + 2 * n1, np = n1 * n2;
    const bool iz = z >= 0 && z < n1, iy = y >= 0 && y < n2, ix = x >= 0 && x < n3;
    return ((f & 1u) && iy && ix) ? y
         : ((f & 2u) && iy && ix) ? n2 + y
         : ((f & 4u) && iz && ix) ? b2 + z
         : ((f & 8u) && iz && ix) ? b1 + z
         : ((f & 16u) && iz && iy) ? bp + z * n2 + y
         : ((f & 32u) && iz && iy) ? bp + np + z * n2 + y : -1;
  };
  auto map_of = [&](int cell, F& ma, F& mb) {
    ma = F(1);
    mb = F(0);
    if (p.mapF) {
      ma = (F)p.mapF[cell];
      mb = (F)p.mapF[nc + cell];
    }
  };

  // ---- what this thread loads every direction
  const int gx = x0 + tx, gy = y0 + ty;
  // column window j = 0..NW-1 at z = z0 - 2 + j
  int wcell[NW];
  F wA[NW], wB[NW];
  unsigned long long wflag = 0;  // 6 bits per window slot
  static_assert(6 * NW <= 64 && 6 * TZ <= 32, "zero-incoming flag packing");
  int wzoff[CURVED ? NW : 1];
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int gz = z0 - 2 + j;
    wcell[j] = gcell(gz, gy, gx);
    map_of(wcell[j], wA[j], wB[j]);
    const unsigned f = zi_flags(gz, gy, gx);
    if (CURVED) wzoff[j] = zi_offset(f, gz, gy, gx);
    else wflag |= (unsigned long long)f << (6 * j);
  }
  // y halo: waves 0..3 load row ty of {y0-2, y0-1, y0+TY, y0+TY+1} for the TZ own planes
  const bool yh = ty < 4;                  // the four waves that load the y halo rows
  const int hry = ty < 2 ? ty : TY + ty;  // region row
  const int hgy = y0 - 2 + hry;
  int ycell[TZ];
  F yA[TZ], yB[TZ];
  unsigned yflag = 0;
  int yzoff[CURVED ? TZ : 1];
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    ycell[k] = gcell(z0 + k, hgy, gx);
    map_of(ycell[k], yA[k], yB[k]);
    const unsigned f = zi_flags(z0 + k, hgy, gx);
    if (CURVED) yzoff[k] = zi_offset(f, z0 + k, hgy, gx);
    else yflag |= f << (6 * k);
  }
  // x halo: lanes < 4 TZ of each wave, column hc = lane % 4 of {x0-2, x0-1,
  // x0+TX, x0+TX+1} on row ty, plane lane / 4
  const bool xh = tx < 4 * TZ;
  const int hcol = tx % 4, hk = (tx / 4) % TZ;
  const int hrx = hcol < 2 ? hcol : TX + hcol;  // region column
  const int hgx = x0 - 2 + hrx;
  const int xcell = gcell(z0 + hk, gy, hgx);
  F xA, xB;
  map_of(xcell, xA, xB);
  const unsigned xflag = zi_flags(z0 + hk, gy, hgx);
  const int xzoff = CURVED ? zi_offset(xflag, z0 + hk, gy, hgx) : -1;

  // ---- own cells (the window's planes 2 .. TZ+1; overhang cells are not stored)
  bool valid[TZ];
#pragma unroll
  for (int k = 0; k < TZ; ++k) valid[k] = gx < n3 && gy < n2 && z0 + k < n1;
  auto own = [&](int k) -> long long { return wcell[k + 2]; };
  // byte offsets of the loaded cells within one direction's plane: they fit in
  // 32 bits (checked on the host), so every access in the direction loop is a
  // uniform base plus an unsigned offset and needs no 64-bit address arithmetic
  unsigned woff[NW], yoff[TZ];
#pragma unroll
  for (int j = 0; j < NW; ++j) woff[j] = (unsigned)wcell[j] * (unsigned)sizeof(S);
#pragma unroll
  for (int k = 0; k < TZ; ++k) yoff[k] = (unsigned)ycell[k] * (unsigned)sizeof(S);
  const unsigned xoff = (unsigned)xcell * (unsigned)sizeof(S);
  // Stores go through buffer resources with these offsets, and so do the
  // loads at rest; the moving kernels' loads, which would need a resource per
  // plane (too many scalar registers in these register-bound kernels), index
  // with the cell numbers.
  const unsigned pbytes = (unsigned)nc * (unsigned)sizeof(S);
  auto ld = [&](const S* base, unsigned off, int cell) -> S {
    if constexpr (MOVING) return base[cell];
    else return bload<S>(plane_rsrc(base, pbytes), off);
  };

  // ---- coefficients of the faces this thread computes (direction independent)
  auto ahat_of = [&](int c) -> double {
    double aa, as;
    opac(a, p.rho, p.Tcoef, p.ka, p.ks, c, aa, as);
    return (MOVING ? p.uhat[c] : 1.0) * (aa + as);
  };
  // the face between cells (z, y, x) - d and (z, y, x) along axis `axis`
  struct Face {
    F u, v, d;     // E Wu, E Wd, Dc:  P = u + d, Q = v - d
    F aL, aR;      // advection: (1-E) max(vL, 0), (1-E) min(vR, 0)
  };
  // ahL, ahR: ahat of the cells below and above the face
  auto make_face = [&](int axis, int z, int y, int x, double ahL, double ahR) -> Face {
    const int dz = axis == 0, dy = axis == 1, dx = axis == 2;
    const double tau = a.abar * 0.5 * (ahL + ahR) * a.dt;
    double P, Q, U, V, E;
    face_coefs(tau, P, Q, U, V, E);
    Face fc;
    fc.u = (F)(2.0 * U);
    fc.v = (F)(2.0 * V);
    fc.d = (F)(P - 2.0 * U);
    fc.aL = fc.aR = F(0);
    if (MOVING) {
      const double* vel = p.vel + axis * nc;
      const double vm2 = vel[gcell(z - 2 * dz, y - 2 * dy, x - 2 * dx)];
      const double vm1 = vel[gcell(z - dz, y - dy, x - dx)];
      const double v0 = vel[gcell(z, y, x)];
      const double vp1 = vel[gcell(z + dz, y + dy, x + dx)];
      const double vL = vm1 + 0.5 * lim_slope(vm1 - vm2, v0 - vm1, a.limiter);
      const double vR = v0 - 0.5 * lim_slope(v0 - vm1, vp1 - v0, a.limiter);
      fc.aL = (F)((1.0 - E) * fmax(vL, 0.0));
      fc.aR = (F)((1.0 - E) * fmin(vR, 0.0));
    }
    return fc;
  };
  // lower faces of the own cells along x and y (fcx, fcy), their upper faces
  // (fcxu, fcyu: the same operands as the neighbours' lower faces), and the
  // TZ + 1 z faces of the column
  Face fcx[TZ], fcy[TZ], fcz[TZ + 1], fcxu[TZ], fcyu[TZ];
  if (MOVING) {
    // (the moving kernels are register bound: no values are kept across faces)
#pragma unroll
    for (int f = 0; f <= TZ; ++f) {
      fcz[f] = make_face(0, z0 + f, gy, gx, ahat_of(gcell(z0 + f - 1, gy, gx)), ahat_of(gcell(z0 + f, gy, gx)));
      if (f < TZ) {
        fcx[f] = make_face(2, z0 + f, gy, gx, ahat_of(gcell(z0 + f, gy, gx - 1)), ahat_of(gcell(z0 + f, gy, gx)));
        fcy[f] = make_face(1, z0 + f, gy, gx, ahat_of(gcell(z0 + f, gy - 1, gx)), ahat_of(gcell(z0 + f, gy, gx)));
        fcxu[f] = make_face(2, z0 + f, gy, gx + 1, ahat_of(gcell(z0 + f, gy, gx)), ahat_of(gcell(z0 + f, gy, gx + 1)));
        fcyu[f] = make_face(1, z0 + f, gy + 1, gx, ahat_of(gcell(z0 + f, gy, gx)), ahat_of(gcell(z0 + f, gy + 1, gx)));
      }
    }
  } else {
    // walk up the column z0-1 .. z0+TZ, evaluating each cell's ahat once
    double ahp = ahat_of(gcell(z0 - 1, gy, gx));
#pragma unroll
    for (int f = 0; f <= TZ; ++f) {
      const double ahn = ahat_of(gcell(z0 + f, gy, gx));
      fcz[f] = make_face(0, z0 + f, gy, gx, ahp, ahn);
      if (f < TZ) {
        fcx[f] = make_face(2, z0 + f, gy, gx, ahat_of(gcell(z0 + f, gy, gx - 1)), ahn);
        fcy[f] = make_face(1, z0 + f, gy, gx, ahat_of(gcell(z0 + f, gy - 1, gx)), ahn);
        fcxu[f] = make_face(2, z0 + f, gy, gx + 1, ahn, ahat_of(gcell(z0 + f, gy, gx + 1)));
        fcyu[f] = make_face(1, z0 + f, gy + 1, gx, ahn, ahat_of(gcell(z0 + f, gy + 1, gx)));
      }
      ahp = ahn;
    }
  }

  // ---- own-cell data used in the direction loop
  F bA[TZ], bB[TZ];                        // lazy map of the stage-2 base intensity
  double u0[MOVING ? TZ : 1], u1[MOVING ? TZ : 1], u2[MOVING ? TZ : 1], u3[MOVING ? TZ : 1];
  double abh[MOVING ? TZ : 1];             // (alpha^a + alpha^s) h
  double nu0k[TZ];                         // n^0 = 1/lapse (1 when flat)
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    const long long c = own(k);
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
  // curved: the record word this thread stages every direction
  const F* gsrc = nullptr;
  long long gstride = 0;
  if (CURVED && t < NREC * 4) {
    const int rec = t >> 2, comp = t & 3;
    if (rec < NRX) {  // phi rows (k, ty) and centre factors
      const int i1 = z0 + rec / TY, i2 = y0 + rec % TY;
      if (i1 < n1 && i2 < n2) {
        gsrc = (const F*)p.rec_p_v + ((long long)i1 * n2 + i2) * 4 + comp;
        gstride = (long long)n1 * n2 * 4;
      }
    } else if (rec < NRX + NRY) {  // theta faces (k, 0..TY)
      const int r2 = rec - NRX, i1 = z0 + r2 / (TY + 1), i2 = y0 + r2 % (TY + 1);
      if (i1 < n1 && i2 <= n2) {
        gsrc = (const F*)p.rec_t_v + ((long long)i1 * (n2 + 1) + i2) * 4 + comp;
        gstride = (long long)n1 * (n2 + 1) * 4;
      }
    } else {  // r faces (0..TZ, ty)
      const int r3 = rec - NRX - NRY, i1 = z0 + r3 / TY, i2 = y0 + r3 % TY;
      if (i1 <= n1 && i2 < n2) {
        gsrc = (const F*)p.rec_r_v + ((long long)i1 * n2 + i2) * 4 + comp;
        gstride = (long long)(n1 + 1) * n2 * 4;
      }
    }
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
  // per-direction constants through the constant address space: uniform
  // scalar loads, which wait on the scalar counter only (a vector load here
  // would wait behind the plane stores and prefetches of the direction loop)
  const CPtr<F> dirF = (CPtr<F>)p.dirF_v;
  const CPtr<double> wdir = (CPtr<double>)p.w;
  const CPtr<double> dirD = (CPtr<double>)p.dirD;
  const S* angD = (const S*)p.angD_v;

  // ---- prefetch of direction 0
  S pw[NW], py[TZ], px, pb[TZ], pda[CURVED ? TZ : 1];
  F gpre = F(0);
  auto prefetch = [&](int s) {
    const S* Is = Iflux + (long long)s * nc;
#pragma unroll
    for (int j = 0; j < NW; ++j) pw[j] = ld(Is, woff[j], wcell[j]);
#pragma unroll
    for (int k = 0; k < TZ; ++k) py[k] = yh ? ld(Is, yoff[k], ycell[k]) : S(0);
    px = ld(Is, xoff, xcell);
    if (STAGE2) {
      const S* Ib = Ibase + (long long)s * nc;
#pragma unroll
      for (int k = 0; k < TZ; ++k) pb[k] = ld(Ib, woff[k + 2], wcell[k + 2]);
    }
    if (CURVED) {
      if (gsrc) gpre = gsrc[(long long)s * gstride];
      const S* As = angD + (long long)s * nc;
#pragma unroll
      for (int k = 0; k < TZ; ++k) pda[k] = ld(As, woff[k + 2], wcell[k + 2]);
    }
  };
  prefetch(0);
  // Direction 0's loads complete before the loop: then the only loads pending
  // at the top of an iteration are the prefetch of the previous one, issued
  // before its stores, and the compiler's wait for them can leave those stores
  // in flight (s_waitcnt vmcnt(0), other counters untouched)
  __builtin_amdgcn_s_waitcnt(0x0F70);

  // a thread with no zero-incoming ghost among its slots skips the checks
  bool anyghost = false;
  if (CURVED) {
#pragma unroll
    for (int j = 0; j < NW; ++j) anyghost |= wzoff[j] >= 0;
#pragma unroll
    for (int k = 0; k < TZ; ++k) anyghost |= yzoff[k] >= 0;
    anyghost |= xh && xzoff >= 0;
  } else {
    anyghost = wflag != 0ull || yflag != 0u || (xh && xflag != 0u);
  }
  // flat at rest: the direction component is taken out of the face fluxes and
  // applied once per cell in the divergence
  constexpr bool NUOUT = !CURVED && !MOVING;

  for (int s = 0; s < ns; ++s) {
    const int buf = s & 1;
    auto& pl = plb[buf];
    // direction components along i1 (z), i2 (y), i3 (x)
    const F nz = dirF[s], ny = dirF[ns + s], nx = dirF[2 * ns + s];
    // flat zero-incoming: the outside sides that receive zero for this direction
    const unsigned inc = (upos(nz) ? 1u : 0u) | (uneg(nz) ? 2u : 0u) | (upos(ny) ? 4u : 0u) |
                         (uneg(ny) ? 8u : 0u) | (upos(nx) ? 16u : 0u) | (uneg(nx) ? 32u : 0u);
    const unsigned char* zs = CURVED ? p.zin + (long long)s * a.zin_stride : nullptr;
    auto ghost_zero = [&](unsigned flags6, int zoff) -> bool {
      if (CURVED) return zoff >= 0 && zs[zoff] != 0;
      return (flags6 & inc) != 0u;
    };
    // 1. column window in registers, own planes and halos to LDS
    F w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) w[j] = wA[j] * (F)pw[j] + wB[j];
    F yv[TZ];
#pragma unroll
    for (int k = 0; k < TZ; ++k) yv[k] = yA[k] * (F)py[k] + yB[k];
    F xv = xA * (F)px + xB;
    if (anyghost) {
#pragma unroll
      for (int j = 0; j < NW; ++j)
        if (ghost_zero((unsigned)(wflag >> (6 * j)) & 63u, CURVED ? wzoff[j] : -1)) w[j] = F(0);
#pragma unroll
      for (int k = 0; k < TZ; ++k)
        if (ghost_zero((yflag >> (6 * k)) & 63u, CURVED ? yzoff[k] : -1)) yv[k] = F(0);
      if (ghost_zero(xflag, xzoff)) xv = F(0);
    }
#pragma unroll
    for (int k = 0; k < TZ; ++k) pl[k][ty + 2][tx + 2] = w[k + 2];
    if (yh) {
#pragma unroll
      for (int k = 0; k < TZ; ++k) pl[k][hry][tx + 2] = yv[k];
    }
    if (xh) pl[hk][ty + 2][hrx] = xv;
    F base[TZ], dang[CURVED ? TZ : 1];
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
      base[k] = STAGE2 ? bA[k] * (F)pb[k] + bB[k] : w[k + 2];
      if (CURVED) dang[k] = (F)pda[k];
    }
    F* GR = grec[CURVED ? buf : 0];
    if (CURVED && t < NREC * 4) GR[t] = gpre;
    __syncthreads();
    if (s + 1 < ns) prefetch(s + 1);

    F ddx[TZ], ddy[TZ];  // differences of the x and y face fluxes of the own cells
    F fz[TZ + 1];        // z faces of the column
    // 2. half slopes and both faces of the own cells along every axis: x and y
    // from the staged planes, z from the column window.  A face shared by two
    // cells is evaluated by both threads from the same operands.
    //
    // With the cell values vm1 | v0 either side of a face and their half slopes
    // hL, hR, the modified flux of Sec. 3.5 is
    //   nu > 0:  nu (u (vm1 + hL) + v (v0 - hR) + d (vm1 - v0))
    //   nu < 0:  nu (v (vm1 + hL) + u (v0 - hR) - d (vm1 - v0))
    // plus the advection term aL (vm1 + hL) + aR (v0 - hR) for a moving fluid.
    // Curved: the face record's gP, gN (one of them zero) and gA weight the two
    // branches and the advection term.  Flat: the sign of the direction
    // component is uniform over a face group, so each group takes one branch
    // (POS); at rest nu is applied once per cell in the divergence.
    // dq = v0 - vm1 is the difference the slopes have already formed, so
    // vm1 - v0 = -dq (exactly) costs nothing here.
    auto fpos = [&](auto pos_tag, const Face& fc, int rec, F nu, F vm1, F hL, F v0, F hR, F dq) -> F {
      constexpr int POS = decltype(pos_tag)::value;
      const F L = vm1 + hL, Rr = v0 - hR, D = -dq;
      F f;
      if (CURVED) {
        const F* r = GR + rec * 4;
        f = r[0] * (fc.u * L + fc.v * Rr + fc.d * D) + r[1] * (fc.v * L + fc.u * Rr - fc.d * D);
        if (MOVING) f += r[2] * (fc.aL * L + fc.aR * Rr);
      } else {
        f = POS ? fc.u * L + fc.v * Rr + fc.d * D : fc.v * L + fc.u * Rr - fc.d * D;
        if (!NUOUT) f *= nu;
        if (MOVING) f += fc.aL * L + fc.aR * Rr;
      }
      return f;
    };
    // upper minus lower face flux of the cell c2 from the values c0 .. c4 along the axis
    auto div1 = [&](auto pos, const Face& lo, const Face& hi, int rlo, int rhi, F nu, F c0, F c1, F c2,
                    F c3, F c4) -> F {
      const F d01 = c1 - c0, d12 = c2 - c1, d23 = c3 - c2, d34 = c4 - c3;
      const F hm = half_slope<LIM>(d01, d12), h0 = half_slope<LIM>(d12, d23), hp = half_slope<LIM>(d23, d34);
      return fpos(pos, hi, rhi, nu, c2, h0, c3, hp, d23) - fpos(pos, lo, rlo, nu, c1, hm, c2, h0, d12);
    };
    auto xpart = [&](auto pos) {
#pragma unroll
      for (int k = 0; k < TZ; ++k)
        ddx[k] = div1(pos, fcx[k], fcxu[k], k * TY + ty, k * TY + ty, nx, pl[k][ty + 2][tx],
                      pl[k][ty + 2][tx + 1], w[k + 2], pl[k][ty + 2][tx + 3], pl[k][ty + 2][tx + 4]);
    };
    auto ypart = [&](auto pos) {
#pragma unroll
      for (int k = 0; k < TZ; ++k)
        ddy[k] = div1(pos, fcy[k], fcyu[k], NRX + k * (TY + 1) + ty, NRX + k * (TY + 1) + ty + 1, ny,
                      pl[k][ty][tx + 2], pl[k][ty + 1][tx + 2], w[k + 2], pl[k][ty + 3][tx + 2],
                      pl[k][ty + 4][tx + 2]);
    };
    auto zpart = [&](auto pos) {
      F dz[NW - 1], sz[NW];
#pragma unroll
      for (int j = 0; j + 1 < NW; ++j) dz[j] = w[j + 1] - w[j];
#pragma unroll
      for (int j = 1; j <= TZ + 2; ++j) sz[j] = half_slope<LIM>(dz[j - 1], dz[j]);
#pragma unroll
      for (int f = 0; f <= TZ; ++f)
        fz[f] = fpos(pos, fcz[f], NRX + NRY + f * TY + ty, nz, w[f + 1], sz[f + 1], w[f + 2], sz[f + 2],
                     dz[f + 1]);
    };
    using TPos = std::integral_constant<int, 1>;
    using TNeg = std::integral_constant<int, 0>;
    if (CURVED) {
      xpart(TPos{});
      ypart(TPos{});
      zpart(TPos{});
    } else {
      if (upos(nx)) xpart(TPos{}); else xpart(TNeg{});
      if (upos(ny)) ypart(TPos{}); else ypart(TNeg{});
      if (upos(nz)) zpart(TPos{}); else zpart(TNeg{});
    }

    // 3. divergence, update, interaction sums
    const double ws = wdir[s];
    const double hw4 = a.h / (4.0 * kPi) * ws;
    const F cz = NUOUT ? h * nz * idx0 : h * idx0, cy = NUOUT ? h * ny * idx1 : h * idx1,
            cx = NUOUT ? h * nx * idx2 : h * idx2;
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
      const F dx = ddx[k], dy = ddy[k];
      const F dz = fz[k + 1] - fz[k];
      F It;
      if (CURVED) {
        // X = n^0 n_0 I updated by the area-weighted face fluxes; x = 1/(dV n^0 n_0),
        // zero where |n_0| is below the cut (I~ = 0 there)
        const F x = GR[(k * TY + ty) * 4 + 3];
        It = (x != F(0) ? base[k] : F(0)) - h * (x * (dz + dy + dx) + dang[k]);
      } else {
        It = base[k] - (dz * cz + dy * cy + dx * cx);
      }
      // every lane stores: a cell outside the grid gets an offset past the
      // plane, which the buffer's range check drops.  Unconditional stores
      // keep the count of outstanding vector operations known, so the wait
      // for the next direction's loads need not wait for these stores too.
      bstore<S>(plane_rsrc(Iout + (long long)s * nc, pbytes), valid[k] ? woff[k + 2] : kDropOffset, (S)It);
      // ---- interaction sums (FP64)
      const double Itd = (double)(S)It;
      if (MOVING) {
        const double nb = u0[k] - (u1[k] * dirD[s] + u2[k] * dirD[ns + s] + u3[k] * dirD[2 * ns + s]);
        // with Ib = I~ nb^4, dOb = w / nb^2 and den = n^0 + nb abar h:
        //   Ib dOb = w I~ nb^2,  n^0 Ib dOb / den,  nb h dOb / (4 pi den) = h w / (4 pi nb den)
        // (one division: q = 1 / (nb den))
        const double wI = ws * Itd * (nb * nb);
        const double q = rcp_pos(nb * (nu0k[k] + nb * abh[k]));  // nb > 0, den > 0
        acc[k][0] += wI;
        acc[k][1] += wI * nb * q;  // times n^0 when the cell is solved
        acc[k][2] += hw4 * q;
      } else {
        acc[k][0] += ws * Itd;
      }
    }
  }

  // ---- per-cell implicit temperature and the interaction map
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    if (!valid[k]) continue;
    const long long c = own(k);
    if (!MOVING && p.sumE) {
      // one bin of a multi-group step: the solve couples all bins later
      p.sumE[c] = acc[k][0];
      continue;
    }
    double aak, ask;
    opac(a, p.rho, p.Tcoef, p.ka, p.ks, c, aak, ask);
    const double ab = aak + ask, rrk = p.rho[c], T0k = p.Tstart[c];
    const bool live = rrk >= a.rho_floor;
    double Em, A1, A2;
    if (MOVING) {
      Em = acc[k][0];
      A1 = nu0k[k] * acc[k][1];
      A2 = acc[k][2];
    } else {
      const double cs = 1.0 / (1.0 + ab * a.h);
      Em = acc[k][0];
      A1 = cs * Em;
      A2 = a.h / (4.0 * kPi * (1.0 + ab * a.h)) * a.W0;
    }
    Solve so{T0k, 0.0, 1.0, false};
    if (live) {
      const bool brems = a.model == RT_OPAC_BREMS || a.model == RT_OPAC_BREMS_M3;
      const double jc = brems ? (p.ka ? p.ka[c] : 1.0) : (p.jv ? p.jv[c] : 0.0);
      so = solve_cell(a, rrk, T0k, aak, ask, Em, A1, A2, jc);
      if (!so.ok && p.fail) atomicAdd(p.fail, 1ull);
    }
    const bool use = live && so.ok;
    p.Tout[c] = use ? so.T : T0k;
    if (MOVING) {
      // parameters of the direction-dependent map, applied by the materialisation
      p.mapO[c] = use ? so.Q : 0.0;
      p.mapO[nc + c] = ab;
      // > 0: apply the interaction times this factor (alpha_-/alpha_+ in
      // Method 3, else 1), 0: keep I~, < 0: zero (rows next to the axis)
      const int gyk = (int)((c / n3) % n2);
      const bool pole = CURVED && (gyk < a.pole_rows || gyk >= n2 - a.pole_rows);
      p.mapO[2 * nc + c] = pole ? -1.0 : (use ? so.r : 0.0);
    } else {
      const double al = use ? so.r / (1.0 + ab * a.h) : 1.0;
      const double be = use ? so.r * a.h * so.Q / (4.0 * kPi * (1.0 + ab * a.h)) : 0.0;
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
              const double* __restrict__ nu0, int n3, int acc) {
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
      for (int m = 0; m < 10; ++m) Rout[m * nc + c] = (acc ? Rout[m * nc + c] : 0.0) + R[m];
    if (Gout)
      for (int m = 0; m < 4; ++m) Gout[m * nc + c] = (acc ? Gout[m * nc + c] : 0.0) - g[m] / h;
    return;
  }
  const double Q = map[c], ab = map[nc + c];
  const double code = map[2 * nc + c];  // > 0: apply times code, 0: keep, < 0: zero
  const bool use = code > 0.0, zero = code < 0.0;
  const double n0c = nu0 ? nu0[c / n3] : 1.0;
  const double u0 = uhat[c], u1 = uhat[nc + c], u2 = uhat[2 * nc + c], u3 = uhat[3 * nc + c];
  const double hQ = h / (4.0 * kPi) * Q;
  double R[10];
  for (int m = 0; m < 10; ++m) R[m] = 0.0;
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  // batches of B directions, the next batch's loads issued before this
  // batch's arithmetic (the batches are disjoint directions).  Stores go
  // through buffer resources and every lane stores (a cell that keeps I~
  // stores at an offset the range check drops), so waiting for the next
  // batch's loads does not wait for this batch's stores.
  constexpr int B = 8;
  const unsigned pbytes = (unsigned)nc * (unsigned)sizeof(S);
  const unsigned soff = (use || zero) ? (unsigned)c * (unsigned)sizeof(S) : kDropOffset;
  S v[B];
#pragma unroll
  for (int u = 0; u < B; ++u) v[u] = I[(long long)min(u, ns - 1) * nc + c];
  for (int s0 = 0; s0 < ns; s0 += B) {
    S vn[B];
#pragma unroll
    for (int u = 0; u < B; ++u) vn[u] = I[(long long)min(s0 + B + u, ns - 1) * nc + c];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int s = s0 + u;
      if (s >= ns) break;
      const double It = (double)v[u];
      double Io = It;
      if (use) {
        // (c_s I~ nb^4 + d_s Q) / nb^4 with c_s = n^0 / den, d_s = nb h / (4 pi den),
        // den = n^0 + nb abar h, as one division
        const double nb = u0 - (u1 * dirD[s] + u2 * dirD[ns + s] + u3 * dirD[2 * ns + s]);
        const double nb3 = nb * nb * nb;
        Io = code * (n0c * nb3 * It + hQ) * rcp_pos((n0c + nb * ab * h) * nb3);  // nb > 0
      } else if (zero) {
        Io = 0.0;
      }
      bstore<S>(plane_rsrc(I + (long long)s * nc, pbytes), soff, (S)Io);
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
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = vn[u];
  }
  if (Rout)
    for (int m = 0; m < 10; ++m) Rout[m * nc + c] = R[m];
  if (Gout)
    for (int m = 0; m < 4; ++m) Gout[m * nc + c] = -g[m] / h;
}

// At-rest materialisation with two neighbouring cells per thread (vector
// loads and stores of the pair, four directions in flight), optionally with
// the moments and the 4-force of the new intensity.  nc must be even.
template <typename S, bool MOM>
__global__ void __launch_bounds__(256)
k_materialize_pair(long long nc, int ns, double h, const double* __restrict__ map,
                   S* __restrict__ I, const double* __restrict__ W16,
                   double* __restrict__ Rout, double* __restrict__ Gout, int acc) {
  using V2 = typename std::conditional<std::is_same<S, float>::value, float2, double2>::type;
  const long long c = 2 * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= nc) return;
  const double al0 = map[c], al1 = map[c + 1], be0 = map[nc + c], be1 = map[nc + c + 1];
  double R0[MOM ? 10 : 1], R1[MOM ? 10 : 1], g0[MOM ? 4 : 1], g1[MOM ? 4 : 1];
  if (MOM) {
#pragma unroll
    for (int m = 0; m < 10; ++m) R0[m] = R1[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) g0[m] = g1[m] = 0.0;
  }
  V2* q = reinterpret_cast<V2*>(I + c);
  const long long stride = nc / 2;
  // batches of B directions: all loads of a batch are issued before its stores
  // (different directions never alias, which the compiler cannot see)
  constexpr int B = 8;
  for (int s0 = 0; s0 < ns; s0 += B) {
    V2 v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = q[(long long)min(s0 + u, ns - 1) * stride];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int s = s0 + u;
      if (s >= ns) break;
      const double t0 = (double)v[u].x, t1 = (double)v[u].y;
      V2 o;
      o.x = (S)(al0 * t0 + be0);
      o.y = (S)(al1 * t1 + be1);
      q[(long long)s * stride] = o;
      if (MOM) {
        const double o0 = (double)o.x, o1 = (double)o.y;
        const double* Ws = W16 + s * 16;
#pragma unroll
        for (int m = 0; m < 10; ++m) {
          R0[m] += Ws[m] * o0;
          R1[m] += Ws[m] * o1;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          g0[m] += Ws[m] * (o0 - t0);
          g1[m] += Ws[m] * (o1 - t1);
        }
      }
    }
  }
  if (MOM) {
    if (Rout)
      for (int m = 0; m < 10; ++m) {
        Rout[m * nc + c] = (acc ? Rout[m * nc + c] : 0.0) + R0[m];
        Rout[m * nc + c + 1] = (acc ? Rout[m * nc + c + 1] : 0.0) + R1[m];
      }
    if (Gout)
      for (int m = 0; m < 4; ++m) {
        Gout[m * nc + c] = (acc ? Gout[m * nc + c] : 0.0) - g0[m] / h;
        Gout[m * nc + c + 1] = (acc ? Gout[m * nc + c + 1] : 0.0) - g1[m] / h;
      }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
// Order the tiles so that the tiles of one XCD that are resident together form
// a compact brick: a tile's halo planes then come from L2 (the neighbouring
// tiles stage the same direction at about the same time) instead of HBM.
// The order is a permutation of the tiles; codes pack (tx, ty, tz).
hipError_t tile_order(rt_ctx* c, int tx, int ty, int tz, int TYc, int TZc, int resident,
                      bool may_alloc, const unsigned** out) {
  *out = nullptr;
  if (tx > 1024 || ty > 2048 || tz > 2048) return hipSuccess;  // natural order
  const long long key = (((long long)tx * 4096 + ty) * 4096 + tz) * 64 * 64 +
                        (long long)(TYc * 8 + TZc) * 64 + std::min(resident, 63);
  if (key != c->tile_order_key && !may_alloc) return hipSuccess;  // natural order, nothing allocated
  if (key != c->tile_order_key) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int conc = std::max(1, cus / 8 * resident);  // tiles in flight per XCD
    const int GX = std::min(tx, 2);
    int GY = 1, GZ = 1;
    double best = 1e30;
    for (int gy = 1; gy <= ty; ++gy) {
      const int gz = std::max(1, std::min(tz, conc / (GX * gy)));
      const double aspect = std::fabs(std::log((double)(gy * TYc) / (gz * TZc)));
      const double fill = std::fabs(std::log((double)(GX * gy * gz) / conc));
      if (aspect + 2.0 * fill < best) {
        best = aspect + 2.0 * fill;
        GY = gy;
        GZ = gz;
      }
    }
    std::vector<unsigned> ord;
    ord.reserve((size_t)tx * ty * tz);
    for (int z0 = 0; z0 < tz; z0 += GZ)
      for (int y0 = 0; y0 < ty; y0 += GY)
        for (int x0 = 0; x0 < tx; x0 += GX)
          for (int z = z0; z < std::min(tz, z0 + GZ); ++z)
            for (int y = y0; y < std::min(ty, y0 + GY); ++y)
              for (int x = x0; x < std::min(tx, x0 + GX); ++x)
                ord.push_back((unsigned)x | ((unsigned)y << 10) | ((unsigned)z << 21));
    if (c->d_tile_order) (void)hipFree(c->d_tile_order);
    c->d_tile_order = nullptr;
    c->tile_order_key = -1;
    hipError_t e = hipMalloc((void**)&c->d_tile_order, ord.size() * sizeof(unsigned));
    if (e != hipSuccess) return e;
    e = hipMemcpy(c->d_tile_order, ord.data(), ord.size() * sizeof(unsigned), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    c->tile_order_key = key;
  }
  *out = c->d_tile_order;
  return hipSuccess;
}

template <typename Kern>
hipError_t launch_ordered(rt_ctx* c, Kern kern, StageArgs a, StagePtrs p, int TYc, int TZc,
                          hipStream_t st, bool may_alloc) {
  int resident = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, reinterpret_cast<const void*>(kern),
                                                   TX * TYc, 0) != hipSuccess)
    resident = 1;
  hipError_t e = tile_order(c, a.tiles_x, a.tiles_y, a.tiles_z, TYc, TZc, std::max(resident, 1),
                            may_alloc, &p.tile_order);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(8 * a.tiles_per_xcd), dim3(TX * TYc), 0, st, a, p);
  return hipGetLastError();
}

// MOVE: the moving-fluid family (moving fluid or curved geometry), else at rest
template <typename S, typename F, int TZ, int LIM, bool MOVE>
hipError_t launch_tiled(rt_ctx* c, StageArgs a, const StagePtrs& p, bool stage2, hipStream_t st,
                        bool ma) {
  constexpr int TY = !MOVE ? 8 : 4;  // as in k_stage
  a.tiles_x = (c->n[2] + TX - 1) / TX;
  a.tiles_y = (c->n[1] + TY - 1) / TY;
  a.tiles_z = (c->n[0] + TZ - 1) / TZ;
  a.ntiles = a.tiles_x * a.tiles_y * a.tiles_z;
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  if constexpr (MOVE) {
    if (c->curved) {
      // curved geometry always runs the moving-fluid form (direction-dependent map)
      return stage2 ? launch_ordered(c, k_stage<S, F, TZ, true, true, LIM, true>, a, p, TY, TZ, st, ma)
                    : launch_ordered(c, k_stage<S, F, TZ, false, true, LIM, true>, a, p, TY, TZ, st, ma);
    }
    return stage2 ? launch_ordered(c, k_stage<S, F, TZ, true, true, LIM, false>, a, p, TY, TZ, st, ma)
                  : launch_ordered(c, k_stage<S, F, TZ, false, true, LIM, false>, a, p, TY, TZ, st, ma);
  } else {
    return stage2 ? launch_ordered(c, k_stage<S, F, TZ, true, false, LIM, false>, a, p, TY, TZ, st, ma)
                  : launch_ordered(c, k_stage<S, F, TZ, false, false, LIM, false>, a, p, TY, TZ, st, ma);
  }
}
}  // namespace

hipError_t launch_stage(rt_ctx* c, const StageArgs& a, const StagePtrs& p, bool stage2,
                        hipStream_t st, bool may_alloc) {
  // every pointer the kernel dereferences must be there: the interaction
  // outputs unless only the per-cell sums are asked for (at rest)
  if (!p.Iflux_v || !p.Iout_v || !p.rho || !p.Tcoef || (stage2 && !p.Ibase_v))
    return hipErrorInvalidValue;
  if (p.sumE ? (c->moving || c->curved) : (!p.Tout || !p.mapO || !p.Tstart)) return hipErrorInvalidValue;
  const bool mc = a.limiter == RT_LIM_MC;
  // the moving-fluid and curved forms carry more per-cell state (the fluid
  // velocity, advection weights, records): two cells per column (one in FP64)
  // keep them in registers
  const bool mv = c->moving || c->curved;
  if (c->fp32 && mv)
    return mc ? launch_tiled<float, float, 2, RT_LIM_MC, true>(c, a, p, stage2, st, may_alloc)
              : launch_tiled<float, float, 2, RT_LIM_MINMOD, true>(c, a, p, stage2, st, may_alloc);
  if (c->fp32) {
    // columns of 4 cells, or of 2 when columns of 4 leave fewer than two tiles
    // per compute unit (small grids: the same per-cell arithmetic, so the same
    // results, on twice as many workgroups)
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long tiles4 = (long long)((c->n[2] + TX - 1) / TX) * ((c->n[1] + 7) / 8) * ((c->n[0] + 3) / 4);
    if (tiles4 < 2LL * cus && c->n[0] > 2)
      return mc ? launch_tiled<float, float, 2, RT_LIM_MC, false>(c, a, p, stage2, st, may_alloc)
                : launch_tiled<float, float, 2, RT_LIM_MINMOD, false>(c, a, p, stage2, st, may_alloc);
    return mc ? launch_tiled<float, float, 4, RT_LIM_MC, false>(c, a, p, stage2, st, may_alloc)
              : launch_tiled<float, float, 4, RT_LIM_MINMOD, false>(c, a, p, stage2, st, may_alloc);
  }
  if (mv)
    return mc ? launch_tiled<double, double, 1, RT_LIM_MC, true>(c, a, p, stage2, st, may_alloc)
              : launch_tiled<double, double, 1, RT_LIM_MINMOD, true>(c, a, p, stage2, st, may_alloc);
  return mc ? launch_tiled<double, double, 2, RT_LIM_MC, false>(c, a, p, stage2, st, may_alloc)
            : launch_tiled<double, double, 2, RT_LIM_MINMOD, false>(c, a, p, stage2, st, may_alloc);
}

hipError_t launch_materialize(rt_ctx* c, void* I, const double* map, double h, double* R,
                              double* G, hipStream_t st, bool acc) {
  const int ac = acc ? 1 : 0;
  dim3 grid((unsigned)((c->nc + 255) / 256)), block(256);
  if (!c->moving && c->nc % 2 == 0) {
    const dim3 g2((unsigned)((c->nc / 2 + 255) / 256));
    const bool mom = R || G;
    if (c->fp32) {
      if (mom)
        hipLaunchKernelGGL((k_materialize_pair<float, true>), g2, block, 0, st, c->nc, c->ns, h, map,
                           (float*)I, c->d_W16, R, G, ac);
      else
        hipLaunchKernelGGL((k_materialize_pair<float, false>), g2, block, 0, st, c->nc, c->ns, h, map,
                           (float*)I, c->d_W16, R, G, ac);
    } else {
      if (mom)
        hipLaunchKernelGGL((k_materialize_pair<double, true>), g2, block, 0, st, c->nc, c->ns, h, map,
                           (double*)I, c->d_W16, R, G, ac);
      else
        hipLaunchKernelGGL((k_materialize_pair<double, false>), g2, block, 0, st, c->nc, c->ns, h, map,
                           (double*)I, c->d_W16, R, G, ac);
    }
    return hipGetLastError();
  }
  if (c->fp32) {
    if (c->moving)
      hipLaunchKernelGGL((k_materialize<float, true>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (float*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2], ac);
    else
      hipLaunchKernelGGL((k_materialize<float, false>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (float*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2], ac);
  } else {
    if (c->moving)
      hipLaunchKernelGGL((k_materialize<double, true>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (double*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2], ac);
    else
      hipLaunchKernelGGL((k_materialize<double, false>), grid, block, 0, st, c->nc, c->ns, h, map,
                         (double*)I, c->d_uhat, c->d_dir, c->d_w, c->d_W16, R, G, c->d_nu0, c->n[2], ac);
  }
  return hipGetLastError();
}

}  // namespace rt
