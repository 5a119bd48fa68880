// Multi-group interaction for a fluid at rest in flat space (Sec. 3.1, Eq.
// radiative_transfer_discrete_non_gray with no frequency flux: the fluid-frame
// frequency of a photon does not change along its path, so each bin of
// frequency is transported as the gray equation and the bins couple only
// through the gas temperature).
//
// Per cell, with the per-bin E-_g = sum_s w_s I~_gs written by the stage
// kernels, alpha^a_g = rho kappa_a,g, alpha^s = rho kappa_s and
// alpha_g = alpha^a_g + alpha^s, Method 1's semi-implicit update (Sec. 3.6.2,
// Eq. fluid_interaction_discrete) in every bin with the emission at T_+:
//   c_g = 1/(1 + alpha_g h), A1_g = c_g E-_g, A2_g = h W0/(4 pi (1 + alpha_g h)),
//   q_g = 1 - alpha^s A2_g, S_g(T) = 4 pi alpha^a_g B_g(T),
//   E+_g = (A1_g + A2_g S_g)/q_g,
// and the energy balance Y (T_+ - T_-) = -sum_g (E+_g - E-_g) (Eq.
// ideal_gas_difference), i.e. the root of
//   F(T) = Y (T - T_-) + sum_g ((A1_g + A2_g S_g(T))/q_g - E-_g),
// which increases with T from F(0) < 0; F(T_hi) >= 0 at
// T_hi = T_- + sum_g (E-_g - A1_g/q_g)/Y.  Newton inside that bracket, with
// bisection where a step leaves it.  The map of bin g is then the at-rest
// lazy map I = alpha_g I~ + beta_g with alpha_g = c_g and
// beta_g = h (S_g + alpha^s E+_g)/(4 pi (1 + alpha_g h)).
//
// B_g(T) = int_{nu_g}^{nu_g+1} B_nu dnu with B_nu = 15/(4 pi^5) nu^3/(e^(nu/T) - 1)
// (a_rad = k_B = h = 1), i.e. B_g = T^4/(4 pi) (15/pi^4) D(nu_g/T, nu_g+1/T),
// D(a, b) = int_a^b x^3/(e^x - 1) dx, evaluated by the two classical series of
// the incomplete Planck integral: below x = 2 the Bernoulli series of
// x^3/(e^x - 1) = sum_k B_k x^(k+2)/k! integrated term by term, above it the
// upper tail int_x^inf = sum_n e^(-n x) (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4)
// from 1/(e^x - 1) = sum_n e^(-n x).
#include <hip/hip_runtime.h>

#include <cmath>

#include "ctx.hpp"

namespace rt {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kPlanckC = 15.0 / (kPi * kPi * kPi * kPi);  // 1 / int_0^inf x^3/(e^x - 1) dx

struct MgArgs {
  long long nc;
  int ng, max_iter;
  double h, gamma, rho_floor, W0, rtol;
  double nu[RT_MAX_GROUPS + 1];
};

// The split between the two series is x = 2: below it the Bernoulli series
// (ratio of successive terms about (x / 2 pi)^2) needs the 17 terms below, above
// it the exponential series at most 19.
constexpr double kSplit = 2.0;

// int_0^x t^3/(e^t - 1) dt for 0 <= x <= 2: x^3/3 - x^4/8 + sum_k c_k x^(2k+3),
// c_k = B_2k / ((2k)! (2k + 3)) (Bernoulli numbers B_2k); the first omitted
// term is below 1e-18 of the sum
__device__ __forceinline__ double planck_lo(double x) {
  constexpr double c[17] = {
      1.0 / 6.0 / (2.0 * 5.0),
      -1.0 / 30.0 / (24.0 * 7.0),
      1.0 / 42.0 / (720.0 * 9.0),
      -1.0 / 30.0 / (40320.0 * 11.0),
      5.0 / 66.0 / (3628800.0 * 13.0),
      -691.0 / 2730.0 / (479001600.0 * 15.0),
      7.0 / 6.0 / (87178291200.0 * 17.0),
      -3617.0 / 510.0 / (20922789888000.0 * 19.0),
      43867.0 / 798.0 / (6402373705728000.0 * 21.0),
      -174611.0 / 330.0 / (2432902008176640000.0 * 23.0),
      854513.0 / 138.0 / (1124000727777607680000.0 * 25.0),
      -236364091.0 / 2730.0 / (620448401733239439360000.0 * 27.0),
      8553103.0 / 6.0 / (403291461126605635584000000.0 * 29.0),
      -23749461029.0 / 870.0 / (304888344611713860501504000000.0 * 31.0),
      8615841276005.0 / 14322.0 / (265252859812191058636308480000000.0 * 33.0),
      -7709321041217.0 / 510.0 / (263130836933693530167218012160000000.0 * 35.0),
      2577687858367.0 / 6.0 / (295232799039604140847618609643520000000.0 * 37.0)};
  const double x2 = x * x;
  double s = c[16];
#pragma unroll
  for (int k = 15; k >= 0; --k) s = s * x2 + c[k];
  return x2 * x * (1.0 / 3.0 - 0.125 * x + x2 * s);
}

// 1/n for the exponential series
__constant__ double kInvN[24] = {1.0,        1.0 / 2.0,  1.0 / 3.0,  1.0 / 4.0,  1.0 / 5.0,  1.0 / 6.0,
                                 1.0 / 7.0,  1.0 / 8.0,  1.0 / 9.0,  1.0 / 10.0, 1.0 / 11.0, 1.0 / 12.0,
                                 1.0 / 13.0, 1.0 / 14.0, 1.0 / 15.0, 1.0 / 16.0, 1.0 / 17.0, 1.0 / 18.0,
                                 1.0 / 19.0, 1.0 / 20.0, 1.0 / 21.0, 1.0 / 22.0, 1.0 / 23.0, 1.0 / 24.0};

// int_x^inf t^3/(e^t - 1) dt for 2 <= x < 745, given e1 = e^-x
__device__ __forceinline__ double planck_hi(double x, double e1) {
  const double x2 = x * x, x3 = x2 * x, x6 = 6.0 * x;
  double en = e1, s = 0.0;
  for (int n = 0; n < 24; ++n) {
    const double in = kInvN[n];
    const double term = en * in * (x3 + in * (3.0 * x2 + in * (x6 + 6.0 * in)));
    s += term;
    if (term <= 1e-17 * s) break;
    en *= e1;
  }
  return s;
}

// Values of one bin edge at x = nu/T: lo = int_0^min(x, 2), hi = int_max(x, 2)^inf
// of t^3/(e^t - 1), and x^4/(e^x - 1) (0 at x = 0 and as x -> inf).  A bin's
// integral is then (lo(b) - lo(a)) + (hi(a) - hi(b)), without the cancellation
// of a difference of two complete integrals.
struct EdgeVal {
  double lo, hi, x4;
};
__device__ __forceinline__ EdgeVal edge_val(double x, double lo2, double hi2) {
  EdgeVal e;
  if (!(x < 745.0)) {  // also the edge at infinity
    e.lo = lo2;
    e.hi = 0.0;
    e.x4 = 0.0;
    return e;
  }
  const double x2 = x * x;
  if (x <= kSplit) {
    e.lo = planck_lo(x);
    e.hi = hi2;
    e.x4 = x > 0.0 ? x2 * x2 / expm1(x) : 0.0;
  } else {
    const double e1 = exp(-x);
    e.lo = lo2;
    e.hi = planck_hi(x, e1);
    e.x4 = x2 * x2 * e1 / (1.0 - e1);
  }
  return e;
}

// K_g = alpha^a_g (15/pi^4) A2_g/q_g, with A2_g/q_g = A2f/(den_g - alpha^s A2f)
__device__ __forceinline__ double bin_K(double aa, double as, double h, double A2f) {
  return aa * kPlanckC * A2f / (1.0 + (aa + as) * h - as * A2f);
}

// NGR > 0: at most NGR bins, whose K_g stay in registers; 0: any number, K_g
// recomputed from kappa_a,g (cache hits) in every iteration
template <int NGR>
__global__ void __launch_bounds__(256)
k_mg_solve(MgArgs a, const double* __restrict__ Emg, const double* __restrict__ rho,
           const double* __restrict__ kag, const double* __restrict__ ks, const double* T_start,
           const double* T_guess, double* T_out, double* __restrict__ map,
           unsigned long long* __restrict__ fail) {
  constexpr int kUnroll = NGR > 0 ? NGR : 1;  // the bin loops: unrolled when bounded
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nc = a.nc;
  if (c >= nc) return;
  const double r = rho[c], T0 = T_start[c];
  const bool live = r >= a.rho_floor;
  const double as = (live && ks) ? r * ks[c] : 0.0;
  const double Y = r / (a.gamma - 1.0);
  const double A2f = a.h * a.W0 / (4.0 * kPi);
  const double lo2 = planck_lo(kSplit), hi2 = planck_hi(kSplit, exp(-kSplit));
  // F(T) = Y (T - T_-) - X + T^4 sum_g K_g D_g(T), X = sum_g (E-_g - A1_g/q_g)
  // (the bracket's excess; A1_g/q_g = E-_g/(den_g - alpha^s A2f)).  The bins share
  // their edges, so each Newton iteration evaluates the ng + 1 edges once.
  double excess = 0.0;
  double Kr[NGR > 0 ? NGR : 1];
  if (live) {
#pragma unroll kUnroll
    for (int g = 0; g < (NGR > 0 ? NGR : a.ng); ++g) {
      if (NGR > 0 && g >= a.ng) break;
      const double aa = r * kag[g * nc + c], den = 1.0 + (aa + as) * a.h;
      const double Em = Emg[g * nc + c];
      excess += Em - Em / (den - as * A2f);
      if (NGR > 0) Kr[g] = bin_K(aa, as, a.h, A2f);
    }
  }
  auto eval = [&](double T, double& F, double& dF) {
    const double iT = 1.0 / T, T3 = T * T * T;
    double sD = 0.0, sdD = 0.0;
    EdgeVal ea = edge_val(a.nu[0] * iT, lo2, hi2);
#pragma unroll kUnroll
    for (int g = 0; g < (NGR > 0 ? NGR : a.ng); ++g) {
      if (NGR > 0 && g >= a.ng) break;
      const EdgeVal eb = edge_val(a.nu[g + 1] * iT, lo2, hi2);
      const double K = NGR > 0 ? Kr[g] : bin_K(r * kag[g * nc + c], as, a.h, A2f);
      const double D = (eb.lo - ea.lo) + (ea.hi - eb.hi);
      sD += K * D;
      sdD += K * (4.0 * D - eb.x4 + ea.x4);
      ea = eb;
    }
    F = Y * (T - T0) - excess + T3 * T * sD;
    dF = Y + T3 * sdD;
  };
  double Tp = T0;
  bool ok = false;
  if (live) {
    double lo = 0.0, hi = T0 + excess / Y;
    if (Y > 0.0 && T0 > 0.0 && hi > 0.0) {
      // start from the guess (the stage's coefficient temperature) when it lies
      // inside the bracket
      const double Tg = T_guess[c];
      double x = (Tg > 0.0 && Tg < hi) ? Tg : ((T0 < hi) ? T0 : 0.5 * hi);
      const int iters = max(a.max_iter, 120);
      for (int it = 0; it < iters; ++it) {
        double F, dF;
        eval(x, F, dF);
        if (F > 0.0) hi = x;
        else lo = x;
        const double step = F / dF;
        double xn = x - step;
        // converged: the Newton step is within the tolerance (tested before the
        // bracket guard, which would replace a step onto the bracket's end)
        if (fabs(step) <= a.rtol * x) {
          if (xn >= lo && xn <= hi) x = xn;
          ok = true;
          break;
        }
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        x = xn;
        if (hi - lo <= a.rtol * x) {
          ok = true;
          break;
        }
      }
      Tp = x;
    }
    if (!ok && fail) atomicAdd(fail, 1ull);
  }
  T_out[c] = ok ? Tp : T0;
  if (!ok) {
    for (int g = 0; g < a.ng; ++g) {
      map[2 * g * nc + c] = 1.0;
      map[(2 * g + 1) * nc + c] = 0.0;
    }
    return;
  }
  const double iT = 1.0 / Tp, T4 = Tp * Tp * Tp * Tp;
  EdgeVal ea = edge_val(a.nu[0] * iT, lo2, hi2);
  for (int g = 0; g < a.ng; ++g) {
    const EdgeVal eb = edge_val(a.nu[g + 1] * iT, lo2, hi2);
    const double aa = r * kag[g * nc + c], den = 1.0 + (aa + as) * a.h;
    const double Em = Emg[g * nc + c], A1 = Em / den, A2 = A2f / den, q = 1.0 - as * A2;
    const double S = aa * kPlanckC * T4 * ((eb.lo - ea.lo) + (ea.hi - eb.hi));
    const double Ep = (A1 + A2 * S) / q;
    map[2 * g * nc + c] = 1.0 / den;
    map[(2 * g + 1) * nc + c] = a.h * (S + as * Ep) / (4.0 * kPi * den);
    ea = eb;
  }
}

}  // namespace

hipError_t launch_mg_solve(rt_ctx* c, double h, const double* Emg, const double* T_start,
                           const double* T_guess, double* T_out, double* map, hipStream_t st) {
  MgArgs a{};
  a.nc = c->nc;
  a.ng = c->ng;
  a.max_iter = c->opac.newton_max_iter;
  a.h = h;
  a.gamma = c->opac.gamma;
  a.rho_floor = c->desc.rho_floor;
  a.W0 = c->W0;
  a.rtol = c->opac.newton_rtol;
  for (int g = 0; g <= c->ng; ++g) a.nu[g] = c->nu_edges[g];
  const dim3 grid((unsigned)((c->nc + 255) / 256)), block(256);
  if (c->ng <= 4)
    hipLaunchKernelGGL(k_mg_solve<4>, grid, block, 0, st, a, Emg, c->d_rho, c->d_ka_g, c->d_ks, T_start, T_guess,
                       T_out, map, c->d_count);
  else if (c->ng <= 8)
    hipLaunchKernelGGL(k_mg_solve<8>, grid, block, 0, st, a, Emg, c->d_rho, c->d_ka_g, c->d_ks, T_start, T_guess,
                       T_out, map, c->d_count);
  else
    hipLaunchKernelGGL(k_mg_solve<0>, grid, block, 0, st, a, Emg, c->d_rho, c->d_ka_g, c->d_ks, T_start, T_guess,
                       T_out, map, c->d_count);
  return hipGetLastError();
}

}  // namespace rt
