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
// the incomplete Planck integral: below x = 1 the Bernoulli series of
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

// int_0^x t^3/(e^t - 1) dt for 0 <= x <= 1: x^3/3 - x^4/8 + sum_k c_k x^(2k+3),
// c_k = B_2k / ((2k)! (2k + 3)); the k = 13 term is below 1e-20 of the sum
__device__ __forceinline__ double planck_lo(double x) {
  constexpr double c[12] = {
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
      -236364091.0 / 2730.0 / (620448401733239439360000.0 * 27.0)};
  const double x2 = x * x;
  double s = c[11];
#pragma unroll
  for (int k = 10; k >= 0; --k) s = s * x2 + c[k];
  return x2 * x * (1.0 / 3.0 - 0.125 * x + x2 * s);
}

// int_x^inf t^3/(e^t - 1) dt for x >= 1
__device__ __forceinline__ double planck_hi(double x) {
  if (!(x < 745.0)) return 0.0;
  const double e1 = exp(-x), x2 = x * x, x3 = x2 * x;
  double en = e1, s = 0.0;
  for (int n = 1; n <= 64; ++n) {
    const double in = 1.0 / n;
    const double term = en * in * (x3 + in * (3.0 * x2 + in * (6.0 * x + 6.0 * in)));
    s += term;
    if (term <= 1e-17 * s) break;
    en *= e1;
  }
  return s;
}

// D(a, b) = int_a^b x^3/(e^x - 1) dx, 0 <= a < b (b may be +inf)
__device__ double planck_bin(double a, double b) {
  if (b <= 1.0) return planck_lo(b) - planck_lo(a);
  if (a >= 1.0) return planck_hi(a) - planck_hi(b);
  return (planck_lo(1.0) - planck_lo(a)) + (planck_hi(1.0) - planck_hi(b));
}

// x^4/(e^x - 1), 0 at x = 0 and as x -> inf
__device__ __forceinline__ double planck_x4(double x) {
  if (!(x > 0.0) || !(x < 745.0)) return 0.0;
  const double x2 = x * x;
  return x2 * x2 / expm1(x);
}

__global__ void __launch_bounds__(256)
k_mg_solve(MgArgs a, const double* __restrict__ Emg, const double* __restrict__ rho,
           const double* __restrict__ kag, const double* __restrict__ ks, const double* T_start,
           double* T_out, double* __restrict__ map, unsigned long long* __restrict__ fail) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nc = a.nc;
  if (c >= nc) return;
  const double r = rho[c], T0 = T_start[c];
  const bool live = r >= a.rho_floor;
  const double as = (live && ks) ? r * ks[c] : 0.0;
  const double Y = r / (a.gamma - 1.0);
  const double A2f = a.h * a.W0 / (4.0 * kPi);
  // F(T) and F'(T); the per-bin terms are recomputed (a handful of flops) to
  // keep registers independent of the number of bins
  auto eval = [&](double T, double& F, double& dF) {
    F = Y * (T - T0);
    dF = Y;
    const double iT = 1.0 / T, T3 = T * T * T, T4 = T3 * T;
    for (int g = 0; g < a.ng; ++g) {
      const double aa = r * kag[g * nc + c], den = 1.0 + (aa + as) * a.h;
      const double Em = Emg[g * nc + c], A1 = Em / den, A2 = A2f / den, q = 1.0 - as * A2;
      const double xl = a.nu[g] * iT, xh = a.nu[g + 1] * iT;
      const double D = planck_bin(xl, xh);
      const double S = aa * kPlanckC * T4 * D;
      const double dS = aa * kPlanckC * T3 * (4.0 * D - planck_x4(xh) + planck_x4(xl));
      F += (A1 + A2 * S) / q - Em;
      dF += A2 * dS / q;
    }
  };
  double Tp = T0;
  bool ok = false;
  if (live) {
    double excess = 0.0;
    for (int g = 0; g < a.ng; ++g) {
      const double aa = r * kag[g * nc + c], den = 1.0 + (aa + as) * a.h;
      const double Em = Emg[g * nc + c], q = 1.0 - as * A2f / den;
      excess += Em - Em / den / q;
    }
    double lo = 0.0, hi = T0 + excess / Y;
    if (Y > 0.0 && T0 > 0.0 && hi > 0.0) {
      double x = (T0 > 0.0 && T0 < hi) ? T0 : 0.5 * hi;
      const int iters = max(a.max_iter, 120);
      for (int it = 0; it < iters; ++it) {
        double F, dF;
        eval(x, F, dF);
        if (F > 0.0) hi = x;
        else lo = x;
        double xn = x - F / dF;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const double dx = xn - x;
        x = xn;
        if (fabs(dx) <= a.rtol * x || hi - lo <= a.rtol * x) {
          ok = true;
          break;
        }
      }
      Tp = x;
    }
    if (!ok && fail) atomicAdd(fail, 1ull);
  }
  T_out[c] = ok ? Tp : T0;
  const double iT = ok ? 1.0 / Tp : 0.0, T4 = Tp * Tp * Tp * Tp;
  for (int g = 0; g < a.ng; ++g) {
    double al = 1.0, be = 0.0;
    if (ok) {
      const double aa = r * kag[g * nc + c], den = 1.0 + (aa + as) * a.h;
      const double Em = Emg[g * nc + c], A1 = Em / den, A2 = A2f / den, q = 1.0 - as * A2;
      const double S = aa * kPlanckC * T4 * planck_bin(a.nu[g] * iT, a.nu[g + 1] * iT);
      const double Ep = (A1 + A2 * S) / q;
      al = 1.0 / den;
      be = a.h * (S + as * Ep) / (4.0 * kPi * den);
    }
    map[2 * g * nc + c] = al;
    map[(2 * g + 1) * nc + c] = be;
  }
}

}  // namespace

hipError_t launch_mg_solve(rt_ctx* c, double h, const double* Emg, const double* T_start, double* T_out,
                           double* map, hipStream_t st) {
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
  hipLaunchKernelGGL(k_mg_solve, grid, block, 0, st, a, Emg, c->d_rho, c->d_ka_g, c->d_ks, T_start, T_out,
                     map, c->d_count);
  return hipGetLastError();
}

}  // namespace rt
