// Hand-written adjoint of one predictor-corrector step for a fluid at rest
// with a fixed emissivity (temperature-independent opacities): gradients with
// respect to the intensity of the step start, the per-cell absorption opacity
// kappa_a and the emissivity j.
//
// Forward (per stage, h = dt/2 then dt; tau uses the full dt in both stages):
//   I~ = I_base - h D(I_flux),  D = sum_a (F(l+1/2) - F(l-1/2)) / dx_a,
//   F  = nu (P I_l + Q I_l+1 + U2 hL - V2 hR)   (nu > 0; mirrored for nu < 0)
//   with hL, hR the half limited slopes and P, Q, U2, V2 functions of tau;
//   I_out = c I~ + d Q,  c = 1/(1 + alpha h),  d = h c/(4 pi),
//   Q = S + alpha^s E+,  E+ = (c E- + A2 S)/q,  E- = sum_s w_s I~_s,
//   A2 = d sum_s w_s,  q = 1 - A2 alpha^s,  S = 4 pi j,  alpha = rho (kappa_a + kappa_s).
// Reverse: the interaction adjoint per cell, then the transport adjoint in
// gather form (each cell collects the flux-derivative contributions of the
// faces whose stencils contain it), then the tau-gradients of the faces are
// reduced onto the cells' opacities.  No floating-point atomics: every sum has
// one writer and a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ctx.hpp"
#include "stage.hpp"

namespace rt {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ int wrapc(int i, int n, bool periodic) {
  if (periodic) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// flux weights of a face and their derivatives with respect to tau
struct Wts {
  double P, Q, U2, V2;     // F = nu (P IcL + Q IcR + U2 hL - V2 hR)
  double dP, dQ, dU2, dV2; // d/dtau
};

__device__ Wts weights(double tau) {
  const double E = exp(-tau), dE = -E;
  double f2, f4, d2, d4;
  if (tau < 1e-4) {
    const double t2 = tau * tau;
    f2 = 1.0 - 0.25 * t2;
    f4 = tau * (1.0 - 0.25 * t2 * t2);
    d2 = -0.5 * tau;
    d4 = 1.0 - 1.25 * t2 * t2;
  } else {
    const double t2 = tau * tau, t4 = t2 * t2;
    const double g = -expm1(-t2), k = -expm1(-t4);
    const double sg = sqrt(g), sk = sqrt(k);
    f2 = sg / tau;
    f4 = sk / tau;
    // d/dtau sqrt(1 - e^{-tau^2})/tau and sqrt(1 - e^{-tau^4})/tau
    d2 = exp(-t2) / sg - sg / t2;
    d4 = 2.0 * t2 * exp(-t4) / sk - sk / t2;
  }
  const double Sm = f2 + f4, Sm2 = Sm * Sm;
  const double Wu = f2 / Sm, Wd = f4 / Sm, Dc = f2 * f4 / Sm;
  const double dWu = (d2 * f4 - f2 * d4) / Sm2;
  const double dDc = (d2 * f4 * f4 + f2 * f2 * d4) / Sm2;
  Wts w;
  w.P = E * Wu + Dc;
  w.Q = E * Wd - Dc;
  w.U2 = E * Wu;
  w.V2 = E * Wd;
  w.dP = dE * Wu + E * dWu + dDc;
  w.dQ = dE * Wd - E * dWu - dDc;
  w.dU2 = dE * Wu + E * dWu;
  w.dV2 = dE * Wd - E * dWu;
  return w;
}

// half of the limited slope and its partial derivatives (the active branch)
template <int LIM>
__device__ __forceinline__ double hslope(double p, double q, double& dp, double& dq) {
  dp = dq = 0.0;
  if (!(p * q > 0.0)) return 0.0;
  if (LIM == RT_LIM_MC) {
    const double ap = fabs(p), aq = fabs(q), as = 0.25 * fabs(p + q);
    if (ap <= aq && ap <= as) {
      dp = 1.0;
      return p;
    }
    if (aq <= as) {
      dq = 1.0;
      return q;
    }
    dp = dq = 0.25;
    return 0.25 * (p + q);
  }
  if (fabs(p) <= fabs(q)) {
    dp = 0.5;
    return 0.5 * p;
  }
  dq = 0.5;
  return 0.5 * q;
}

struct AdjArgs {
  int n[3];
  long long nc;
  int ns;
  int bc_lo[3], bc_hi[3];
  double inv_dx[3];
  double h, dt, abar, rho_floor, W0;
};

__device__ __forceinline__ void cell_opac(const AdjArgs& a, const double* rho, const double* ka,
                                          const double* ks, long long c, double& r, double& aa,
                                          double& as) {
  r = rho[c];
  aa = ka ? r * ka[c] : 0.0;
  as = ks ? r * ks[c] : 0.0;
  if (!(r >= a.rho_floor)) aa = as = 0.0;
}

// ---------------------------------------------------------------------------
// interaction adjoint, one thread per cell: gIt = dL/dI~ from gI = dL/dI_out;
// adds dL/dkappa_a and dL/dj of this interaction
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256)
k_src_adj(AdjArgs a, const S* __restrict__ It, const S* gI, S* gIt, const double* __restrict__ rho,
          const double* __restrict__ ka, const double* __restrict__ ks,
          const double* __restrict__ jv, const double* __restrict__ w, double* __restrict__ gka,
          double* __restrict__ gj) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.nc) return;
  double r, aa, as;
  cell_opac(a, rho, ka, ks, c, r, aa, as);
  if (!(r >= a.rho_floor)) {
    for (int s = 0; s < a.ns; ++s) gIt[(long long)s * a.nc + c] = gI[(long long)s * a.nc + c];
    return;
  }
  const double h = a.h, ab = aa + as;
  const double cc = 1.0 / (1.0 + ab * h);
  const double dd = h * cc / (4.0 * kPi);
  const double A2 = dd * a.W0;
  const double q = 1.0 - A2 * as;
  const double Se = 4.0 * kPi * (jv ? jv[c] : 0.0);
  double Em = 0.0, G = 0.0, GI = 0.0;
  for (int s = 0; s < a.ns; ++s) {
    const double x = (double)It[(long long)s * a.nc + c], g = (double)gI[(long long)s * a.nc + c];
    Em += w[s] * x;
    G += g;
    GI += g * x;
  }
  const double Ep = (cc * Em + A2 * Se) / q;
  const double Q = Se + as * Ep;
  // dL/dI~_s = c g_s + (G d alpha^s c / q) w_s
  const double kw = G * dd * as * cc / q;
  for (int s = 0; s < a.ns; ++s) {
    const long long i = (long long)s * a.nc + c;
    gIt[i] = (S)(cc * (double)gI[i] + kw * w[s]);
  }
  // parameter derivatives through alpha = rho (kappa_a + kappa_s) and S = 4 pi j
  const double dc = -h * cc * cc;
  const double ddd = h * dc / (4.0 * kPi);
  const double dA2 = ddd * a.W0;
  const double dq = -as * dA2;
  const double dEp = (dc * Em + dA2 * Se) / q - Ep * dq / q;
  const double dQ = as * dEp;
  const double galpha = dc * GI + (ddd * Q + dd * dQ) * G;
  if (gka) gka[c] += r * galpha;
  if (gj) gj[c] += 4.0 * kPi * dd * (1.0 + as * A2 / q) * G;
}

// ---------------------------------------------------------------------------
// transport adjoint (gather form), one thread per cell, all directions:
//   out = add0 + add1 - h * D^T(gIt)  evaluated at the forward I_flux,
// and the per-face sums dL/dtau_f = sum_s gF_f,s dF_f,s/dtau (stored per face:
// the lower face of each cell, plus the upper boundary face of the last cell
// of non-periodic axes, which is face index n of that axis).
// ---------------------------------------------------------------------------
template <typename S, int LIM>
__global__ void __launch_bounds__(256)
k_tr_adj(AdjArgs a, const S* __restrict__ If, const S* __restrict__ gIt, const S* add0,
         const S* add1, S* out, const double* __restrict__ dir, const double* __restrict__ rho,
         const double* __restrict__ ka, const double* __restrict__ ks, double* __restrict__ gtau) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.nc) return;
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int ii[3] = {(int)(c / ((long long)n2 * n3)), (int)((c / n3) % n2), (int)(c % n3)};
  const long long st[3] = {(long long)n2 * n3, n3, 1};
  auto alpha_hat = [&](long long cell) {
    double r, aa, as;
    cell_opac(a, rho, ka, ks, cell, r, aa, as);
    return aa + as;  // fluid at rest: u-hat^0 = 1
  };
  // per axis: the faces f = m-1 .. m+2 (lower-face index, f in [0, n]) that can
  // hold this cell in their stencil, with their weights; the thread owns the
  // tau-gradient of its lower face (and of face n when it is the last cell)
  double taug[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  for (int s = 0; s < a.ns; ++s) {
    const long long off = (long long)s * a.nc;
    double acc = 0.0;
    if (add0) acc += (double)add0[off + c];
    if (add1) acc += (double)add1[off + c];
    for (int ax = 0; ax < 3; ++ax) {
      const int na = ax == 0 ? n1 : (ax == 1 ? n2 : n3);
      const int m = ii[ax];
      const bool per = a.bc_lo[ax] == RT_BC_PERIODIC;
      const double nu = dir[ax * a.ns + s];
      const bool pos = nu > 0.0;
      const long long base = c - (long long)m * st[ax];
      // forward value at (possibly ghost) position p along the axis
      auto val = [&](int p) -> double {
        if (!per) {
          if (p < 0 && a.bc_lo[ax] == RT_BC_ZERO_INCOMING && nu > 0.0) return 0.0;
          if (p >= na && a.bc_hi[ax] == RT_BC_ZERO_INCOMING && nu < 0.0) return 0.0;
        }
        return (double)If[off + base + (long long)wrapc(p, na, per) * st[ax]];
      };
      // does position p feed this cell (m)?  zeroed ghosts feed nothing
      auto feeds = [&](int p) -> bool {
        if (!per) {
          if (p < 0 && a.bc_lo[ax] == RT_BC_ZERO_INCOMING && nu > 0.0) return false;
          if (p >= na && a.bc_hi[ax] == RT_BC_ZERO_INCOMING && nu < 0.0) return false;
        }
        return wrapc(p, na, per) == m;
      };
      auto gcell = [&](int p) -> double {  // dL/dI~ at cell p; ghosts are not updated
        if (!per && (p < 0 || p >= na)) return 0.0;
        return (double)gIt[off + base + (long long)wrapc(p, na, per) * st[ax]];
      };
      const int nfaces = per ? na : na + 1;
      int seen[4];
      int nseen = 0;
      for (int k = -1; k <= 2; ++k) {
        int f = m + k;
        if (per) f = wrapc(f, na, true);
        if (f < 0 || f >= nfaces) continue;
        bool dup = false;
        for (int u = 0; u < nseen; ++u) dup |= seen[u] == f;
        if (dup) continue;
        seen[nseen++] = f;
        // stencil positions of face f (between cells f-1 and f); for periodic
        // axes use the unwrapped positions nearest to m
        const int p0 = f - 2;  // stencil positions p0 .. p0+3 (wrapped or clamped on use)
        const double v0 = val(p0), v1 = val(p0 + 1), v2 = val(p0 + 2), v3 = val(p0 + 3);
        const int L = p0 + 1, R = p0 + 2;  // cells either side of the face
        const double gF = (gcell(R) - gcell(L)) * a.inv_dx[ax] * a.h;
        if (gF == 0.0) continue;
        // weights of this face
        const long long cl = base + (long long)wrapc(L, na, per) * st[ax];
        const long long cr = base + (long long)wrapc(R, na, per) * st[ax];
        const double tau = a.abar * 0.5 * (alpha_hat(cl) + alpha_hat(cr)) * a.dt;
        const Wts W = weights(tau);
        const double cP = pos ? W.P : W.Q, cQ = pos ? W.Q : W.P;
        const double cU = pos ? W.U2 : W.V2, cV = pos ? W.V2 : W.U2;
        double a0, a1, b1, b2;
        const double hL = hslope<LIM>(v1 - v0, v2 - v1, a0, a1);
        const double hR = hslope<LIM>(v2 - v1, v3 - v2, b1, b2);
        // dF/d(positions p0..p0+3)
        const double g0 = nu * (-cU * a0);
        const double g1 = nu * (cP + cU * (a0 - a1) + cV * b1);
        const double g2 = nu * (cQ + cU * a1 - cV * (b1 - b2));
        const double g3 = nu * (-cV * b2);
        double contrib = 0.0;
        if (feeds(p0)) contrib += g0;
        if (feeds(p0 + 1)) contrib += g1;
        if (feeds(p0 + 2)) contrib += g2;
        if (feeds(p0 + 3)) contrib += g3;
        // F contributes -h F/dx to I~(L) and +h F/dx to I~(R): dL/dF = gF
        acc += gF * contrib;
        // tau-gradient of the faces this thread owns
        const int slot = f == m ? 0 : ((!per && m == na - 1 && f == na) ? 1 : -1);
        if (slot >= 0) {
          const double dcP = pos ? W.dP : W.dQ, dcQ = pos ? W.dQ : W.dP;
          const double dcU = pos ? W.dU2 : W.dV2, dcV = pos ? W.dV2 : W.dU2;
          const double dFdt = nu * (dcP * v1 + dcQ * v2 + dcU * hL - dcV * hR);
          taug[ax][slot] += gF * dFdt;
        }
      }
    }
    out[off + c] = (S)acc;
  }
  // store per-face tau gradients: axis ax, lower face of this cell, and face n
  for (int ax = 0; ax < 3; ++ax) {
    gtau[(long long)ax * 2 * a.nc + c] = taug[ax][0];
    gtau[(long long)ax * 2 * a.nc + a.nc + c] = taug[ax][1];
  }
}

// ---------------------------------------------------------------------------
// tau_f = abar (alpha-hat_L + alpha-hat_R)/2 dt: dL/dalpha-hat of a cell sums
// abar dt / 2 times the tau-gradient of every face that uses it (its own lower
// and upper faces, and, for clamped ghosts, the boundary faces where it stands
// in for the ghost); dL/dkappa_a = rho dL/dalpha-hat.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_tau_to_kappa(AdjArgs a, const double* __restrict__ gtau, const double* __restrict__ rho,
               double* __restrict__ gka) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.nc) return;
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int ii[3] = {(int)(c / ((long long)n2 * n3)), (int)((c / n3) % n2), (int)(c % n3)};
  const long long st[3] = {(long long)n2 * n3, n3, 1};
  double g = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const int na = ax == 0 ? n1 : (ax == 1 ? n2 : n3);
    const int m = ii[ax];
    const bool per = a.bc_lo[ax] == RT_BC_PERIODIC;
    const long long base = c - (long long)m * st[ax];
    const double* lower = gtau + (long long)ax * 2 * a.nc;  // lower face of each cell
    const double* upper = lower + a.nc;                      // face n, held by the last cell
    // face between m-1 and m (lower face of m): uses m once as its right cell,
    // and twice when m = 0 on a clamped axis (the ghost is a copy of m)
    double gl = lower[c];
    double gu;  // face between m and m+1
    if (m + 1 < na)
      gu = lower[base + (long long)(m + 1) * st[ax]];
    else
      gu = per ? lower[base] : upper[c];
    g += gl + gu;
    if (!per && m == 0) g += gl;       // left ghost copies cell 0
    if (!per && m == na - 1) g += gu;  // right ghost copies cell n-1
  }
  const double r = rho[c];
  if (r >= a.rho_floor) gka[c] += r * 0.5 * a.abar * a.dt * g;
}

template <typename S>
__global__ void __launch_bounds__(256)
k_apply_map(long long nc, int ns, const double* __restrict__ map, const S* __restrict__ in,
            S* __restrict__ out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double al = map[c], be = map[nc + c];
  for (int s = 0; s < ns; ++s) {
    const long long i = (long long)s * nc + c;
    out[i] = (S)(al * (double)in[i] + be);
  }
}

}  // namespace

hipError_t launch_adjoint_step(rt_ctx* c, const void* I_n, const double* T_n, double dt,
                               const void* gI_np1, void* gI_n, double* g_ka, double* g_j,
                               hipStream_t st) {
  // ---- forward recompute: X = I~ of stage 1, Y = I*, Z = I~ of stage 2
  StageArgs sa{};
  sa.n1 = c->n[0];
  sa.n2 = c->n[1];
  sa.n3 = c->n[2];
  sa.nc = c->nc;
  sa.ns = c->ns;
  for (int ax = 0; ax < 3; ++ax) {
    sa.bc_lo[ax] = c->desc.bc_lo[ax];
    sa.bc_hi[ax] = c->desc.bc_hi[ax];
    sa.inv_dx[ax] = 1.0 / c->dx[ax];
  }
  sa.dt = dt;
  sa.abar = c->desc.abar;
  sa.limiter = c->desc.limiter;
  sa.model = c->opac.model;
  sa.gamma = c->opac.gamma;
  sa.C_a = c->opac.C_a;
  sa.C_s = c->opac.C_s;
  sa.rho_floor = c->desc.rho_floor;
  sa.max_iter = c->opac.newton_max_iter;
  sa.rtol = c->opac.newton_rtol;
  sa.W0 = c->W0;
  for (int k = 0; k < 10; ++k) sa.Wsum[k] = c->Wsum[k];
  StagePtrs p{};
  p.rho = c->d_rho;
  p.ka = c->d_ka;
  p.ks = c->d_ks;
  p.jv = c->d_j;
  p.uhat = c->d_uhat;
  p.vel = c->d_v;
  p.dirF_v = c->fp32 ? (const void*)c->d_dir_f : (const void*)c->d_dir;
  p.dirD = c->d_dir;
  p.w = c->d_w;
  p.W16 = c->d_W16;
  p.fail = c->d_count;
  // the temperature is unchanged in this model (T_out goes to scratch)
  void* X = c->d_Itil;
  void* Y = c->d_gC;
  void* Z = c->d_gD;
  sa.h = 0.5 * dt;
  p.Iflux_v = I_n;
  p.mapF = nullptr;
  p.Iout_v = X;
  p.mapO = c->d_mapB;
  p.Tstart = T_n;
  p.Tcoef = T_n;
  p.Tout = c->d_Tstar;
  hipError_t e = launch_stage(c, sa, p, false, st);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((c->nc + 255) / 256)), block(256);
  if (c->fp32)
    hipLaunchKernelGGL(k_apply_map<float>, grid, block, 0, st, c->nc, c->ns, c->d_mapB,
                       (const float*)X, (float*)Y);
  else
    hipLaunchKernelGGL(k_apply_map<double>, grid, block, 0, st, c->nc, c->ns, c->d_mapB,
                       (const double*)X, (double*)Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sa.h = dt;
  p.Iflux_v = Y;
  p.mapF = nullptr;
  p.Ibase_v = I_n;
  p.mapB = nullptr;
  p.Iout_v = Z;
  p.mapO = c->d_mapA;
  e = launch_stage(c, sa, p, true, st);
  if (e != hipSuccess) return e;

  // ---- reverse
  AdjArgs a{};
  for (int ax = 0; ax < 3; ++ax) {
    a.n[ax] = c->n[ax];
    a.bc_lo[ax] = c->desc.bc_lo[ax];
    a.bc_hi[ax] = c->desc.bc_hi[ax];
    a.inv_dx[ax] = 1.0 / c->dx[ax];
  }
  a.nc = c->nc;
  a.ns = c->ns;
  a.dt = dt;
  a.abar = c->desc.abar;
  a.rho_floor = c->desc.rho_floor;
  a.W0 = c->W0;
  const bool mc = c->desc.limiter == RT_LIM_MC;
  void* gA = c->d_gA;  // dL/dI~ of stage 2 (also the base contribution to dL/dI^n)
  void* gB = c->d_gB;  // dL/dI*, then dL/dI~ of stage 1
#define RT_ADJ_LAUNCH(S)                                                                            \
  do {                                                                                              \
    a.h = dt;                                                                                       \
    hipLaunchKernelGGL(k_src_adj<S>, grid, block, 0, st, a, (const S*)Z, (const S*)gI_np1, (S*)gA, \
                       c->d_rho, c->d_ka, c->d_ks, c->d_j, c->d_w, g_ka, g_j);                     \
    if (mc)                                                                                         \
      hipLaunchKernelGGL((k_tr_adj<S, RT_LIM_MC>), grid, block, 0, st, a, (const S*)Y,             \
                         (const S*)gA, (const S*)nullptr, (const S*)nullptr, (S*)gB, c->d_dir,     \
                         c->d_rho, c->d_ka, c->d_ks, c->d_gcell);                                  \
    else                                                                                            \
      hipLaunchKernelGGL((k_tr_adj<S, RT_LIM_MINMOD>), grid, block, 0, st, a, (const S*)Y,         \
                         (const S*)gA, (const S*)nullptr, (const S*)nullptr, (S*)gB, c->d_dir,     \
                         c->d_rho, c->d_ka, c->d_ks, c->d_gcell);                                  \
    if (g_ka)                                                                                       \
      hipLaunchKernelGGL(k_tau_to_kappa, grid, block, 0, st, a, c->d_gcell, c->d_rho, g_ka);       \
    a.h = 0.5 * dt;                                                                                 \
    hipLaunchKernelGGL(k_src_adj<S>, grid, block, 0, st, a, (const S*)X, (const S*)gB, (S*)gB,     \
                       c->d_rho, c->d_ka, c->d_ks, c->d_j, c->d_w, g_ka, g_j);                     \
    if (mc)                                                                                         \
      hipLaunchKernelGGL((k_tr_adj<S, RT_LIM_MC>), grid, block, 0, st, a, (const S*)I_n,           \
                         (const S*)gB, (const S*)gA, (const S*)gB, (S*)gI_n, c->d_dir, c->d_rho,   \
                         c->d_ka, c->d_ks, c->d_gcell);                                            \
    else                                                                                            \
      hipLaunchKernelGGL((k_tr_adj<S, RT_LIM_MINMOD>), grid, block, 0, st, a, (const S*)I_n,       \
                         (const S*)gB, (const S*)gA, (const S*)gB, (S*)gI_n, c->d_dir, c->d_rho,   \
                         c->d_ka, c->d_ks, c->d_gcell);                                            \
    if (g_ka)                                                                                       \
      hipLaunchKernelGGL(k_tau_to_kappa, grid, block, 0, st, a, c->d_gcell, c->d_rho, g_ka);       \
  } while (0)
  if (c->fp32)
    RT_ADJ_LAUNCH(float);
  else
    RT_ADJ_LAUNCH(double);
#undef RT_ADJ_LAUNCH
  return hipGetLastError();
}

}  // namespace rt
