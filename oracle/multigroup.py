"""Multi-group (frequency-binned) transport for a fluid at rest in flat space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The finite-volume equation integrated over a frequency bin (Sec. 3.1, Eq.
radiative_transfer_discrete_non_gray) adds to the gray one a flux through the
bin's frequency boundaries, carried by r^nu.  The paper leaves frequency
dependent transport to future work and gives no r^nu; the reading taken here
is the case where it vanishes identically: a fluid at rest in flat space,
where the fluid-frame frequency of a photon is the same everywhere along its
path.  Then:

  * I_gs = the intensity of direction s integrated over bin g
    [nu_g, nu_(g+1)) of fluid-frame frequency (the last edge may be +inf);
    summed over bins it is the gray intensity;
  * every bin is transported as the gray equation (Sec. 3.4-3.5) with its own
    optical depth tau_g = abar (alpha_g,l + alpha_g,l+1)/2 dt, alpha_g =
    alpha^a_g + alpha^s;
  * the bins couple only through the gas temperature.  Absorption is
    alpha^a_g = rho kappa_a,g (per cell and bin, constant in time), emission
    follows Kirchhoff's law with the bin-integrated Planck function B_g(T),
    and scattering (alpha^s = rho kappa_s) is isotropic and elastic, so it
    stays inside the bin;
  * units of Sec. 4.11 (a_rad = k_B = 1; frequency in units of k_B/h):
    B_nu(T) = 15/(4 pi^5) nu^3/(exp(nu/T) - 1), whose integral over all
    frequencies is T^4/(4 pi), the gray B(T).

The implicit interaction is Method 1's (Sec. 3.6.2, Eq. fluid_interaction_
discrete, Eq. semi_implicit_T) in every bin, with the emission taken at T_+:
  I+_gs = c_g I~_gs + d_g (S_g + alpha^s E+_g),   S_g = 4 pi alpha^a_g B_g(T_+),
  c_g = 1/(1 + alpha_g h),  d_g = h/(4 pi (1 + alpha_g h)),
  E+_g = (A1_g + A2_g S_g)/q_g,  A1_g = c_g E-_g,  A2_g = d_g sum_s w_s,
  q_g = 1 - alpha^s A2_g,
  Y (T_+ - T_-) = -sum_g (E+_g - E-_g)     (Eq. ideal_gas_difference).
With one bin [0, inf) this is Method 1 exactly.  The temperature equation
  F(T) = Y (T - T_-) + sum_g ((A1_g + A2_g S_g(T))/q_g - E-_g) = 0
has F increasing in T, F(0) < 0 and F(T_hi) >= 0 at
T_hi = T_- + sum_g (E-_g - A1_g/q_g)/Y, so its root is unique; the oracle
finds it by bisection.
"""
import math

import numpy as np
import torch

from . import transport as tr
from .step import moments

F64 = torch.float64
PLANCK_NORM = 15.0 / math.pi ** 4     # int_0^inf x^3/(e^x - 1) dx = pi^4/15
_GL_X, _GL_W = np.polynomial.legendre.leggauss(32)
_PANELS = 10
_X_TAIL = 150.0                       # beyond x_lo + 150 the integrand is < e^-140 of its value at x_lo


def planck_x3_integral(x_lo, x_hi):
    """int_{x_lo}^{x_hi} x^3/(e^x - 1) dx, elementwise over arrays of bounds
    (x_hi may be +inf), by Gauss-Legendre quadrature (32 nodes) on 10 equal
    panels of [x_lo, min(x_hi, x_lo + 150)]."""
    x_lo = np.asarray(x_lo, dtype=np.float64)
    x_hi = np.minimum(np.asarray(x_hi, dtype=np.float64), x_lo + _X_TAIL)
    width = (x_hi - x_lo) / _PANELS
    total = np.zeros(np.broadcast(x_lo, x_hi).shape)
    for k in range(_PANELS):
        a = x_lo + k * width
        x = a[..., None] + 0.5 * width[..., None] * (_GL_X + 1.0)
        f = np.where(x > 0, x ** 3 / np.expm1(np.where(x > 0, x, 1.0)), 0.0)
        total = total + 0.5 * width * (f * _GL_W).sum(-1)
    return total


def planck_group(T, nu_lo, nu_hi):
    """B_g(T) = int_{nu_lo}^{nu_hi} B_nu(T) dnu = T^4/(4 pi) * 15/pi^4 *
    int_{nu_lo/T}^{nu_hi/T} x^3/(e^x - 1) dx (T > 0; array T, scalar edges)."""
    Tn = np.asarray(T, dtype=np.float64)
    frac = PLANCK_NORM * planck_x3_integral(nu_lo / Tn, nu_hi / Tn)
    return Tn ** 4 / (4.0 * math.pi) * frac


def interact_mg(It, T_start, rho, ka, ks, w, h, gamma, edges, rho_floor, iters=80):
    """Implicit interaction of all bins.  It [G, Ns, *cells]; ka [G, *cells]
    (kappa_a per bin), ks, rho, T_start [*cells]; w [Ns]; edges [G + 1].
    Returns (I_out, T_out, failed)."""
    G = It.shape[0]
    w = torch.as_tensor(w, dtype=F64)
    W0 = float(w.sum())
    live = rho >= rho_floor
    zero = torch.zeros_like(rho)
    as_ = torch.where(live, rho * ks, zero)
    aa = [torch.where(live, rho * ka[g], zero) for g in range(G)]
    Em = [torch.tensordot(w, It[g], dims=1) for g in range(G)]
    cg = [1.0 / (1.0 + (aa[g] + as_) * h) for g in range(G)]
    dg = [h / (4.0 * math.pi * (1.0 + (aa[g] + as_) * h)) for g in range(G)]
    A1 = [cg[g] * Em[g] for g in range(G)]
    A2 = [dg[g] * W0 for g in range(G)]
    q = [1.0 - as_ * A2[g] for g in range(G)]
    Y = rho / (gamma - 1.0)
    Ts = T_start.numpy()

    def S(g, T):
        return aa[g] * 4.0 * math.pi * torch.as_tensor(planck_group(T, edges[g], edges[g + 1]))

    def F(T):
        Tt = torch.as_tensor(T)
        out = Y * (Tt - T_start)
        for g in range(G):
            out = out + (A1[g] + A2[g] * S(g, T)) / q[g] - Em[g]
        return out

    hi = T_start + sum((Em[g] - A1[g] / q[g]) for g in range(G)) / torch.where(live, Y, torch.ones_like(Y))
    ok = live & (Y > 0) & (T_start > 0) & (hi > 0)
    lo_np = np.zeros_like(Ts)
    hi_np = torch.where(ok, hi, torch.ones_like(hi)).numpy().copy()
    for _ in range(iters):
        mid = 0.5 * (lo_np + hi_np)
        Fm = F(np.maximum(mid, 1e-300)).numpy()
        pos = Fm > 0
        hi_np = np.where(pos, mid, hi_np)
        lo_np = np.where(pos, lo_np, mid)
    Tp = torch.as_tensor(0.5 * (lo_np + hi_np))
    Tp = torch.where(ok, Tp, T_start)
    Iout = torch.empty_like(It)
    for g in range(G):
        Sg = S(g, np.maximum(Tp.numpy(), 1e-300))
        Ep = (A1[g] + A2[g] * Sg) / q[g]
        Ig = cg[g] * It[g] + dg[g] * (Sg + as_ * Ep)
        Iout[g] = torch.where(ok, Ig, It[g])
    Tout = torch.where(ok, Tp, T_start)
    return Iout, Tout, live & ~ok


def step_mg(pb, ka, edges, I, T, dt):
    """Predictor-corrector step (Sec. 3.7) of all bins: stage 1 transports every
    bin by dt/2 from I^n and applies the interaction from T^n; stage 2
    transports by dt with the fluxes of I*, from I^n, and applies the
    interaction from T^n again.  pb is a flat, at-rest Problem (its kappa_s and
    rho are used; its kappa_a is ignored), ka [G, *cells].  Returns
    (I^(n+1), T^(n+1))."""
    g = pb.geo.grid
    ks = pb.kappa_s if pb.kappa_s is not None else pb.zeros()
    G = I.shape[0]

    def stage(I_flux, I_base, h):
        It = torch.empty_like(I)
        for k in range(G):
            live = pb.rho >= pb.rho_floor
            ah = torch.where(live, pb.rho * (ka[k] + ks), pb.zeros())
            It[k] = tr.transport(I_flux[k], I_base[k], h, dt, pb.geo, ah, pb.v, pb.abar,
                                 pb.bc_lo, pb.bc_hi, pb.limiter)
        return It

    It1 = stage(I, I, 0.5 * dt)
    Is, Ts, f1 = interact_mg(It1, T, pb.rho, ka, ks, g.w, 0.5 * dt, pb.gamma, edges, pb.rho_floor)
    It2 = stage(Is, I, dt)
    In, Tn, f2 = interact_mg(It2, T, pb.rho, ka, ks, g.w, dt, pb.gamma, edges, pb.rho_floor)
    pb.failed.append(int(f1.sum()) + int(f2.sum()))
    return In, Tn, It2


def moments_mg(I, nhat, w):
    """R-hat^(ab) of the radiation summed over bins (Eq. R), [10, *cells]."""
    return moments(I.sum(0), nhat, w)
