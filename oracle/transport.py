"""Explicit transport sub-step: reconstruction, numerical fluxes, divergence.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows, in order:
  Sec. 3.4  piecewise-linear (PLI) reconstruction of I-hat at spatial faces,
            each direction separately, with a limited slope;
  Sec. 3.5  the spatial flux: vacuum upwind flux (Eq. spatial_fluxes_vacuum)
            and its modified signal-speed form (Eq. rad_speeds, Eq. flux_Jiang)
            with exponential cut-off, cell-centre diffusion term and
            advection term; the n_0 sign restriction;
  Sec. 3.1  the update of <n^0 n_0 I> by the flux divergence
            (Eq. radiative_transfer_discrete, gray form).

Readings of the printed flux (the paper's L/R labels, the extra n^i on the
diffusion term and the advection upwinding are garbled) are the ones listed in
the design notes: the upwind state carries the speed with the exp(-tau^2)
factor, the downwind state the one with exp(-tau^4) (so tau -> 0 gives the
vacuum upwind flux exactly), the diffusion term is -|n^a| S (I_(l+1) - I_l)
with no extra n^a, and the advection term is max(v_L,0) I_L + min(v_R,0) I_R.
tau = abar * (alpha-hat_l + alpha-hat_(l+1))/2 * dt is direction independent.
"""
import torch

PERIODIC, OUTFLOW, ZERO_INCOMING = 0, 1, 2
LIM_MC, LIM_MINMOD = 0, 1


def limited_slope(p, q, limiter):
    """Slope limiter for PLI.  MC: minmod(2p, 2q, (p+q)/2); minmod: minmod(p, q)."""
    if limiter == LIM_MC:
        m = torch.minimum(torch.minimum(2.0 * p.abs(), 2.0 * q.abs()), 0.5 * (p + q).abs())
    else:
        m = torch.minimum(p.abs(), q.abs())
    return torch.where(p * q > 0, torch.sign(p) * m, torch.zeros_like(p))


def speed_factors(tau):
    """f2 = sqrt(1-exp(-tau^2))/tau and f4 = sqrt(1-exp(-tau^4))/tau of Eq. rad_speeds
    (|S| = |n^a| f2 on the upwind side, |n^a| f4 on the other), with their
    tau -> 0 limits 1 and 0 (series below tau = 1e-4)."""
    small = tau < 1e-4
    ts = torch.where(small, torch.ones_like(tau), tau)
    f2 = torch.sqrt(-torch.expm1(-ts * ts)) / ts
    f4 = torch.sqrt(-torch.expm1(-(ts * ts) * (ts * ts))) / ts
    t2 = tau * tau
    f2 = torch.where(small, 1.0 - 0.25 * t2, f2)
    f4 = torch.where(small, tau * (1.0 - 0.25 * t2 * t2), f4)
    return f2, f4


def _wrap(x, lo):
    """The two cells that wrap around periodically below (lo) or above the line."""
    n = x.shape[-1]
    idx = [(n - 2) % n, (n - 1) % n] if lo else [0, 1 % n]
    return x[..., idx]


def _pad_cells(x, bc_lo, bc_hi):
    """Two ghost cells on each side of the last axis for a per-cell field:
    periodic wrap, otherwise a copy of the edge cell."""
    lo = _wrap(x, True) if bc_lo == PERIODIC else x[..., :1].expand(*x.shape[:-1], 2)
    hi = _wrap(x, False) if bc_hi == PERIODIC else x[..., -1:].expand(*x.shape[:-1], 2)
    return torch.cat([lo, x, hi], dim=-1)


def _pad_intensity(x, bc_lo, bc_hi, nu_lo, nu_hi):
    """Ghost cells for I-hat (Sec. 3.4 boundary handling): periodic wrap,
    outflow copy, or zero-incoming (zero where the boundary-face n^a points
    into the domain, a copy of the edge cell elsewhere)."""
    def side(bc, edge, wrap, incoming):
        if bc == PERIODIC:
            return wrap
        g = edge.expand(*edge.shape[:-1], 2)
        if bc == ZERO_INCOMING:
            g = torch.where(incoming, torch.zeros_like(g), g)
        return g
    lo = side(bc_lo, x[..., :1], _wrap(x, True), nu_lo > 0)
    hi = side(bc_hi, x[..., -1:], _wrap(x, False), nu_hi < 0)
    return torch.cat([lo, x, hi], dim=-1)


def face_fluxes(P, nu, n_low0_f, n_up0_f, tau, vL, vR, limiter):
    """Numerical flux F at the N+1 faces of a padded line P[..., N+4].

    F = n_0 * { e^-tau n^a (f2 I_up + f4 I_dn)/(f2 + f4)
                - |n^a| f2 f4/(f2 + f4) (I_(l+1) - I_l) }
        + (1 - e^-tau) n_0 n^0 (max(v_L,0) I_L + min(v_R,0) I_R)
    (Eq. flux_Jiang with the speeds of Eq. rad_speeds; tau = 0 gives the
    vacuum flux of Eq. spatial_fluxes_vacuum)."""
    n = P.shape[-1] - 4
    D = limited_slope(P[..., 1:n + 3] - P[..., 0:n + 2], P[..., 2:n + 4] - P[..., 1:n + 3], limiter)
    IL = P[..., 1:n + 2] + 0.5 * D[..., 0:n + 1]
    IR = P[..., 2:n + 3] - 0.5 * D[..., 1:n + 2]
    IcL = P[..., 1:n + 2]
    IcR = P[..., 2:n + 3]
    E = torch.exp(-tau)
    f2, f4 = speed_factors(tau)
    up = nu > 0
    Iup = torch.where(up, IL, IR)
    Idn = torch.where(up, IR, IL)
    Fr = E * nu * (f2 * Iup + f4 * Idn) / (f2 + f4) - nu.abs() * (f2 * f4 / (f2 + f4)) * (IcR - IcL)
    adv = (1.0 - E) * n_up0_f * (torch.clamp(vL, min=0.0) * IL + torch.clamp(vR, max=0.0) * IR)
    return n_low0_f * (Fr + adv)


def spatial_divergence(I, geo, alpha_hat, v, dt, abar, bc_lo, bc_hi, limiter):
    """(1/Delta V) sum_a [Delta A_a F_a]_(l-1/2)^(l+1/2) for every direction and cell
    (second term of Eq. radiative_transfer_discrete)."""
    div = torch.zeros_like(I)
    for a in range(3):
        X = I.movedim(1 + a, -1)
        nu = geo.face_nu(a).movedim(1 + a, -1)
        nl0 = geo.face_n_low0(a).movedim(1 + a, -1)
        nu0 = geo.face_n_up0(a).movedim(1 + a, -1)
        dA = geo.face_dA(a).movedim(a, -1)
        P = _pad_intensity(X, bc_lo[a], bc_hi[a], nu[..., :1], nu[..., -1:])
        al = _pad_cells(alpha_hat.movedim(a, -1), bc_lo[a], bc_hi[a])
        n = X.shape[-1]
        tau = abar * 0.5 * (al[..., 1:n + 2] + al[..., 2:n + 3]) * dt
        vp = _pad_cells(v[a].movedim(a, -1), bc_lo[a], bc_hi[a])
        Dv = limited_slope(vp[..., 1:n + 3] - vp[..., 0:n + 2], vp[..., 2:n + 4] - vp[..., 1:n + 3], limiter)
        vL = vp[..., 1:n + 2] + 0.5 * Dv[..., 0:n + 1]
        vR = vp[..., 2:n + 3] - 0.5 * Dv[..., 1:n + 2]
        F = face_fluxes(P, nu, nl0, nu0, tau, vL, vR, limiter)
        ok = geo.face_sign_ok(a, bc_lo[a] == PERIODIC) if hasattr(geo, "face_sign_ok") else None
        if ok is not None:
            # no flux between cells where n_0 changes sign (Sec. 3.5)
            F = torch.where(ok.movedim(1 + a, -1), F, torch.zeros_like(F))
        AF = dA * F
        div = div + (AF[..., 1:] - AF[..., :-1]).movedim(-1, 1 + a)
    return div / geo.dV()


def transport(I_flux, I_base, h, dt, geo, alpha_hat, v, abar, bc_lo, bc_hi, limiter,
              angular=None, n0_cut=None):
    """Explicit transport by h (Eq. radiative_transfer_discrete without the source):
    X = n^0 n_0 I;  X' = X(I_base) - h [spatial + angular flux divergence of I_flux];
    I~ = X' / (n^0 n_0).  Where |n_0| < n0_cut the intensity is zeroed (Sec. 3.5)."""
    n_up0 = geo.n_up0()
    n_low0 = geo.n_low0()
    X = n_up0 * n_low0 * I_base
    div = spatial_divergence(I_flux, geo, alpha_hat, v, dt, abar, bc_lo, bc_hi, limiter)
    if angular is not None:
        div = div + angular(I_flux)
    It = (X - h * div) / (n_up0 * n_low0)
    if n0_cut is not None:
        It = torch.where(n_low0.abs() < n0_cut, torch.zeros_like(It), It)
    return It
