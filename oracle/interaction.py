"""Implicit radiation-fluid interaction, paper Sec. 3.6.2.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Scale-free units of Sec. 4.11: c = G = a_rad = k_B/(mu m_p) = 1, so
B(T) = T^4/(4 pi) and Y = rho/(Gamma - 1).

Steps, in the paper's order, for every cell (vectorised over cells):
  1. density floor (Sec. 3.8): rho < rho_floor -> no interaction;
  2. boost to the fluid frame (Eq. fluid_to_coordinate, first row):
     nbar^0_s = u^0 - u.n_s,  Ibar_s = I_s (nbar^0_s)^4,
     dObar_s = w_s / (nbar^0_s)^2;
  3. explicit opacities at T_coef: alpha^a, alpha^s, alpha = alpha^a + alpha^s;
  4. A1, A2 (Eq. A1, Eq. A2) and Ebar_- (Eq. Ebar_calc);
  5. the temperature equation: Method 1 quartic (Eq. semi_implicit_T) or
     Method 2 (Eq. implicit_T, alpha_P^a = N T_+^(-7/2)), solved by Newton;
     Method 3 (Eq. T_almost_fully_implicit, the total opacity semi-implicit),
     solved by bisection; or a fixed emissivity (S_+ = 4 pi j, T unchanged);
  6. Ebar_+ from the energy balance (Eq. ideal_gas_difference);
  7. Ibar_+ from Eq. fluid_interaction_discrete (Method 3: with the factor
     alpha_-/alpha_+ of its rewritten A1', A2'), then back to the tetrad
     frame, I_+ = Ibar_+ / (nbar^0)^4.

Method 3, as read here.  Writing the implicit update of each direction as
  Ibar_+ = (1/(alpha dt)) [n^0/(n^0/(alpha dt) + nbar^0)] Ibar_-
         + (1/(alpha dt)) [nbar^0 dt/(4 pi (n^0/(alpha dt) + nbar^0))] S,
S = alpha_P^a T_+^4 + alpha^s Ebar_+, the method takes alpha_+ = alpha(T_+)
in the factor outside the brackets and alpha_- = alpha(T_coef) inside, so the
angular integrals are those of Methods 1-2 (A1, A2, computed once) and every
direction's update carries the factor r = alpha_-/alpha_+.  Integrated over
solid angle: Ebar_+ = r (A1 + A2 S).  With Ebar_+ = E0 - Y T_+
(Eq. ideal_gas_difference, E0 = Ebar_- + Y T_-) and the bremsstrahlung law
alpha^a = N T^-7/2 (so alpha_P^a T_+^4 = N sqrt(T_+)), multiplying by
alpha_+ T_+^3.5 dt gives the printed polynomial
  -Y alpha^s (dt - B2) T^4.5 - B2 N T^4 - [B2 alpha^s E0 + B1 - E0 alpha^s dt] T^3.5
  - Y N dt T + E0 N dt = 0
term by term when its A1', A2' are the bare integrals B1 = alpha_- dt A1,
B2 = alpha_- dt A2 (as printed, A1' and A2' also carry the prefactor
1/(alpha_+ dt), which would make the polynomial inconsistent).  The root
sought is the one with a non-negative gas energy, T_+ in (0, E0/Y), where
  F(T) = (E0 - Y T)(N T^-3.5 + alpha^s (1 - alpha_- A2)) - alpha_- (A1 + A2 N sqrt T)
is strictly decreasing from +inf to F(E0/Y) < 0: it is unique.
"""
import math
import torch

KIRCHHOFF_CONST, BREMS, FIXED_EMISSIVITY, BREMS_M3 = 0, 1, 2, 3


def opacities(model, rho, T, kappa_a, kappa_s, C_a, C_s, rho_floor):
    """Fluid-frame absorption and scattering coefficients alpha = rho kappa
    (Sec. 3.6.2).  Bremsstrahlung-like model: alpha^a = C_a rho^2 T^-7/2 times
    kappa_a, a per-cell dimensionless factor (1 when not given), alpha^s =
    C_s rho.  Zero below the density floor (Sec. 3.8)."""
    if model in (BREMS, BREMS_M3):
        aa = C_a * rho * rho * T.pow(-3.5) * kappa_a
        as_ = C_s * rho
    else:
        aa = rho * kappa_a
        as_ = rho * kappa_s
    live = rho >= rho_floor
    z = torch.zeros_like(rho)
    return torch.where(live, aa, z), torch.where(live, as_, z)


def newton_positive_root(a, b, K, p, max_iter=50, rtol=1e-14):
    """Positive root of a T^p + b T + K = 0 (a >= 0, b > 0, K < 0, p > 1).

    The function is convex and increasing on T > 0; starting from
    T0 = min(-K/b, (-K/a)^(1/p)), which lies above the root, Newton's
    iterates decrease monotonically to it (Sec. 3.6.2 solves the
    temperature equation with Newton-Raphson).  Returns (T, converged)."""
    T = -K / b
    T = torch.where(a > 0, torch.minimum(T, (-K / torch.where(a > 0, a, torch.ones_like(a))).pow(1.0 / p)), T)
    done = torch.zeros_like(T, dtype=torch.bool)
    for _ in range(max_iter):
        f = a * T.pow(p) + b * T + K
        fp = p * a * T.pow(p - 1) + b
        dT = f / fp
        Tn = torch.where(done, T, T - dT)
        done = done | (dT.abs() <= rtol * Tn.abs())
        T = Tn
    return T, done


def method3_root(Y, E0, Nbar, as_, ab, A1, A2, iters=200):
    """T_+ of Method 3: the root of F(T) = (E0 - Y T)(N T^-3.5 + alpha^s (1 -
    alpha_- A2)) - alpha_- (A1 + A2 N sqrt T) in (0, E0/Y), by bisection
    (F decreases strictly there).  Returns (T, ok)."""
    ok = (E0 > 0) & (Y > 0) & (Nbar > 0) & (A1 >= 0) & (1.0 - ab * A2 > 0)
    one = torch.ones_like(E0)
    hi = torch.where(ok, E0 / torch.where(ok, Y, one), one)
    lo = torch.zeros_like(hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        F = ((E0 - Y * mid) * (Nbar * mid.pow(-3.5) + as_ * (1.0 - ab * A2))
             - ab * (A1 + A2 * Nbar * mid.sqrt()))
        pos = F > 0
        lo = torch.where(pos, mid, lo)
        hi = torch.where(pos, hi, mid)
    return 0.5 * (lo + hi), ok


def interact(It, T_start, T_coef, rho, u_hat, n_up0, nhat, w, h, model,
             gamma, kappa_a, kappa_s, j, C_a, C_s, rho_floor,
             max_iter=50, rtol=1e-14, diag=None):
    """Source step for all cells.  It [Ns, *cells]; per-cell fields [*cells];
    u_hat [4, *cells]; nhat [Ns, 3]; w [Ns].  Returns (I_out, T_out, failed).
    If `diag` is a dict, the per-cell intermediates (nb0, Em, A1, A2, Y, q, K,
    Tp, Sp, Ep) are stored in it."""
    ns = It.shape[0]
    cshape = It.shape[1:]
    bc = (ns,) + (1,) * len(cshape)
    nx, ny, nz = (nhat[:, k].reshape(bc) for k in range(3))
    ws = w.reshape(bc)
    # 2. boost
    nb0 = u_hat[0] - (u_hat[1] * nx + u_hat[2] * ny + u_hat[3] * nz)
    Ib = It * nb0.pow(4)
    dOb = ws / (nb0 * nb0)
    # 3. explicit opacities (at T_coef)
    aa, as_ = opacities(model, rho, T_coef, kappa_a, kappa_s, C_a, C_s, rho_floor)
    ab = aa + as_
    # 4. angular integrals
    den = n_up0 + nb0 * ab * h
    c = n_up0 / den
    d = nb0 * h / (4.0 * math.pi * den)
    Em = (Ib * dOb).sum(0)
    A1 = (c * Ib * dOb).sum(0)
    A2 = (d * dOb).sum(0)
    # 5. temperature equation
    Y = rho / (gamma - 1.0)
    q = 1.0 - A2 * as_
    K = A1 - Y * q * T_start - q * Em
    r = torch.ones_like(Y)        # alpha_- / alpha_+ (Method 3), else 1
    if model == FIXED_EMISSIVITY:
        Sp = 4.0 * math.pi * j
        Tp = T_start
        Ep = (A1 + A2 * Sp) / q
        ok = torch.ones_like(Tp, dtype=torch.bool)
    elif model == BREMS_M3:
        Nbar = C_a * rho * rho * kappa_a
        E0 = Em + Y * T_start
        Tp, ok = method3_root(Y, E0, Nbar, as_, ab, A1, A2)
        Tp = torch.where(ok, Tp, T_start)
        Sp = torch.where(ok, Nbar * Tp.sqrt(), torch.zeros_like(Tp))
        Ep = E0 - Y * Tp
        ab_plus = Nbar * Tp.pow(-3.5) + as_
        r = torch.where(ok, ab / ab_plus, torch.ones_like(Y))
    else:
        valid = (K < 0) & (q > 0)
        Ks = torch.where(valid, K, -torch.ones_like(K))
        b = Y * q
        if model == BREMS:
            # Method 2: A2 N sqrt(T) + Y q T + K = 0, Newton in y = sqrt(T)
            Nbar = C_a * rho * rho * kappa_a
            y, conv = newton_positive_root(b, A2 * Nbar, Ks, 2.0, max_iter, rtol)
            Tp = y * y
            Sp = Nbar * y
        else:
            # Method 1: A2 alpha^a T^4 + Y q T + K = 0
            Tp, conv = newton_positive_root(A2 * aa, b, Ks, 4.0, max_iter, rtol)
            Sp = aa * Tp.pow(4)
        ok = valid & conv
        Tp = torch.where(ok, Tp, T_start)
        Sp = torch.where(ok, Sp, torch.zeros_like(Sp))
        # 6. energy balance
        Ep = Em - Y * (Tp - T_start)
    # 7. implicit intensity update and return to the tetrad frame
    Ibp = r * (c * Ib + d * (Sp + as_ * Ep))
    Iout = Ibp / nb0.pow(4)
    live = rho >= rho_floor
    use = live & ok
    Iout = torch.where(use, Iout, It)
    Tout = torch.where(use, Tp, T_start)
    failed = live & ~ok
    if diag is not None:
        diag.update(nb0=nb0, Em=Em, A1=A1, A2=A2, Y=Y, q=q, K=K, Tp=Tp, Sp=Sp, Ep=Ep, r=r,
                    abar_a=aa, abar_s=as_)
    return Iout, Tout, failed
