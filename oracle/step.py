"""Predictor-corrector step and radiation moments.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.7 (Temporal Update): fluxes are computed, the radiation is advanced
explicitly by half a step, the interaction is applied implicitly; the
corrector repeats this with quantities from the half step.  For a fixed
fluid this reads (design-note reading of the corrector):
  stage 1:  I~ = I^n - dt/2 div F(I^n);   (I*, T*) = source(I~, dt/2, T_start=T^n, T_coef=T^n)
  stage 2:  I~ = I^n - dt   div F(I*);    (I^(n+1), T^(n+1)) = source(I~, dt, T_start=T^n, T_coef=T*)
Operator splitting of transport and interaction is Sec. 3.6.

Moments: R^(alpha beta) = integral n^alpha n^beta I dOmega (Eq. R), on the
grid R-hat^(ab) = sum_s w_s n-hat^a n-hat^b I_s with n-hat^0 = 1; the
radiation 4-force of the interaction step is G^a = -(R-hat^(0a)_after -
R-hat^(0a)_before)/dt (Sec. 3.6.3, sign as force on the fluid).
"""
from dataclasses import dataclass, field
import math
import torch

from . import interaction as src
from . import transport as tr

F64 = torch.float64
# storage order of the 10 independent components of a symmetric 4x4 tensor
SYM10 = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


@dataclass
class Problem:
    """Everything held fixed during a step: geometry, fluid, opacity model."""
    geo: object
    rho: torch.Tensor                       # [N1,N2,N3]
    u_hat: torch.Tensor                     # [4,N1,N2,N3] tetrad-frame fluid 4-velocity
    v: torch.Tensor                         # [3,N1,N2,N3] coordinate 3-velocity u^a/u^0
    model: int = src.KIRCHHOFF_CONST
    gamma: float = 5.0 / 3.0
    kappa_a: torch.Tensor = None
    kappa_s: torch.Tensor = None
    j: torch.Tensor = None
    C_a: float = 1.0
    C_s: float = 1.0
    rho_floor: float = 5e-4
    abar: float = 1.0
    bc_lo: tuple = (tr.PERIODIC,) * 3
    bc_hi: tuple = (tr.PERIODIC,) * 3
    limiter: int = tr.LIM_MC
    n0_cut: float = None
    angular: object = None                  # callable I -> angular flux divergence (curved)
    pole_rows: int = 0                      # rows next to each theta boundary zeroed (curved)
    newton_max_iter: int = 50
    newton_rtol: float = 1e-14
    failed: list = field(default_factory=list)

    def zeros(self):
        return torch.zeros_like(self.rho)

    def kappa_default(self):
        """kappa_a when none is given: the bremsstrahlung factor defaults to 1,
        the absorption opacity of the other models to 0."""
        if self.model in (src.BREMS, src.BREMS_M3):
            return torch.ones_like(self.rho)
        return self.zeros()


def effective_opacity(pb, T):
    """Direction-independent tetrad-frame opacity alpha-hat = u-hat^0 alpha-bar used
    in tau (Sec. 3.5), evaluated at temperature T; zero below the density floor."""
    ka = pb.kappa_a if pb.kappa_a is not None else pb.kappa_default()
    ks = pb.kappa_s if pb.kappa_s is not None else pb.zeros()
    aa, as_ = src.opacities(pb.model, pb.rho, T, ka, ks, pb.C_a, pb.C_s, pb.rho_floor)
    return pb.u_hat[0] * (aa + as_)


def source(pb, It, h, T_start, T_coef):
    g = pb.geo.grid
    ka = pb.kappa_a if pb.kappa_a is not None else pb.kappa_default()
    ks = pb.kappa_s if pb.kappa_s is not None else pb.zeros()
    jj = pb.j if pb.j is not None else pb.zeros()
    Iout, Tout, failed = src.interact(
        It, T_start, T_coef, pb.rho, pb.u_hat, pb.geo.n_up0().reshape(pb.geo.n_up0().shape[1:]),
        torch.tensor(g.n, dtype=F64), torch.tensor(g.w, dtype=F64), h, pb.model, pb.gamma,
        ka, ks, jj, pb.C_a, pb.C_s, pb.rho_floor, pb.newton_max_iter, pb.newton_rtol)
    pb.failed.append(int(failed.sum()))
    return Iout, Tout


def stage(pb, I_flux, I_base, h, dt, T_start, T_coef):
    """One operator-split stage: explicit transport by h, then the implicit source."""
    ah = effective_opacity(pb, T_coef)
    It = tr.transport(I_flux, I_base, h, dt, pb.geo, ah, pb.v, pb.abar, pb.bc_lo, pb.bc_hi,
                      pb.limiter, angular=pb.angular, n0_cut=pb.n0_cut)
    Iout, Tout = source(pb, It, h, T_start, T_coef)
    if pb.pole_rows:
        # intensity zeroed in the rows next to each pole (torus setup of Sec. 5)
        k = pb.pole_rows
        Iout = Iout.clone()
        Iout[:, :, :k] = 0.0
        Iout[:, :, -k:] = 0.0
    return Iout, Tout, It


def step(pb, I, T, dt, want_G=False):
    """Predictor-corrector step (Sec. 3.7).  Returns (I^(n+1), T^(n+1)[, G])."""
    Is, Ts, _ = stage(pb, I, I, 0.5 * dt, dt, T, T)
    In, Tn, It = stage(pb, Is, I, dt, dt, T, Ts)
    if not want_G:
        return In, Tn
    g = pb.geo.grid
    R1 = moments(In, g.n, g.w)
    R0 = moments(It, g.n, g.w)
    G = -(R1[0:4] - R0[0:4]) / dt
    return In, Tn, G


def moments(I, nhat, w):
    """R-hat^(ab) = sum_s w_s n^a n^b I_s (Eq. R), n^0 = 1.  Returns [10, *cells]
    in the order 00,01,02,03,11,12,13,22,23,33."""
    nhat = torch.as_tensor(nhat, dtype=F64)
    w = torch.as_tensor(w, dtype=F64)
    n4 = torch.cat([torch.ones(nhat.shape[0], 1, dtype=F64), nhat], dim=1)
    Wt = torch.stack([w * n4[:, a] * n4[:, b] for a, b in SYM10], dim=1)   # [Ns, 10]
    flat = I.reshape(I.shape[0], -1)
    return (Wt.T @ flat).reshape((10,) + I.shape[1:])


def energy_density(I, w):
    """J = R-hat^00 / (4 pi): mean intensity."""
    return torch.tensordot(torch.as_tensor(w, dtype=F64), I, dims=1) / (4.0 * math.pi)
