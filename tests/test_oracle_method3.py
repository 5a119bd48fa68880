"""Pins of the oracle's Method 3 temperature solve (Sec. 3.6.2, the total
opacity semi-implicit, Eq. T_almost_fully_implicit), each against something
other than the oracle's own bisection:
  * the root is the one a library polynomial solver (numpy.roots) finds for
    the printed polynomial, written in y = sqrt(T) (degree 9), with the
    angular integrals read as the bare integrals B1 = alpha_- dt A1,
    B2 = alpha_- dt A2;
  * the per-direction update integrates to the energy balance: sum_s w_s
    Ibar_+ = E0 - Y T_+, so radiation + gas energy is conserved every step;
  * when the gas pins the temperature (Y >> E) Method 3 reduces to Method 2:
    the relaxation rate is the bremsstrahlung law rho^2 T^-7/2;
  * the paper's equilibration setup relaxes to the T_eq of T^4 + Y T = u;
  * stiff relaxation (high density, low temperature, alpha dt ~ 1e3): Method 3
    stays closer than Method 2 to a reference resolved with 200 sub-steps.
"""
import math

import numpy as np
import torch

from oracle import interaction as src
from oracle import step as st
from oracle.setup import build_flat

F64 = torch.float64


def _cell(rho, T0, I0, gamma=5 / 3, model="brems_m3", C_s=0.0, g=1):
    n = (1, 1, 1)
    wl = dict(n=n, xlo=(0, 0, 0), xhi=n, generation=g, weights="voronoi", bc=("periodic",) * 3,
              model=model, gamma=gamma, C_a=1.0, C_s=C_s, rho=np.full(n, rho), T=np.full(n, T0),
              kappa_a=None, kappa_s=None, j=None, u=None, I0_iso=np.full(n, I0))
    return build_flat(wl)


def _interact_diag(rho, T0, I0, h, C_s, model="brems_m3", aniso=0.0, seed=0):
    pb, I, T = _cell(rho, T0, I0, C_s=C_s, model=model)
    g = pb.geo.grid
    if aniso:
        rng = np.random.default_rng(seed)
        I = I * torch.as_tensor(1.0 + aniso * rng.uniform(-1, 1, (g.ns, 1, 1, 1)))
    d = {}
    Iout, Tout, failed = src.interact(
        I, T, T, pb.rho, pb.u_hat, torch.ones((1, 1, 1), dtype=F64), torch.tensor(g.n, dtype=F64),
        torch.tensor(g.w, dtype=F64), h, pb.model, pb.gamma, pb.kappa_default(), pb.zeros(), pb.zeros(),
        pb.C_a, pb.C_s, pb.rho_floor, diag=d)
    return I, Iout, Tout, failed, d, g


def test_method3_root_matches_numpy_roots_of_the_printed_polynomial():
    rng = np.random.default_rng(7)
    for _ in range(12):
        rho, T0 = rng.uniform(0.3, 3.0), rng.uniform(0.3, 2.5)
        I0, h, C_s = rng.uniform(0.0, 2.0), rng.uniform(0.05, 2.0), rng.choice([0.0, 0.7])
        _, _, Tout, failed, d, _ = _interact_diag(rho, T0, I0, h, C_s)
        assert not bool(failed.any())
        Y, Em, A1, A2 = (float(d[k].reshape(-1)[0]) for k in ("Y", "Em", "A1", "A2"))
        N = rho * rho
        a_s = C_s * rho
        a_m = N * T0 ** -3.5 + a_s                     # explicit alpha_- at T_coef = T0
        E0 = Em + Y * T0
        B1, B2 = a_m * h * A1, a_m * h * A2
        # -Y as (dt - B2) y^9 - B2 N y^8 - [B2 as E0 + B1 - E0 as dt] y^7 - Y N dt y^2 + E0 N dt
        coef = np.zeros(10)
        coef[0] = -Y * a_s * (h - B2)
        coef[1] = -B2 * N
        coef[2] = -(B2 * a_s * E0 + B1 - E0 * a_s * h)
        coef[7] = -Y * N * h
        coef[9] = E0 * N * h
        k0 = next(i for i in range(10) if coef[i] != 0.0)
        roots = np.roots(coef[k0:])
        cand = [r.real ** 2 for r in roots if abs(r.imag) < 1e-9 * abs(r) and r.real > 0
                and r.real ** 2 < E0 / Y]
        assert len(cand) == 1, cand
        assert abs(float(Tout.reshape(-1)[0]) - cand[0]) < 1e-9 * cand[0]


def test_method3_update_integrates_to_the_energy_balance():
    """sum_s w_s Ibar_+ = E0 - Y T_+ with an anisotropic I_- (fluid at rest:
    Ibar = I); hence E + Y T is conserved."""
    for C_s in (0.0, 1.3):
        I, Iout, Tout, _, d, g = _interact_diag(1.4, 0.8, 0.6, 0.4, C_s, aniso=0.5, seed=3)
        w = torch.tensor(g.w, dtype=F64).reshape(-1, 1, 1, 1)
        E_in, E_out = float((w * I).sum()), float((w * Iout).sum())
        Y = float(d["Y"].reshape(-1)[0])
        T0 = 0.8
        assert abs((E_out + Y * float(Tout.reshape(-1)[0])) - (E_in + Y * T0)) < 1e-13 * (E_in + Y * T0)
        assert abs(E_out - float(d["Ep"].reshape(-1)[0])) < 1e-13 * abs(E_out)
        assert float(d["r"].reshape(-1)[0]) != 1.0


def test_method3_reduces_to_the_bremsstrahlung_rate_when_T_is_pinned():
    dt = 0.4
    for rho, T0 in ((0.5, 0.7), (2.0, 1.6), (1.3, 1.0)):
        pb, I, T = _cell(rho, T0, 0.01, gamma=1.0 + 1e-7)
        B = T0 ** 4 / (4 * math.pi)
        d0 = I[0].item() - B
        for _ in range(3):
            I, T = st.step(pb, I, T, dt)
        alpha = ((d0 / (I[0].item() - B)) ** (1.0 / 3.0) - 1.0) / dt
        assert abs(alpha / (rho ** 2 * T0 ** -3.5) - 1.0) < 1e-4


def test_method3_equilibration_paper_setup():
    """Sec. 4.11 setup (rho = 1, Gamma = 5/3, T_gas = 2, T_rad = 1) with the
    bremsstrahlung opacity: the cell relaxes to T^4 + Y T = u, energy
    conserved every step."""
    rho, gam, Tg, Tr = 1.0, 5 / 3, 2.0, 1.0
    Y = rho / (gam - 1)
    u = Tr ** 4 + Y * Tg
    Teq = max(r.real for r in np.roots([1, 0, 0, Y, -u]) if abs(r.imag) < 1e-12 and r.real > 0)
    pb, I, T = _cell(rho, Tg, Tr ** 4 / (4 * math.pi), gamma=gam)
    g = pb.geo.grid
    for _ in range(150):
        I, T = st.step(pb, I, T, 0.4)
        E = st.moments(I, g.n, g.w)[0]
        assert abs((E + Y * T).item() - u) < 1e-13 * u
    assert abs(T.item() - Teq) < 1e-10


def test_method3_is_closer_than_method2_on_a_stiff_cell():
    """High density and low temperature (alpha dt ~ 1e3), gas hotter than the
    radiation: one step of each method against 200 Method 2 sub-steps."""
    rho, T0, I0, dt = 6.0, 0.35, 0.002, 0.4
    out = {}
    for model in ("brems", "brems_m3"):
        pb, I, T = _cell(rho, T0, I0, model=model)
        I, T = st.step(pb, I, T, dt)
        out[model] = T.item()
    pb, I, T = _cell(rho, T0, I0, model="brems")
    for _ in range(200):
        I, T = st.step(pb, I, T, dt / 200)
    ref = T.item()
    assert abs(out["brems_m3"] - ref) < abs(out["brems"] - ref), (out, ref)
