"""Pins of oracle pieces that conservation laws cannot see.

Energy conservation and the closed-form relaxation tests hold for any
upwinding of the advection term, any opacity law and any slope limiter that
keeps the scheme conservative, so each of those pieces needs a check of its
own, against a textbook result:

  * the advection term of the modified flux (Sec. 3.5, third term of
    Eq. flux_Jiang): in the optically thick limit a jump carried by the fluid
    is moved by the first-order upwind (Godunov) rule, whose one-step result
    for a step profile is the Courant number;
  * the bremsstrahlung-like opacity law alpha^a = C_a rho^2 T^-7/2 (Sec. 3.6.2,
    the law behind Eq. implicit_T): with the gas temperature pinned (Y >> E),
    the discrete intensity relaxes to B(T) by the factor 1/(1 + alpha^a dt)
    per step, so the rate read off the evolution must follow rho^2 T^-7/2;
  * the minmod limiter (PLI of Sec. 3.4, the limiter option): textbook values
    and the TVD property that a face state lies between the two cell averages
    sharing the face.

It also holds the measurement behind the curved FP64 temperature bar of the
GPU parity tests: a rounding-level change of the intensity moves T by ~1e3
times more just above the density floor, while the gas-energy form of the
comparison stays at the rounding level.
"""
import math

import numpy as np
import torch

import workloads as W
from oracle import step as st
from oracle import transport as tr
from oracle.geometry import FlatCartesian
from oracle.grid import GeodesicGrid
from oracle.setup import build_flat

F64 = torch.float64


# --------------------------------------------------------------------------
# advection term: upwind in the fluid velocity
# --------------------------------------------------------------------------
def _step_profile_transport(v):
    """One transport sub-step (h = dt = 0.4, dx = 1) of a periodic step profile
    (1 on the first half of the x line, 0 on the second) carried by a uniform
    fluid velocity v along x, at tau = 4000 (optically thick)."""
    g = GeodesicGrid(0)
    n = (8, 1, 1)
    geo = FlatCartesian(n, (0, 0, 0), n, g)
    prof = torch.tensor([1.0] * 4 + [0.0] * 4, dtype=F64)
    I = prof.reshape(1, -1, 1, 1).expand(g.ns, -1, 1, 1).clone()
    alpha = torch.full(n, 1e4, dtype=F64)
    vel = torch.zeros((3,) + n, dtype=F64)
    vel[0] = v
    It = tr.transport(I, I, 0.4, 0.4, geo, alpha, vel, 1.0, (0,) * 3, (0,) * 3, tr.LIM_MC)
    return It


def test_advection_term_is_upwind_in_the_fluid_velocity():
    """tau >> 1 (e^-tau = 0, radiative speeds ~ 1/tau): the flux is the fluid's
    advection term, n_0 n^0 v I_upwind.  The MC slopes vanish at both jumps, so
    the first-order upwind rule gives, with Courant number sigma = |v| h/dx:
    the cell downstream of the 1 -> 0 jump rises to sigma, the first cell past
    the 0 -> 1 jump falls to 1 - sigma, every other cell keeps its value
    (exactly, up to the O(h/tau) radiative diffusion).  A downwind choice
    leaves the downstream cell at 0."""
    h = 0.4
    for v in (0.5, -0.5):
        It = _step_profile_transport(v)[:, :, 0, 0]
        sigma = abs(v) * h
        ref = torch.tensor([1.0] * 4 + [0.0] * 4, dtype=F64)
        if v > 0:
            ref[4] = sigma          # downstream of 1 -> 0 (between cells 3 and 4)
            ref[0] = 1.0 - sigma    # past 0 -> 1 (between cells 7 and 0, periodic)
        else:
            ref[7] = sigma          # cell 0's 1 flows into cell 7 (periodic)
            ref[3] = 1.0 - sigma    # cell 3 empties into cell 2, cell 4's 0 flows in
        assert torch.allclose(It, ref.expand_as(It), rtol=0, atol=1e-4), (v, It[0])


def test_advection_term_carries_a_thick_jump_at_the_fluid_speed():
    """Many steps of the two transport stages of Sec. 3.7 (the interaction
    left out): in the optically thick limit the radiation of an opaque flow
    moves with it, its centroid advancing by v t, and stays within the initial
    bounds."""
    g = GeodesicGrid(0)
    nx = 64
    n = (nx, 1, 1)
    geo = FlatCartesian(n, (0, 0, 0), n, g)
    x = torch.arange(nx, dtype=F64) + 0.5
    prof = torch.exp(-((x - 20.0) / 5.0) ** 2)
    I = prof.reshape(1, -1, 1, 1).expand(g.ns, -1, 1, 1).clone()
    alpha = torch.full(n, 1e4, dtype=F64)
    v = 0.3
    vel = torch.zeros((3,) + n, dtype=F64)
    vel[0] = v
    dt, nsteps = 0.4, 100
    for _ in range(nsteps):
        Is = tr.transport(I, I, dt / 2, dt, geo, alpha, vel, 1.0, (0,) * 3, (0,) * 3, tr.LIM_MC)
        I = tr.transport(Is, I, dt, dt, geo, alpha, vel, 1.0, (0,) * 3, (0,) * 3, tr.LIM_MC)
    p = I[0, :, 0, 0]
    c = float((p * x).sum() / p.sum())
    assert abs(c - (20.0 + v * nsteps * dt)) < 0.05, c
    assert float(p.min()) > -1e-6 and float(p.max()) <= 1.0 + 1e-12


# --------------------------------------------------------------------------
# bremsstrahlung-like opacity law
# --------------------------------------------------------------------------
def _one_cell_brems(rho, T0, I0, gamma):
    n = (1, 1, 1)
    wl = dict(n=n, xlo=(0, 0, 0), xhi=n, generation=1, weights="voronoi", bc=("periodic",) * 3,
              model="brems", gamma=gamma, C_a=1.0, C_s=0.0, rho=np.full(n, rho), T=np.full(n, T0),
              kappa_a=None, kappa_s=None, j=None, u=None, I0_iso=np.full(n, I0))
    return build_flat(wl)


def test_brems_relaxation_rate_follows_rho2_T_minus_3p5():
    """One isolated cell (a uniform periodic box: no transport), no
    scattering, Gamma - 1 = 1e-7 so the gas heat capacity pins T: each step
    maps I - B(T) to (I - B(T))/(1 + alpha^a dt) with alpha^a = rho^2 T^-7/2
    (stage 2 restarts from I^n with h = dt), and the intensity tends to
    B(T) = T^4/(4 pi).  The rate read off the evolution, for four (rho, T)
    pairs spanning a factor 20 in rho^2 T^-7/2, must equal the law."""
    dt = 0.4
    rates = []
    for rho, T0 in ((0.5, 0.7), (2.0, 1.6), (1.3, 1.0), (0.8, 2.2)):
        pb, I, T = _one_cell_brems(rho, T0, 0.01, 1.0 + 1e-7)
        B = T0 ** 4 / (4 * math.pi)
        d0 = I[0].item() - B
        for _ in range(3):
            I, T = st.step(pb, I, T, dt)
        d3 = I[0].item() - B
        assert abs(T.item() - T0) < 1e-5 * T0
        # per-step factor 1/(1 + alpha dt)  ->  alpha
        alpha = ((d0 / d3) ** (1.0 / 3.0) - 1.0) / dt
        law = rho ** 2 * T0 ** -3.5
        rates.append(alpha / law)
        assert abs(alpha / law - 1.0) < 1e-4, (rho, T0, alpha, law)
        # isotropic: every direction relaxes alike
        assert torch.allclose(I, torch.full_like(I, I[0].item()), rtol=1e-13)
    assert max(rates) - min(rates) < 2e-4


def test_brems_equilibrium_is_planck():
    """Long evolution with the same pinned T: the intensity reaches
    B(T) = T^4/(4 pi) (emission C_a rho^2 sqrt(T) balances absorption
    C_a rho^2 T^-7/2 times 4 pi I only at the Planck value)."""
    rho, T0 = 1.7, 0.9
    pb, I, T = _one_cell_brems(rho, T0, 0.2, 1.0 + 1e-7)
    for _ in range(200):
        I, T = st.step(pb, I, T, 0.4)
    B = T.item() ** 4 / (4 * math.pi)
    assert abs(I[0].item() / B - 1.0) < 1e-9


# --------------------------------------------------------------------------
# minmod limiter
# --------------------------------------------------------------------------
def test_minmod_limiter_textbook():
    """minmod(p, q) = sign(p) min(|p|, |q|) when p q > 0, else 0."""
    p = torch.tensor([1.0, -1.0, 1.0, 0.1, 3.0, -2.5, 0.0, 4.0], dtype=F64)
    q = torch.tensor([2.0, -3.0, -1.0, 3.0, 0.1, -0.5, 1.0, 4.0], dtype=F64)
    out = tr.limited_slope(p, q, tr.LIM_MINMOD)
    assert out.tolist() == [1.0, -1.0, 0.0, 0.1, 0.1, -0.5, 0.0, 4.0]


def test_limited_face_states_lie_between_neighbours():
    """TVD property of the limited PLI states (both limiters): the state at a
    face, reconstructed from either side, lies between the two cell averages
    that share the face (so no new extrema are created)."""
    rng = np.random.default_rng(9)
    for lim in (tr.LIM_MC, tr.LIM_MINMOD):
        for _ in range(20):
            P = torch.tensor(rng.uniform(-1, 1, 40) * rng.choice([1e-3, 1.0, 1e3]), dtype=F64)
            D = tr.limited_slope(P[1:-1] - P[:-2], P[2:] - P[1:-1], lim)   # slopes of cells 1..38
            c = P[1:-1]
            up = c + 0.5 * D          # state at the upper face of each cell
            dn = c - 0.5 * D          # state at the lower face
            hi_nb, lo_nb = P[2:], P[:-2]
            tol = 1e-15 * P.abs().max()
            assert bool(((up - torch.minimum(c, hi_nb)) >= -tol).all())
            assert bool(((up - torch.maximum(c, hi_nb)) <= tol).all())
            assert bool(((dn - torch.minimum(c, lo_nb)) >= -tol).all())
            assert bool(((dn - torch.maximum(c, lo_nb)) <= tol).all())


def test_minmod_is_more_diffusive_than_mc():
    """Textbook ordering: |minmod slope| <= |MC slope| everywhere, strictly
    smaller for smooth unequal differences."""
    rng = np.random.default_rng(4)
    p = torch.tensor(rng.uniform(-1, 1, 1000), dtype=F64)
    q = torch.tensor(rng.uniform(-1, 1, 1000), dtype=F64)
    a = tr.limited_slope(p, q, tr.LIM_MINMOD).abs()
    b = tr.limited_slope(p, q, tr.LIM_MC).abs()
    assert bool((a <= b).all())
    same_sign = (p * q > 0) & ((p - q).abs() > 1e-3)
    assert bool((a[same_sign] < b[same_sign]).all())


# --------------------------------------------------------------------------
# conditioning of T in the curved parity cases
# --------------------------------------------------------------------------
def test_curved_temperature_conditioning_near_density_floor():
    """The measurement behind comparing T through the gas energy in the curved
    FP64 parity tests: on the reduced torus (12x16x8, generation 1, one step),
    flipping the last bits of I^n (relative 1e-14, random sign) moves T by a
    relative ~1e3 times more in cells just above the density floor (Y there is
    ~1e-3 of the radiation energy), while Y |dT| / (Y T + E) stays at the
    rounding level of the radiation sums."""
    from oracle.setup import build_ks
    n = (12, 16, 8)
    wl = W.torus_ks(n=n, a=0.9, generation=1)
    wl["pole_rows"] = 2
    wl["M"] = 1.0
    I0 = W.random_intensity(42, n, 11, 0.5, 1.5)
    pb, _, T0, dt = build_ks(wl)
    eps = 1e-14
    Ia, Ta = st.step(pb, torch.as_tensor(I0).clone(), T0.clone(), dt)
    sgn = np.random.default_rng(5).choice([-1.0, 1.0], size=I0.shape)
    Ib, Tb = st.step(pb, torch.as_tensor(I0 * (1 + eps * sgn)), T0.clone(), dt)
    dT = (Ta - Tb).abs()
    rel_T = (dT / Ta.abs()).max().item()
    assert rel_T > 100 * eps, rel_T            # T alone is ill-conditioned here
    rho = torch.as_tensor(wl["rho"])
    Y = rho / (wl["gamma"] - 1.0)
    E = st.moments(Ia, pb.geo.grid.n, pb.geo.grid.w)[0]
    gas = (Y * dT / (Y * Ta.abs() + E.abs())).max().item()
    assert gas < 20 * eps, gas                 # the gas-energy form is not
    i = int((dT / Ta.abs()).argmax())
    assert rho.reshape(-1)[i].item() < 10 * pb.rho_floor
