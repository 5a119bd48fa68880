"""Pins of the oracle's multi-group transport (Sec. 3.1, Eq.
radiative_transfer_discrete_non_gray, read for a fluid at rest in flat space,
where the frequency flux vanishes), each against something other than the
oracle's own quadrature and bisection:
  * the bin-integrated Planck function: the Stefan-Boltzmann total
    (int_0^inf x^3/(e^x - 1) dx = pi^4/15), the Bernoulli series at small x,
    the exponential series of the upper tail, and bins that partition
    [0, inf) summing to T^4/(4 pi);
  * one bin [0, inf) is the gray Method 1 step of the gray oracle;
  * a bin with no opacity is pure transport, whatever the other bins do;
  * uniform T with every bin at its Planck share (any per-cell, per-bin
    opacities) is a fixed point (Kirchhoff's law in every bin);
  * radiation + gas energy is conserved in a periodic box;
  * a uniform box relaxes to the equilibrium of Y T + T^4 = const with every
    bin at its Planck share of the final temperature.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import multigroup as mg
from oracle import step as st
from oracle.setup import build_flat, build_flat_mg

F64 = torch.float64
EDGES = (0.0, 1.0, 3.0, 9.0, math.inf)


def test_planck_total_is_stefan_boltzmann():
    assert abs(mg.planck_x3_integral(0.0, math.inf) / (math.pi ** 4 / 15.0) - 1.0) < 1e-14


@pytest.mark.parametrize("x", [0.05, 0.2, 0.7])
def test_planck_small_x_bernoulli_series(x):
    # x^3/(e^x - 1) = sum_k B_k x^(k+2)/k!  ->  int_0^x = sum_k B_k x^(k+3)/(k! (k+3))
    bern = {0: 1.0, 1: -0.5, 2: 1 / 6, 4: -1 / 30, 6: 1 / 42, 8: -1 / 30, 10: 5 / 66, 12: -691 / 2730}
    ser = sum(b * x ** (k + 3) / (math.factorial(k) * (k + 3)) for k, b in bern.items())
    assert abs(mg.planck_x3_integral(0.0, x) / ser - 1.0) < 1e-13


@pytest.mark.parametrize("x", [0.5, 3.0, 10.0, 30.0])
def test_planck_upper_tail_series(x):
    # 1/(e^t - 1) = sum_n e^(-n t)  ->  int_x^inf t^3 e^(-n t) dt in closed form
    n = np.arange(1, 400, dtype=np.float64)
    tail = (np.exp(-n * x) * (x ** 3 / n + 3 * x ** 2 / n ** 2 + 6 * x / n ** 3 + 6 / n ** 4)).sum()
    assert abs(mg.planck_x3_integral(x, math.inf) / tail - 1.0) < 1e-13


def test_bins_partition_the_planck_function():
    T = np.array([0.05, 0.5, 1.0, 2.0, 7.0])
    tot = sum(mg.planck_group(T, EDGES[g], EDGES[g + 1]) for g in range(4))
    np.testing.assert_allclose(tot, T ** 4 / (4 * math.pi), rtol=1e-14)
    # the share of the lowest bin grows as the gas cools (Wien's law)
    share = mg.planck_group(T, 0.0, 1.0) / (T ** 4 / (4 * math.pi))
    assert np.all(np.diff(share) < 0)


def _box(n=(6, 5, 4), generation=1, seed=11):
    wl = W.multigroup_flat(n=n, generation=generation, seed=seed)
    return wl


def test_one_bin_is_gray_method1():
    wl = _box()
    wl1 = dict(wl, group_edges=(0.0, math.inf), kappa_a_groups=wl["kappa_a_groups"][1:2],
               I0_iso_groups=wl["I0_iso"][None])
    pb, ka, edges, I, T = build_flat_mg(wl1)
    wg = dict(wl, kappa_a=wl["kappa_a_groups"][1])
    pg, Ig, Tg = build_flat(wg)
    for _ in range(2):
        I, T, _ = mg.step_mg(pb, ka, edges, I, T, wl["dt"])
        Ig, Tg = st.step(pg, Ig, Tg, wl["dt"])
    assert (I[0] - Ig).abs().max() <= 1e-13 * Ig.abs().max()
    assert (T - Tg).abs().max() <= 1e-13 * Tg.abs().max()


def test_bin_without_opacity_is_pure_transport():
    wl = _box()
    kag = wl["kappa_a_groups"].copy()
    kag[2] = 0.0
    wl0 = dict(wl, kappa_a_groups=kag, kappa_s=np.zeros(wl["n"]))
    pb, ka, edges, I, T = build_flat_mg(wl0)
    rng = np.random.default_rng(3)
    I[2] = torch.as_tensor(rng.uniform(0.0, 1.0, size=I[2].shape))
    # the same bin alone, as the gray oracle with no absorption, scattering or emission
    wt = dict(wl, model="fixed_emissivity", kappa_a=np.zeros(wl["n"]), kappa_s=np.zeros(wl["n"]),
              j=np.zeros(wl["n"]))
    pt, _, Tt = build_flat(wt)
    It = I[2].clone()
    for _ in range(2):
        I, T, _ = mg.step_mg(pb, ka, edges, I, T, wl["dt"])
        It, Tt = st.step(pt, It, Tt, wl["dt"])
    assert (I[2] - It).abs().max() <= 1e-14 * It.abs().max()


def test_planck_spectrum_at_uniform_temperature_is_a_fixed_point():
    # the interaction alone, with per-cell, per-bin opacities
    wl = _box()
    T0 = 1.3
    wl = dict(wl, T=np.full(wl["n"], T0))
    pb, ka, edges, I, T = build_flat_mg(wl)
    for g in range(4):
        I[g] = float(mg.planck_group(np.array(T0), edges[g], edges[g + 1]))
    Io, To, failed = mg.interact_mg(I, T, pb.rho, ka, pb.kappa_s, pb.geo.grid.w, 0.2, pb.gamma,
                                    edges, pb.rho_floor)
    assert (Io - I).abs().max() <= 1e-13 * I.abs().max()
    assert (To - T0).abs().max() <= 1e-13 * T0 and int(failed.sum()) == 0
    # whole steps in a uniform medium (the modified signal speeds depend on the
    # optical depth of each face, so only there is a uniform field free of
    # flux divergence), with different opacities per bin
    n = wl["n"]
    wl = dict(wl, rho=np.full(n, 0.7),
              kappa_a_groups=np.stack([np.full(n, k) for k in (3.0, 1.0, 0.3, 0.1)]))
    pb, ka, edges, I, T = build_flat_mg(wl)
    for g in range(4):
        I[g] = float(mg.planck_group(np.array(T0), edges[g], edges[g + 1]))
    I0 = I.clone()
    for _ in range(3):
        I, T, _ = mg.step_mg(pb, ka, edges, I, T, wl["dt"])
    assert (I - I0).abs().max() <= 1e-13 * I0.abs().max()
    assert (T - T0).abs().max() <= 1e-13 * T0


def test_energy_is_conserved_in_a_periodic_box():
    wl = _box()
    pb, ka, edges, I, T = build_flat_mg(wl)
    g = pb.geo.grid
    Y = pb.rho / (pb.gamma - 1.0)

    def energy(I, T):
        return float(mg.moments_mg(I, g.n, g.w)[0].sum() + (Y * T).sum())

    e0 = energy(I, T)
    for _ in range(3):
        I, T, _ = mg.step_mg(pb, ka, edges, I, T, wl["dt"])
        assert abs(energy(I, T) / e0 - 1.0) < 1e-13
    assert sum(pb.failed) == 0


def test_uniform_box_relaxes_to_the_planck_spectrum():
    n = (2, 2, 2)
    wl = W.multigroup_flat(n=n, generation=0, seed=5)
    T0 = 1.5
    wl = dict(wl, rho=np.ones(n), T=np.full(n, T0), kappa_s=np.ones(n),
              kappa_a_groups=np.stack([np.full(n, k) for k in (3.0, 1.0, 0.3, 0.1)]),
              I0_iso_groups=np.stack([np.full(n, v) for v in (0.0, 0.3, 0.0, 0.05)]))
    pb, ka, edges, I, T = build_flat_mg(wl)
    g = pb.geo.grid
    Y = 1.0 / (pb.gamma - 1.0)
    E = float(mg.moments_mg(I, g.n, g.w)[0, 0, 0, 0]) + Y * T0
    # equilibrium: Y T + T^4 = E (R^00 = 4 pi B = T^4), by numpy's polynomial roots
    r = np.roots([1.0, 0.0, 0.0, Y, -E])
    Teq = float(max(x.real for x in r if abs(x.imag) < 1e-12 and x.real > 0))
    # (a uniform field has no flux divergence, so a long implicit step is exact transport)
    for _ in range(40):
        I, T, _ = mg.step_mg(pb, ka, edges, I, T, 20.0)
    assert abs(float(T[0, 0, 0]) / Teq - 1.0) < 1e-10
    for k in range(4):
        Bk = mg.planck_group(np.array(Teq), edges[k], edges[k + 1])
        assert abs(float(I[k, :, 0, 0, 0].mean()) / float(Bk) - 1.0) < 1e-9
