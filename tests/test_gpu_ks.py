"""Parity of the curved (Kerr-Schild) HIP path with the FP64 oracle.

Covers the position-dependent spatial fluxes with the n_0 sign rule and cut,
the angular (geodesic-edge) flux, the lapse in the interaction, the rows
zeroed next to the axis, zero-incoming outer boundaries and the
coordinate-frame moments.  Bars: FP64 within 1e-12 (I and R^(ab) element by
element; T through the gas energy, see _check_fp64), FP32 transport within
1e-5 (rel-L2 of J, R^(ab), T).
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from runners import J_of, gpu_context, gpu_run, moments_error, oracle_problem, oracle_run, rel_l2, rel_max

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _say(msg):
    print(msg, flush=True)


def _case(n=(12, 16, 8), a=0.9, generation=1, pole_rows=2, scattering=False, r_in=1.5,
          r_out=50.0, seed=11, M=1.0):
    wl = W.torus_ks(n=n, a=a, generation=generation, scattering=scattering, r_in=r_in, r_out=r_out)
    wl["pole_rows"] = pole_rows
    wl["M"] = M
    if M == 0.0:
        # flat space in spherical coordinates: the fluid is the static observer
        u = np.zeros((4,) + tuple(n))
        u[0] = 1.0
        wl["u"] = u
    ns = 10 * 4 ** generation + 2
    I0 = W.random_intensity(ns, n, seed, 0.5, 1.5)
    _, _, _, dt = _oracle_setup(wl)
    wl["dt"] = dt
    return wl, I0


def _oracle_setup(wl):
    from oracle.setup import build_ks
    return build_ks(wl)


def _check_fp64(g, o, wl, tol=1e-12):
    """I and R^(ab) element by element relative to their maxima; T through the
    gas energy: Y |dT| <= tol (Y T + R^00) per cell, Y = rho/(Gamma-1).  Just
    above the density floor Y is ~1e-3 of the radiation energy, and the
    temperature equation turns a rounding-level change of the radiation sums
    into a 1e3 times larger relative change of T (measured on the oracle by
    perturbing I^n by 1e-14); the gas-energy form is the well-conditioned one."""
    assert rel_max(g["I"], o["I"]) < tol, rel_max(g["I"], o["I"])
    for k in range(10):
        assert (g["R"][k] - o["R"][k]).abs().max() <= tol * o["R"][0].abs().max(), k
    Y = torch.as_tensor(wl["rho"]) / (wl["gamma"] - 1.0)
    err = (Y * (g["T"] - o["T"]).abs() / (Y * o["T"].abs() + o["R"][0].abs())).max()
    assert err < tol, float(err)


def _check_fp32(g, o, tol=1e-5):
    assert rel_l2(J_of(g["R"]), J_of(o["R"])) < tol
    assert moments_error(g["R"], o["R"]) < tol
    assert rel_l2(g["T"], o["T"]) < tol


def test_ks_dt_max_matches_oracle():
    wl, _ = _case()
    ctx = gpu_context(wl)
    assert abs(ctx.dt_max - wl["dt"]) <= 1e-13 * wl["dt"]
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_torus_reduced(precision):
    """a = 0.9 torus, 12x16x8 (ln r, theta, phi), generation 1, 3 steps,
    Keplerian flow inside the torus, rows next to the axis zeroed."""
    wl, I0 = _case()
    _say(f"torus_ks {precision} 12x16x8 g1 3 steps")
    g = gpu_run(wl, 3, precision=precision, I0=I0)
    o = oracle_run(wl, 3, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wl)
    else:
        _check_fp32(g, o)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_torus_method3(precision):
    """The torus with Method 3 (12x16x8, generation 1, 3 steps, Keplerian flow:
    the direction-dependent map carries alpha_-/alpha_+)."""
    wl, I0 = _case()
    wl["model"] = "brems_m3"
    _say(f"torus_ks method 3 {precision} 12x16x8 g1 3 steps")
    g = gpu_run(wl, 3, precision=precision, I0=I0)
    o = oracle_run(wl, 3, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wl)
    else:
        _check_fp32(g, o)


def test_ks_inside_horizon_sign_rule_and_cut():
    """Inner boundary inside the horizon (r_in = 1.2 < r_+ = 1.436 for a = 0.9):
    n_0 changes sign between cells and falls below the cut for some
    directions; generation 2; minmod; scattering; no zeroed rows."""
    wl, I0 = _case(n=(10, 12, 6), generation=2, pole_rows=0, scattering=True, r_in=1.2, r_out=8.0)
    _say("torus_ks fp64 inside horizon 10x12x6 g2 2 steps minmod")
    pb, _, _ = oracle_problem(wl)
    nl0 = pb.geo._n_low0
    assert (np.abs(nl0) < wl["n0_cut"]).any() and (nl0 > 0).any() and (nl0 < 0).any()
    g = gpu_run(wl, 2, I0=I0, limiter="minmod")
    o = oracle_run(wl, 2, I0=I0, limiter=1)
    _check_fp64(g, o, wl)


def test_ks_flat_spherical():
    """M = 0: flat space in (ln r, theta, phi); the angular flux alone keeps
    straight rays straight; zero-incoming outside, generation 2."""
    wl, I0 = _case(n=(8, 10, 6), generation=2, pole_rows=1, M=0.0, a=0.0, r_in=2.0, r_out=9.0)
    _say("flat spherical fp64 8x10x6 g2 3 steps")
    g = gpu_run(wl, 3, I0=I0)
    o = oracle_run(wl, 3, I0=I0)
    _check_fp64(g, o, wl)


def test_ks_coordinate_moments():
    """rt_moments with RT_COORD: R^(mu nu) = e^mu_a e^nu_b R-hat^(ab)."""
    from oracle.kerr import coordinate_moments
    wl, I0 = _case(n=(6, 8, 4))
    ctx = gpu_context(wl)
    I = torch.as_tensor(I0, dtype=F64).reshape(ctx.ns, -1).cuda().contiguous()
    Rc = ctx.moments(I, frame="coord").cpu()
    Rt = ctx.moments(I, frame="tetrad").cpu()
    torch.cuda.synchronize()
    ctx.close()
    pb, _, _ = oracle_problem(wl)
    ref = coordinate_moments(Rt, pb.geo.ec)
    assert (Rc - ref).abs().max() <= 1e-12 * ref.abs().max()


@pytest.mark.parametrize("recon", ["donor", "mapr"])
def test_ks_full_size_fp32_sampled(recon):
    """The a = 0.9 torus at 256x128x64, generation 2 (162 directions), FP32,
    one step in one launch sequence, donor-cell or MAPR angular states;
    sub-boxes away from the r and theta boundaries are recomputed by the
    oracle with a 4-cell halo (the reach of one predictor-corrector step) and
    compared on their interiors."""
    n = (256, 128, 64)
    wl = W.torus_ks(n=n, generation=2)
    wl["angular_recon"] = recon
    ns = 162
    rng = np.random.default_rng(21)
    I0 = rng.uniform(0.5, 1.5, size=(ns,) + n).astype(np.float32)
    ctx = gpu_context(wl, precision="fp32")
    dt = ctx.dt_max
    _say(f"torus_ks {recon} fp32 256x128x64 g2 1 step dt={dt}")
    I = torch.as_tensor(I0).reshape(ns, -1).cuda().contiguous()
    T = torch.as_tensor(wl["T"], dtype=F64).reshape(-1).cuda().contiguous()
    ctx.step(I, T, dt, 1)
    torch.cuda.synchronize()
    Ig = I.cpu().reshape((ns,) + n)
    Tg = T.cpu().reshape(n)
    ctx.close()
    _, wgt, _ = __import__("paper_2508_15532_amd").geodesic_grid(2)
    H, B = 4, 4
    for (c1, c2) in ((20, 64), (120, 40), (200, 90)):
        lo1, hi1, lo2, hi2 = c1 - B - H, c1 + B + H, c2 - B - H, c2 + B + H
        sub = dict(wl)
        dx1 = (wl["xhi"][0] - wl["xlo"][0]) / n[0]
        dx2 = (wl["xhi"][1] - wl["xlo"][1]) / n[1]
        sub["n"] = (hi1 - lo1, hi2 - lo2, n[2])
        sub["xlo"] = (wl["xlo"][0] + lo1 * dx1, wl["xlo"][1] + lo2 * dx2, wl["xlo"][2])
        sub["xhi"] = (wl["xlo"][0] + hi1 * dx1, wl["xlo"][1] + hi2 * dx2, wl["xhi"][2])
        for key in ("rho", "T", "I0_iso"):
            sub[key] = wl[key][lo1:hi1, lo2:hi2]
        sub["u"] = wl["u"][:, lo1:hi1, lo2:hi2]
        sub["pole_rows"] = 0
        sub["bc"] = ("outflow", "outflow", "periodic")
        sub["bc_hi"] = ("outflow", "outflow", "periodic")
        sub["dt"] = dt
        if recon == "mapr":
            sub["mapr_tie_rtol"] = 1e-4          # the FP32 form's tie band
        _say(f"  sub-box r[{lo1}:{hi1}] theta[{lo2}:{hi2}]")
        o = oracle_run(sub, 1, I0=I0[:, lo1:hi1, lo2:hi2].astype(np.float64))
        inner = (slice(H, -H), slice(H, -H))
        Jg = torch.tensordot(torch.as_tensor(wgt), Ig[:, lo1:hi1, lo2:hi2].double(), dims=1)[inner]
        Jo = torch.tensordot(torch.as_tensor(wgt), o["I"], dims=1)[inner]
        assert rel_l2(Jg, Jo) < 1e-5, rel_l2(Jg, Jo)
        assert rel_l2(Ig[:, lo1:hi1, lo2:hi2][:, H:-H, H:-H].double(), o["I"][:, H:-H, H:-H]) < 1e-5
        assert rel_l2(Tg[lo1:hi1, lo2:hi2][inner], o["T"][inner]) < 1e-5


def test_ks_c5_full_size_fp32_sampled():
    """The a = 0.9 turbulent torus at 384x192x128, generation 3 (642
    directions), lognormal density (sigma_ln 0.7) and scattering, FP32: one
    step on the full grid (24 GB per intensity copy, the angular kernel in its
    many-direction form), then sub-boxes away from the r and theta boundaries
    recomputed by the oracle with a 4-cell halo and compared on their
    interiors.  The initial intensity is a seeded rank-2 product a_s b_c + a'_s b'_c
    (built on the GPU, sliced on the host, the same float32 arithmetic)."""
    n = (384, 192, 128)
    gen, ns = 3, 642
    wl = W.torus_ks(n=n, generation=gen, sigma_ln=0.7, scattering=True)
    rng = np.random.default_rng(31)
    nc = n[0] * n[1] * n[2]
    a1, a2 = (rng.uniform(0.2, 1.0, ns).astype(np.float32) for _ in range(2))
    b1, b2 = (rng.uniform(0.2, 1.0, nc).astype(np.float32) for _ in range(2))
    ctx = gpu_context(wl, precision="fp32")
    dt = ctx.dt_max
    _say(f"torus_ks fp32 384x192x128 g3 sigma_ln 0.7 scattering, 1 step dt={dt}")
    dev = torch.device("cuda", 0)
    A1, A2 = (torch.as_tensor(x, device=dev)[:, None] for x in (a1, a2))
    B1, B2 = (torch.as_tensor(x, device=dev)[None, :] for x in (b1, b2))
    I = (A1 * B1 + A2 * B2).contiguous()
    del A1, A2, B1, B2
    T = torch.as_tensor(wl["T"], dtype=F64).reshape(-1).to(dev).contiguous()
    ctx.step(I, T, dt, 1)
    torch.cuda.synchronize()
    Tg = T.cpu().reshape(n)
    I4 = I.view(ns, *n)
    _, wgt, _ = __import__("paper_2508_15532_amd").geodesic_grid(gen)
    H, B = 4, 3
    for (c1, c2) in ((60, 96), (200, 80)):
        lo1, hi1, lo2, hi2 = c1 - B - H, c1 + B + H, c2 - B - H, c2 + B + H
        Ig = I4[:, lo1:hi1, lo2:hi2, :].double().cpu()
        b1s = b1.reshape(n)[lo1:hi1, lo2:hi2]
        b2s = b2.reshape(n)[lo1:hi1, lo2:hi2]
        I0s = (a1[:, None, None, None] * b1s[None] + a2[:, None, None, None] * b2s[None]).astype(np.float64)
        sub = dict(wl)
        dx1 = (wl["xhi"][0] - wl["xlo"][0]) / n[0]
        dx2 = (wl["xhi"][1] - wl["xlo"][1]) / n[1]
        sub["n"] = (hi1 - lo1, hi2 - lo2, n[2])
        sub["xlo"] = (wl["xlo"][0] + lo1 * dx1, wl["xlo"][1] + lo2 * dx2, wl["xlo"][2])
        sub["xhi"] = (wl["xlo"][0] + hi1 * dx1, wl["xlo"][1] + hi2 * dx2, wl["xhi"][2])
        for key in ("rho", "T", "I0_iso"):
            sub[key] = wl[key][lo1:hi1, lo2:hi2]
        sub["u"] = wl["u"][:, lo1:hi1, lo2:hi2]
        sub["pole_rows"] = 0
        sub["bc"] = ("outflow", "outflow", "periodic")
        sub["bc_hi"] = ("outflow", "outflow", "periodic")
        sub["dt"] = dt
        _say(f"  sub-box r[{lo1}:{hi1}] theta[{lo2}:{hi2}]")
        o = oracle_run(sub, 1, I0=I0s)
        inner = (slice(H, -H), slice(H, -H))
        Jg = torch.tensordot(torch.as_tensor(wgt), Ig, dims=1)[inner]
        Jo = torch.tensordot(torch.as_tensor(wgt), o["I"], dims=1)[inner]
        assert rel_l2(Jg, Jo) < 1e-5, rel_l2(Jg, Jo)
        assert rel_l2(Ig[:, H:-H, H:-H], o["I"][:, H:-H, H:-H]) < 1e-5
        assert rel_l2(Tg[lo1:hi1, lo2:hi2][inner], o["T"][inner]) < 1e-5
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_generation4_patches(precision):
    """2562 directions: the angular kernel runs on 19 patches of directions
    with halos of 42-79 rows (several partly filled); 4 x 6 x 70 cells, so the
    256-byte rows of a phi run end in a ragged one."""
    wl, I0 = _case(n=(4, 6, 70), generation=4, pole_rows=1)
    _say(f"torus_ks {precision} g4 4x6x70 1 step")
    g = gpu_run(wl, 1, precision=precision, I0=I0)
    o = oracle_run(wl, 1, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wl)
    else:
        _check_fp32(g, o)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_generation3(precision):
    """642 directions: the angular kernel keeps only the intensities in LDS
    (runs of 8 phi cells in FP64, 16 in FP32) and reads the coefficient rows
    from memory; 5 x 8 x 20 cells, so a phi row spans several workgroups with a
    ragged last one."""
    wl, I0 = _case(n=(5, 8, 20), generation=3, pole_rows=1)
    _say(f"torus_ks {precision} g3 5x8x20 2 steps")
    g = gpu_run(wl, 2, precision=precision, I0=I0)
    o = oracle_run(wl, 2, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wl)
    else:
        _check_fp32(g, o)


def _mapr(wl, precision="fp64"):
    """MAPR angular states; the oracle takes the tie band of the form it is
    compared with (1e-4 relative |g|^2 for FP32, 1e-8 for FP64)."""
    wl = dict(wl)
    wl["angular_recon"] = "mapr"
    if precision == "fp32":
        wl["mapr_tie_rtol"] = 1e-4
    return wl


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_mapr_torus_reduced(precision):
    """MAPR angular edge states on the reduced torus (12x16x8, generation 1,
    3 steps); the result also differs from the donor-cell one, so the MAPR
    kernels are the ones that ran."""
    wl, I0 = _case()
    wm = _mapr(wl, precision)
    _say(f"torus_ks mapr {precision} 12x16x8 g1 3 steps")
    g = gpu_run(wm, 3, precision=precision, I0=I0)
    o = oracle_run(wm, 3, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wm)
        d = gpu_run(wl, 3, precision=precision, I0=I0)
        assert rel_max(g["I"], d["I"]) > 1e-6
    else:
        _check_fp32(g, o)


def test_ks_mapr_inside_horizon_generation2():
    """MAPR with n_0 changing sign and falling below the cut (r_in inside the
    horizon), generation 2, minmod, scattering, 2 steps, FP64."""
    wl, I0 = _case(n=(10, 12, 6), generation=2, pole_rows=0, scattering=True, r_in=1.2, r_out=8.0)
    wm = _mapr(wl)
    _say("torus_ks mapr fp64 inside horizon 10x12x6 g2 2 steps minmod")
    g = gpu_run(wm, 2, I0=I0, limiter="minmod")
    o = oracle_run(wm, 2, I0=I0, limiter=1)
    _check_fp64(g, o, wm)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_mapr_generation3_ragged(precision):
    """MAPR with 642 directions on 5x8x20 cells (800: the last workgroup of each
    direction is partly filled), 2 steps."""
    wl, I0 = _case(n=(5, 8, 20), generation=3, pole_rows=1)
    wm = _mapr(wl, precision)
    _say(f"torus_ks mapr {precision} g3 5x8x20 2 steps")
    g = gpu_run(wm, 2, precision=precision, I0=I0)
    o = oracle_run(wm, 2, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wm)
    else:
        _check_fp32(g, o)


def test_ks_mapr_flat_spherical():
    """M = 0 (flat space in ln r, theta, phi) with MAPR states, generation 2,
    zero-incoming outside, 3 steps, FP64."""
    wl, I0 = _case(n=(8, 10, 6), generation=2, pole_rows=1, M=0.0, a=0.0, r_in=2.0, r_out=9.0)
    wm = _mapr(wl)
    _say("flat spherical mapr fp64 8x10x6 g2 3 steps")
    g = gpu_run(wm, 3, I0=I0)
    o = oracle_run(wm, 3, I0=I0)
    _check_fp64(g, o, wm)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ks_mapr_generation0_pentagons(precision):
    """MAPR on the icosahedron (12 directions, all pentagons: five planes each,
    the padded sixth skipped), 6x8x10 cells, 3 steps."""
    wl, I0 = _case(n=(6, 8, 10), generation=0, pole_rows=1)
    wm = _mapr(wl, precision)
    _say(f"torus_ks mapr {precision} g0 6x8x10 3 steps")
    g = gpu_run(wm, 3, precision=precision, I0=I0)
    o = oracle_run(wm, 3, I0=I0)
    if precision == "fp64":
        _check_fp64(g, o, wm)
    else:
        _check_fp32(g, o)


def test_ks_mapr_generation4():
    """MAPR with 2562 directions (two-pass kernels), 4x6x70 cells, 1 step, FP64."""
    wl, I0 = _case(n=(4, 6, 70), generation=4, pole_rows=1)
    wm = _mapr(wl)
    _say("torus_ks mapr fp64 g4 4x6x70 1 step")
    g = gpu_run(wm, 1, I0=I0)
    o = oracle_run(wm, 1, I0=I0)
    _check_fp64(g, o, wm)
