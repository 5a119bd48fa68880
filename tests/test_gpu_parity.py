"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: plain FP64 form within 1e-12 relative of the oracle (element by
element); FP32 transport form within 1e-5 relative (rel-L2) in J and R^(ab)
and in T.  Workloads come from the seeded generators in `workloads`.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from runners import (J_of, gpu_context, gpu_initial, gpu_run, moments_error, moving_fluid,
                     oracle_run, patch, rel_l2, rel_max)

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _say(msg):
    print(msg, flush=True)


def _check_fp64(g, o, tol=1e-12):
    assert rel_max(g["I"], o["I"]) < tol, rel_max(g["I"], o["I"])
    assert rel_max(g["T"], o["T"]) < tol, rel_max(g["T"], o["T"])
    for k in range(10):
        assert (g["R"][k] - o["R"][k]).abs().max() <= tol * o["R"][0].abs().max(), k


def _check_fp32(g, o, tol=1e-5):
    assert rel_l2(J_of(g["R"]), J_of(o["R"])) < tol
    assert moments_error(g["R"], o["R"]) < tol
    assert rel_l2(g["T"], o["T"]) < tol


def test_blob_fp64_full_config():
    """16^3, generation 1 (42 directions, equal weights), Method 1, 10 steps."""
    wl = W.blob_flat()
    _say("blob_flat fp64 16^3 g1 10 steps")
    g = gpu_run(wl, 10)
    o = oracle_run(wl, 10)
    _check_fp64(g, o)


def test_blob_fp32_full_config():
    wl = W.blob_flat()
    _say("blob_flat fp32 16^3 g1 10 steps")
    g = gpu_run(wl, 10, precision="fp32")
    o = oracle_run(wl, 10)
    _check_fp32(g, o)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_brems_reduced(precision):
    """Method 2 (alpha^a = rho^2 T^-3.5, alpha^s = rho), generation 2, ragged
    10x9x12 periodic box, 5 steps."""
    wl = W.brems_flat(n=(10, 9, 12))
    _say(f"brems_flat {precision} 10x9x12 g2 5 steps")
    g = gpu_run(wl, 5, precision=precision)
    o = oracle_run(wl, 5)
    if precision == "fp64":
        _check_fp64(g, o)
    else:
        _check_fp32(g, o)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_brems_method3_reduced(precision):
    """Method 3 on the bremsstrahlung recipe, ragged 10x9x12 periodic box,
    generation 2, 5 steps; and a stiff variant (density x 6, T x 0.3: alpha dt
    up to ~1e4) where the semi-implicit opacity matters."""
    for stiff in (False, True):
        wl = W.brems_flat(n=(10, 9, 12))
        wl["model"] = "brems_m3"
        if stiff:
            wl["rho"] = wl["rho"] * 6.0
            wl["T"] = wl["T"] * 0.3
        _say(f"brems_m3 {precision} 10x9x12 g2 5 steps stiff={stiff}")
        g = gpu_run(wl, 5, precision=precision)
        o = oracle_run(wl, 5)
        assert o["failed"] == 0
        if precision == "fp64":
            _check_fp64(g, o)
        else:
            _check_fp32(g, o)


CASES = [
    # model, bc, limiter, moving, floor, weights
    ("kirchhoff_const", ("periodic",) * 3, "mc", False, False, "voronoi"),
    ("kirchhoff_const", ("zero_incoming", "outflow", "periodic"), "minmod", False, True, "equal"),
    ("brems", ("outflow", "zero_incoming", "zero_incoming"), "mc", True, False, "voronoi"),
    ("brems", ("periodic", "periodic", "outflow"), "mc", True, True, "voronoi"),
    ("fixed_emissivity", ("zero_incoming",) * 3, "mc", False, False, "voronoi"),
    ("fixed_emissivity", ("periodic", "outflow", "zero_incoming"), "minmod", True, True, "equal"),
    # Method 3 (total opacity semi-implicit)
    ("brems_m3", ("periodic",) * 3, "mc", False, False, "voronoi"),
    ("brems_m3", ("outflow", "zero_incoming", "periodic"), "minmod", True, True, "voronoi"),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_variants_fp64(case):
    model, bc, lim, moving, floor, weights = CASES[case]
    n = (7, 5, 9)
    rng = np.random.default_rng(100 + case)
    wl = W.brems_flat(n=n, generation=1, seed=200 + case)
    wl.update(model=model, bc=bc, weights=weights,
              kappa_a=rng.uniform(0.05, 4.0, n), kappa_s=rng.uniform(0.0, 2.0, n),
              j=rng.uniform(0.0, 1.0, n))
    if moving:
        wl["u"] = moving_fluid(n, 300 + case)
    if floor:
        rho = wl["rho"].copy()
        rho[rng.uniform(size=n) < 0.2] = 1e-5
        wl["rho"] = rho
    I0 = W.random_intensity(42, n, 400 + case, 0.0, 0.3)
    _say(f"variant {case}: {model} {bc} {lim} moving={moving} floor={floor}")
    g = gpu_run(wl, 3, I0=I0, limiter=lim, want_G=True)
    o = oracle_run(wl, 3, I0=I0, limiter={"mc": 0, "minmod": 1}[lim], want_G=True)
    _check_fp64(g, o)
    scale = o["G"].abs().max().item() + 1e-300
    assert (g["G"] - o["G"]).abs().max().item() < 1e-10 * scale


@pytest.mark.parametrize("case", range(len(CASES)))
def test_variants_fp32(case):
    # the FP32 kernels at rest and with a moving fluid (advection term) over the
    # boundary kinds, limiters and models, on two x tiles (the second ragged)
    model, bc, lim, moving, floor, weights = CASES[case]
    n = (9, 6, 70)  # two x tiles, a ragged one among them
    rng = np.random.default_rng(500 + case)
    wl = W.brems_flat(n=n, generation=1, seed=600 + case)
    wl.update(model=model, bc=bc, weights=weights,
              kappa_a=rng.uniform(0.05, 4.0, n), kappa_s=rng.uniform(0.0, 2.0, n),
              j=rng.uniform(0.0, 1.0, n))
    if moving:
        wl["u"] = moving_fluid(n, 700 + case)
    if floor:
        rho = wl["rho"].copy()
        rho[rng.uniform(size=n) < 0.2] = 1e-5
        wl["rho"] = rho
    I0 = W.random_intensity(42, n, 800 + case, 0.0, 0.3)
    _say(f"fp32 variant {case}: {model} {bc} {lim} moving={moving} floor={floor}")
    g = gpu_run(wl, 3, I0=I0, limiter=lim, want_G=True, precision="fp32")
    o = oracle_run(wl, 3, I0=I0, limiter={"mc": 0, "minmod": 1}[lim], want_G=True)
    _check_fp32(g, o)
    gI = g["I"].double()
    assert rel_l2(gI, o["I"]) < 1e-5, rel_l2(gI, o["I"])


@pytest.mark.parametrize("shape", [(1, 1, 37), (1, 6, 1), (3, 1, 70)])
def test_degenerate_axes(shape):
    wl = W.brems_flat(n=shape, generation=1, seed=7)
    _say(f"degenerate axes {shape}")
    g = gpu_run(wl, 3)
    o = oracle_run(wl, 3)
    _check_fp64(g, o)


@pytest.mark.parametrize("gen", [0, 1, 2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [(3, 7, 11), (4, 7, 20)])
def test_moments_mfma(gen, precision, n):
    """R^(ab) from the FP64 matrix cores vs the oracle's contraction, ragged
    cell counts: 231 cells (not a multiple of 4: FP32 takes the general path)
    and 560 (eight whole 64-cell waves through the FP32 16-byte-load kernel
    and a 48-cell tail through the general one)."""
    from oracle import step as st
    from oracle.grid import GeodesicGrid
    G = GeodesicGrid(gen)
    I0 = W.random_intensity(G.ns, n, 50 + gen)
    ctx = gpu_context(W.brems_flat(n=n, generation=gen, seed=1), precision)
    I = torch.as_tensor(I0).reshape(G.ns, -1).to(ctx.intensity_dtype).cuda().contiguous()
    J = torch.empty(ctx.nc, dtype=F64, device="cuda")
    _say(f"moments g{gen} {precision}")
    R = ctx.moments(I, J=J).cpu()
    Iref = I.double().cpu().reshape((G.ns,) + n)
    Ro = st.moments(Iref, G.n, G.w)
    assert (R - Ro).abs().max() < 1e-13 * Ro[0].abs().max()
    assert torch.allclose(J.cpu().reshape(n), Ro[0] / (4 * math.pi), rtol=1e-13)
    ctx.close()


def test_determinism_bitwise():
    wl = W.brems_flat(n=(12, 10, 8), generation=2, seed=3)
    a = gpu_run(wl, 3, precision="fp32")
    b = gpu_run(wl, 3, precision="fp32")
    assert torch.equal(a["I"], b["I"]) and torch.equal(a["T"], b["T"]) and torch.equal(a["R"], b["R"])


def test_restart_equals_continuous_run():
    """10 steps in one call equal 5 + (copy out, copy back) + 5 steps bitwise."""
    wl = W.brems_flat(n=(8, 8, 8), generation=1, seed=4)
    ctx = gpu_context(wl)
    I, T = gpu_initial(ctx, wl)
    I2, T2 = I.clone(), T.clone()
    ctx.step(I, T, wl["dt"], 10)
    ctx.step(I2, T2, wl["dt"], 5)
    I2, T2 = I2.cpu().cuda(), T2.cpu().cuda()
    ctx.step(I2, T2, wl["dt"], 5)
    assert torch.equal(I, I2) and torch.equal(T, T2)
    ctx.close()


@pytest.mark.parametrize("moving", [False, True])
def test_multi_step_call_returns_last_moments(moving):
    """One call of 3 steps equals 3 calls of one step bitwise, including the
    moments R and the 4-force G that the call returns for its last step."""
    n = (6, 5, 70)
    wl = W.brems_flat(n=n, generation=1, seed=9)
    if moving:
        wl["u"] = moving_fluid(n, 19)
    ctx = gpu_context(wl)
    I, T = gpu_initial(ctx, wl)
    I2, T2 = I.clone(), T.clone()
    R, G = (torch.zeros((k, ctx.nc), dtype=F64, device=I.device) for k in (10, 4))
    R2, G2 = torch.zeros_like(R), torch.zeros_like(G)
    _say(f"multi-step call, moving={moving}")
    ctx.step(I, T, wl["dt"], 3, G=G, R=R)
    for _ in range(3):
        ctx.step(I2, T2, wl["dt"], 1, G=G2, R=R2)
    torch.cuda.synchronize()
    assert torch.equal(I, I2) and torch.equal(T, T2)
    assert torch.equal(R, R2) and torch.equal(G, G2)
    ctx.close()


# --------------------------------------------------------------------------
# full-size flat workload (128^3 x 162), in the launch configuration of bench.py
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def brems_full():
    return W.brems_flat()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_sampled_cells(brems_full, precision):
    """One step at 128^3 x 162 on the GPU; for sampled cells the oracle
    recomputes the same step on a periodic 13^3 patch around the cell (the
    step's domain of dependence has radius 4), and the centre must agree."""
    wl = brems_full
    _say(f"full-size 128^3 g2 {precision}: GPU step")
    g = gpu_run(wl, 1, precision=precision)
    rng = np.random.default_rng(77)
    centers = [tuple(int(x) for x in rng.integers(0, 128, 3)) for _ in range(6)] + [(0, 0, 0), (127, 127, 127)]
    r = 6
    for cen in centers:
        sub = dict(wl)
        for key in ("rho", "T", "I0_iso"):
            sub[key] = patch(wl[key], cen, r)
        sub["n"] = (2 * r + 1,) * 3
        sub["xhi"] = sub["n"]
        sub["bc"] = ("outflow",) * 3
        o = oracle_run(sub, 1)
        gi = g["I"][:, cen[0], cen[1], cen[2]]
        oi = o["I"][:, r, r, r]
        gt, ot = g["T"][cen], o["T"][r, r, r]
        tol = 1e-12 if precision == "fp64" else 2e-6
        assert (gi - oi).abs().max() <= tol * oi.abs().max(), (cen, (gi - oi).abs().max())
        assert abs(gt - ot) <= tol * abs(ot), cen


def test_full_size_energy_conservation(brems_full):
    """Periodic box: sum over cells of (E + Y T) is conserved by every step."""
    wl = brems_full
    ctx = gpu_context(wl)
    I, T = gpu_initial(ctx, wl)
    Y = torch.as_tensor(wl["rho"], dtype=F64, device="cuda").reshape(-1) / (wl["gamma"] - 1)
    tot0 = (ctx.moments(I)[0].reshape(-1) + Y * T).sum().item()
    for _ in range(3):
        ctx.step(I, T, wl["dt"], 1)
        tot = (ctx.moments(I)[0].reshape(-1) + Y * T).sum().item()
        assert abs(tot - tot0) < 1e-12 * abs(tot0)
    ctx.close()


def test_full_size_fp32_vs_fp64_100_steps(brems_full):
    """North-star accuracy statement at the full 128^3 x 162 workload: the FP32
    transport form against the plain FP64 form (itself parity-pinned to the
    oracle above) after 100 steps, rel-L2 in J, R^(ab) and T."""
    wl = brems_full
    _say("full-size fp32 vs fp64, 100 steps")
    res = {}
    for prec in ("fp64", "fp32"):
        ctx = gpu_context(wl, prec)
        I, T = gpu_initial(ctx, wl)
        ctx.step(I, T, wl["dt"], 100)
        res[prec] = (ctx.moments(I).cpu(), T.cpu())
        del I
        ctx.close()
        torch.cuda.empty_cache()
    R64, T64 = res["fp64"]
    R32, T32 = res["fp32"]
    eJ = rel_l2(R32[0], R64[0])
    eR = moments_error(R32, R64)
    eT = rel_l2(T32, T64)
    _say(f"fp32 vs fp64 after 100 steps: J {eJ:.3e}  R {eR:.3e}  T {eT:.3e}")
    assert eJ < 1e-5 and eR < 1e-5 and eT < 1e-5


# --------------------------------------------------------------------------
# error paths (forced from the host)
# --------------------------------------------------------------------------
def test_failure_injection_newton_cap():
    """Method 1 with a one-iteration Newton cap cannot meet 1e-14: in debug
    mode every interacting cell is reported and keeps its old state."""
    from paper_2508_15532_amd import _native as N
    n = (4, 4, 4)
    wl = W.brems_flat(n=n, generation=1, seed=5)
    wl.update(model="kirchhoff_const", kappa_a=np.ones(n), kappa_s=np.zeros(n), newton_max_iter=1)
    ctx = gpu_context(wl)
    ctx.set_debug(1)
    I, T = gpu_initial(ctx, wl)
    st = ctx.step(I, T, wl["dt"], 1)
    assert st == N.RT_W_NEWTON
    assert ctx.newton_failures() == 2 * 64
    ctx.close()


def test_failure_injection_nonfinite():
    from paper_2508_15532_amd import RTError
    n = (4, 4, 4)
    wl = W.brems_flat(n=n, generation=1, seed=5)
    ctx = gpu_context(wl)
    ctx.set_debug(1)
    I, T = gpu_initial(ctx, wl)
    I[3, 5] = float("nan")
    with pytest.raises(RTError) as e:
        ctx.step(I, T, wl["dt"], 1)
    assert e.value.status == -5
    ctx.close()


def test_argument_errors():
    import paper_2508_15532_amd as P
    from paper_2508_15532_amd import RTError
    wl = W.brems_flat(n=(4, 4, 4), generation=1, seed=5)
    ctx = P.RTContext(wl["n"], wl["xlo"], wl["xhi"], 1)
    I = torch.zeros((42, 64), dtype=F64, device="cuda")
    T = torch.ones(64, dtype=F64, device="cuda")
    with pytest.raises(RTError) as e:
        ctx.step(I, T, 0.1)
    assert e.value.status == -2
    ctx.close()
    ctx = gpu_context(wl)
    with pytest.raises(RTError) as e:
        ctx.step(I, T, 10.0)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        ctx.step(I.float(), T, 0.1)
    ctx.close()


# --------------------------------------------------------------------------
# limits of the method and degenerate inputs
# --------------------------------------------------------------------------
def test_zero_steps_is_identity():
    wl = W.brems_flat(n=(6, 5, 7), generation=1, seed=9)
    ctx = gpu_context(wl)
    I, T = gpu_initial(ctx, wl)
    I0, T0 = I.clone(), T.clone()
    R = torch.full((10, ctx.nc), -7.0, dtype=F64, device="cuda")
    ctx.step(I, T, wl["dt"], 0, R=R)
    torch.cuda.synchronize()
    assert torch.equal(I, I0) and torch.equal(T, T0) and bool((R == -7.0).all())
    ctx.close()


@pytest.mark.parametrize("regime", ["vacuum", "opaque", "below_floor"])
def test_opacity_limits(regime):
    """Vacuum (tau = 0: pure upwind transport), optically thick cells
    (tau ~ 1e3 per step: the flux reduces to its diffusion form and the
    interaction pins I to B) and density below the floor everywhere (no
    interaction, T unchanged)."""
    n = (9, 6, 8)
    wl = W.brems_flat(n=n, generation=2, seed=13)
    wl["model"] = "kirchhoff_const"
    if regime == "vacuum":
        wl["kappa_a"] = np.zeros(n)
        wl["kappa_s"] = np.zeros(n)
    elif regime == "opaque":
        wl["kappa_a"] = np.full(n, 2.0e3)
        wl["kappa_s"] = np.full(n, 5.0e2)
        wl["rho"] = np.ones(n)
    else:
        wl["kappa_a"] = np.ones(n)
        wl["kappa_s"] = np.ones(n)
        wl["rho"] = np.full(n, 1e-4)
    I0 = W.random_intensity(162, n, 21, 0.2, 1.2)
    _say(f"opacity limit {regime}")
    g = gpu_run(wl, 3, I0=I0)
    o = oracle_run(wl, 3, I0=I0)
    _check_fp64(g, o)
    if regime == "below_floor":
        assert torch.equal(g["T"], torch.as_tensor(wl["T"], dtype=F64))


def test_generation3_step():
    """642 directions (generation 3), ragged 6 x 5 x 7 box, outflow and
    zero-incoming sides."""
    wl = W.brems_flat(n=(6, 5, 7), generation=3, seed=17)
    wl["bc"] = ("outflow", "zero_incoming", "periodic")
    wl["bc_hi"] = ("zero_incoming", "outflow", "periodic")
    _say("generation 3 step, 6x5x7")
    g = gpu_run(wl, 2)
    o = oracle_run(wl, 2)
    _check_fp64(g, o)
