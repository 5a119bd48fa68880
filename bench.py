"""Throughput of the gray transfer step on one MI355X.

One benchmark step is one pass of the whole hot path over the workload:
one rt_step call advancing one step (two transport stages, two implicit
interactions) that also returns R^(ab) of the new intensity and the 4-force.  Workload: flat 128^3 cells x 162
directions (geodesic generation 2), lognormal density (sigma_ln = 1, k^-2
random field), T ~ U[0.5, 2], alpha^a = rho^2 T^-3.5, alpha^s = rho, Method 2,
periodic, dt = 0.4; synthetic inputs from `workloads`, resident in HBM before
the timed region.  The FP32 transport form is the headline value; the plain
FP64 form runs the same workload and its rate is reported beside it.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
MFMA_F64_PEAK_TFS = 78.6       # MI355X published dense FP64 matrix-core rate
# VALU issue: 256 compute units x 4 SIMDs at 2.4 GHz; a 64-lane VALU
# instruction occupies a 16-lane SIMD for 4 cycles (no packed FP32 here), i.e.
# 39.3e12 lane-instructions/s (the 157.3 TFLOP/s FP32 figure counts FMA as two
# flops and packed pairs as two lanes)
SIMDS, CLOCK_HZ, VALU_CYCLES = 256 * 4, 2.4e9, 4
VALU_PEAK_TLANE = SIMDS * 16 * CLOCK_HZ / 1e12
CSRC = os.path.join(ROOT, "paper_2508_15532_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
ACCURACY_FILE = os.path.join(ROOT, "profiles", "accuracy_fp32_vs_oracle.json")


# Per-cell bytes the method moves besides the intensities (per stage): the
# fluid fields rho, kappa_a, kappa_s or j and u^mu (7 x 8 B), and the
# temperatures: stage 1 reads T^n and writes T*, stage 2 reads T^n and T* and
# writes T^(n+1).  R^(ab) (10 x 8 B) where it is formed.
FIELDS_B = 56
R_B = 80


def algorithmic_bytes(kind, elem, ns, nc, ng=0):
    """Bytes a launch of each kernel must move at minimum, counted as the
    method's own transfers: intensities (stage 1 reads I^n and writes I*,
    stage 2 reads I* and I^n and writes I^(n+1)), the per-cell temperatures and
    fluid fields, and R where it is formed.  The lazy interaction maps, halo
    re-reads and the angular-divergence scratch are implementation overhead and
    are not counted (they show in the measured traffic instead)."""
    cd = ns * nc
    if ng:
        # one bin of a multi-group step: the stage kernels read rho, kappa_s and
        # the bin's kappa_a and write the bin's E_-; the solve reads E_- and
        # kappa_a of every bin, rho, kappa_s and T_n and writes T and the
        # per-bin maps; the materialisation accumulates R
        if kind == "stage1":
            return 2 * elem * cd + 32 * nc
        if kind == "stage2":
            return 3 * elem * cd + 32 * nc
        if kind == "mg_solve":
            return (32 * ng + 32) * nc
        if kind == "materialize":
            return 2 * elem * cd + 2 * R_B * nc
        raise KeyError(kind)
    if kind == "stage1":
        return 2 * elem * cd + (16 + FIELDS_B) * nc
    if kind == "stage2":
        return 3 * elem * cd + (24 + FIELDS_B) * nc
    if kind == "materialize":  # read I~, write I^(n+1), R^(ab) out
        return 2 * elem * cd + R_B * nc
    if kind == "moments":      # read I, write 10 components
        return elem * cd + R_B * nc
    if kind == "angular":      # read I, write the angular divergence
        return 2 * elem * cd
    if kind == "adjoint":      # one reverse step: the forward step it re-runs plus its mirror
        return 2 * (5 * elem * cd + (40 + 2 * FIELDS_B) * nc)
    raise KeyError(kind)


def step_algorithmic_bytes(elem, ns, nc, ng=0):
    """Per step, what the method itself must move: 5 intensity transfers per
    cell-direction (stage 1: I^n in, I* out; stage 2: I*, I^n in, I^(n+1) out),
    per cell the temperatures (5 x 8 B) and the fluid fields of both stages
    (2 x 56 B), and R^(ab) of the new intensity (80 B).  With ng frequency
    bins: 5 transfers per cell-direction-bin, per cell and stage rho, kappa_s,
    T_n, T out and kappa_a of every bin, and R."""
    if ng:
        return 5 * elem * ng * ns * nc + (2 * (32 + 8 * ng) + R_B) * nc
    return 5 * elem * ns * nc + (40 + 2 * FIELDS_B + R_B) * nc


def make_inputs(wl, ctx, torch):
    dev = torch.device("cuda", 0)

    def t(x):
        return None if x is None else torch.as_tensor(x, dtype=torch.float64).reshape(-1).to(dev)
    rho, T, u = t(wl["rho"]), t(wl["T"]), t(wl.get("u"))
    ka, ks, j = t(wl.get("kappa_a")), t(wl.get("kappa_s")), t(wl.get("j"))
    ctx.set_opacities(wl["model"], rho, u=u, kappa_a=ka, kappa_s=ks, j=j, gamma=wl["gamma"], C_a=wl.get("C_a", 1.0),
                      C_s=wl.get("C_s", 1.0))
    if wl.get("metric") == "kerr_schild":
        I0 = torch.as_tensor(wl["I0_iso"], dtype=torch.float64).reshape(-1).to(dev)
    else:
        I0 = T ** 4 / (4 * math.pi)
    I = I0.reshape(1, -1).expand(ctx.ns, -1).to(ctx.intensity_dtype).contiguous()
    kag = None
    if wl.get("group_edges") is not None:
        # frequency bins: I [G, Ns, Nc], each bin isotropic with its share
        kag = torch.as_tensor(wl["kappa_a_groups"], dtype=torch.float64).reshape(len(wl["group_edges"]) - 1, -1)
        kag = kag.to(dev).contiguous()
        ctx.set_groups(wl["group_edges"], kag)
        iso = torch.as_tensor(wl["I0_iso_groups"], dtype=torch.float64).reshape(ctx.ng, 1, -1).to(dev)
        del I
        I = iso.expand(ctx.ng, ctx.ns, ctx.nc).to(ctx.intensity_dtype).contiguous()
    R = torch.empty((10, ctx.nc), dtype=torch.float64, device=dev)
    G = torch.empty((4, ctx.nc), dtype=torch.float64, device=dev)
    return (rho, u, G, ka, ks, j, kag), I, T, R


def make_context(wl, precision, P):
    if wl.get("metric") == "kerr_schild":
        ctx = P.RTContext(wl["n"], wl["xlo"], wl["xhi"], wl["generation"], weights=wl["weights"],
                          precision=precision, bc=wl["bc"], bc_hi=wl["bc_hi"],
                          coords="logr_theta_phi", pole_zero_rows=wl["pole_rows"], n0_cut=wl["n0_cut"],
                          angular_recon=wl.get("angular_recon", "donor"))
        dt = ctx.set_metric("kerr_schild", M=wl["M"], a=wl["a"], cfl=wl["cfl"])
        return ctx, dt
    ctx = P.RTContext(wl["n"], wl["xlo"], wl["xhi"], wl["generation"], weights=wl["weights"],
                      precision=precision, bc=wl["bc"])
    ctx.set_metric("flat", cfl=0.4)
    return ctx, wl["dt"]


def run_form(wl, precision, steps, warmup, torch, P, per_call=False):
    """Time `steps` steps of rt_step (moments of every step written to R);
    either one call advancing all steps, or one call per step."""
    ctx, dt = make_context(wl, precision, P)
    keep, I, T, R = make_inputs(wl, ctx, torch)
    G = keep[2]
    for _ in range(warmup):
        ctx.step(I, T, dt, 1, G=G, R=R)
    torch.cuda.synchronize()
    ctx.set_debug(2)                      # HIP events around every launch
    ctx.kernel_times()                    # reset the tally
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if per_call:
        for _ in range(steps):
            ctx.step(I, T, dt, 1, G=G, R=R)
    else:
        ctx.step(I, T, dt, steps, G=G, R=R)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ktimes = ctx.kernel_times()
    ctx.set_debug(0)
    ok = bool(torch.isfinite(R).all().item()) and bool(torch.isfinite(T).all().item())
    ns, nc, ng = ctx.ns, ctx.nc, ctx.ng
    ctx.close()
    del I, T, R, G, keep
    torch.cuda.empty_cache()
    return dict(wall=wall, ktimes=ktimes, ns=ns, nc=nc, ng=ng, finite=ok,
                elem=4 if precision == "fp32" else 8)


# The device code of each kernel kind: its own source file and the header that
# defines its arguments.  A counter record stays valid while these are unchanged.
KERNEL_SOURCES = {
    "stage1": ["stage.hip", "stage.hpp"],
    "stage2": ["stage.hip", "stage.hpp"],
    "materialize": ["stage.hip", "stage.hpp"],
    "angular": ["angular.hip", "stage.hpp"],
    "moments": ["kernels.hip"],
    "mg_solve": ["multigroup.hip"],
    "adjoint": ["adjoint.hip", "stage.hip", "stage.hpp"],
    "tr_adjoint": ["adjoint.hip"],
}


def _code_only(text):
    """Source text without comments and blank lines (a comment edit leaves the
    compiled kernel unchanged)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.split("\n"))
    return "\n".join(ln for ln in lines if ln.strip())


def sources_sha256(names=None):
    """Hash of the code (comments and blank lines removed) of the named library
    sources (default: every kernel and host source), in sorted order."""
    h = hashlib.sha256()
    if names is None:
        names = [n for n in os.listdir(CSRC) if n.endswith((".hip", ".cpp", ".hpp"))]
    for name in sorted(set(names)):
        h.update(name.encode())
        h.update(_code_only(open(os.path.join(CSRC, name), encoding="utf-8").read()).encode())
    return h.hexdigest()


def counters_for(wkey, kernel, elem):
    """Per-launch HBM bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by the
    plain-copy calibration) and VALU wave-instructions (SQ_INSTS_VALU) of
    `kernel` on workload `wkey`, from the committed counter record, if the
    record was taken on the current sources of that kernel; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        ent = rec["per_launch"].get(f"{wkey}/{kernel}_{'fp32' if elem == 4 else 'fp64'}")
        if ent is None or ent.get("sources_sha256") != sources_sha256(KERNEL_SOURCES[kernel]):
            return None
        return ent
    except (OSError, KeyError, ValueError):
        return None


def roofline_block(wkey, r):
    """Roofline of the dominant kernel of a timed run: its algorithmic bytes over
    its mean HIP-event duration against the HBM peak, and, where the committed
    counters of the current sources exist, its measured HBM traffic and VALU
    issue.  The bound is the busier of the two units: HBM (measured traffic, or
    the algorithmic bytes without counters, over the peak) or VALU issue
    (wave-instructions x 4 cycles over the SIMD-cycles of the launch)."""
    kt = {k: v for k, v in r["ktimes"].items() if v[0] > 0}
    dom = max(kt, key=lambda k: kt[k][1])
    launches, tot_ms = kt[dom]
    t = tot_ms / launches / 1e3
    abytes = algorithmic_bytes(dom, r["elem"], r["ns"], r["nc"], r.get("ng", 0))
    hbm = abytes / t / 1e9
    cnt = counters_for(wkey, dom, r["elem"]) or {}
    traffic, valu = cnt.get("bytes"), cnt.get("valu_insts")
    hbm_busy = (traffic if traffic else abytes) / t / 1e9 / HBM_PEAK_GBS
    blk = {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS,
           "traffic": traffic, "kernel": dom, "kernel_avg_ms": t * 1e3,
           "algorithmic_bytes": abytes, "hbm_frac_algorithmic": hbm / HBM_PEAK_GBS,
           "hbm_busy_measured": (traffic / t / 1e9 / HBM_PEAK_GBS) if traffic else None}
    if valu:
        valu_busy = valu * VALU_CYCLES / (SIMDS * CLOCK_HZ * t)
        blk["valu_busy"] = valu_busy
        if valu_busy > hbm_busy:
            # VALU issue bound: achieved = lane-instructions issued per second
            blk.update(bound="alu", achieved=valu * 64 / t / 1e12, peak=VALU_PEAK_TLANE,
                       unit="T VALU lane-instructions/s", frac=valu_busy)
    return blk


def copy_ceiling(torch):
    """Measured device-copy bandwidth: a plain 1 GiB device-to-device copy,
    5 repeats timed with HIP events after one warm-up (bytes read + written
    over the mean time)."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 5
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": 2 * (1 << 30) / (ms / 1e3) / 1e9, "ms": ms, "bytes_moved": 2 * (1 << 30),
            "frac_of_peak": 2 * (1 << 30) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def cpu_baseline(torch):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    a periodic 64^3 sub-box x 162 directions, two steps (about 10-30 s)."""
    import workloads as W
    from oracle import step as st
    from oracle.setup import build_flat
    n, nsteps = 64, 2
    wl = W.brems_flat(n=n)
    pb, I, T = build_flat(wl)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        I, T = st.step(pb, I, T, wl["dt"])
        R = st.moments(I, pb.geo.grid.n, pb.geo.grid.w)
    dt = time.perf_counter() - t0
    assert bool(torch.isfinite(R).all())
    cd = pb.geo.grid.ns * n ** 3 * nsteps
    return {"value": cd / dt, "unit": "cell-direction updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{nsteps} steps (rt_step + moments) of a periodic {n}^3 x {pb.geo.grid.ns} "
                      f"box drawn with the 128^3 workload's recipe ({dt:.1f} s)"}


def run_moments(wl, precision, launches, warmup, torch, P):
    """Time rt_moments (R^(ab) of a whole intensity field: the [cells x dirs] x
    [dirs x 10] FP64 contraction on MFMA) on the workload's initial field."""
    ctx, _ = make_context(wl, precision, P)
    keep, I, T, R = make_inputs(wl, ctx, torch)
    for _ in range(warmup):
        ctx.moments(I, R)
    torch.cuda.synchronize()
    ctx.set_debug(2)
    ctx.kernel_times()
    for _ in range(launches):
        ctx.moments(I, R)
    torch.cuda.synchronize()
    n, ms = ctx.kernel_times()["moments"]
    ctx.set_debug(0)
    ns, nc = ctx.ns, ctx.nc
    elem = 4 if precision == "fp32" else 8
    ctx.close()
    del I, T, R, keep
    torch.cuda.empty_cache()
    avg_s = ms / max(n, 1) / 1e3
    gbs = algorithmic_bytes("moments", elem, ns, nc) / avg_s / 1e9
    tflops = 2.0 * nc * ns * 10 / avg_s / 1e12
    return {"intensity": precision, "launches": n, "avg_ms": avg_s * 1e3,
            "achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "mfma_f64_TFLOPs": tflops, "mfma_frac": tflops / MFMA_F64_PEAK_TFS}


def step_frac(r, steps):
    """Fraction of the HBM peak that the method's own bytes per step
    (step_algorithmic_bytes) over the measured wall time per step amount to."""
    return step_algorithmic_bytes(r["elem"], r["ns"], r["nc"], r.get("ng", 0)) * steps / r["wall"] / 1e9 / HBM_PEAK_GBS


def line_entry(desc, wkey, r, steps):
    return {"workload": desc,
            "value": max(r.get("ng", 0), 1) * r["ns"] * r["nc"] * steps / r["wall"],
            "unit": "cell-direction updates/s",
            "steps": steps,
            "ms_per_step": 1e3 * r["wall"] / steps,
            "roofline": roofline_block(wkey, r),
            "step_hbm_frac": step_frac(r, steps),
            "kernels_ms_per_step": {k: v[1] / steps for k, v in r["ktimes"].items() if v[0]},
            "finite": r["finite"]}


def run_adjoint(torch, P):
    """The adjoint workload: flat 64^3 x 162, FP32, fixed emissivity
    (lognormal kappa_a, j ~ U[0, 1]), zero-incoming faces, 20 steps with the
    loss gradient flowing back through the checkpointed autograd Function
    (checkpoints every 5 steps: forward 20 steps, backward re-runs 15 steps and
    applies 20 adjoint steps).  Reports the time of a whole forward + backward
    and the mean duration of one rt_step_adjoint (HIP events)."""
    import workloads as W
    from paper_2508_15532_amd.autograd import RTSteps
    wl = W.adjoint_flat()
    ctx = P.RTContext(wl["n"], wl["xlo"], wl["xhi"], wl["generation"], weights=wl["weights"],
                      precision="fp32", bc=wl["bc"])
    ctx.set_metric("flat", cfl=0.4)
    dev = torch.device("cuda", 0)
    f64 = torch.float64
    rho = torch.as_tensor(wl["rho"], dtype=f64).reshape(-1).to(dev)
    opac = dict(rho=rho, kappa_s=torch.zeros_like(rho))
    ka = torch.as_tensor(wl["kappa_a"], dtype=f64).reshape(-1).to(dev)
    jj = torch.as_tensor(wl["j"], dtype=f64).reshape(-1).to(dev)
    I0 = torch.zeros((ctx.ns, ctx.nc), dtype=torch.float32, device=dev)
    T = torch.as_tensor(wl["T"], dtype=f64).reshape(-1).to(dev)
    dirs, w, _ = ctx.grid()
    wts = torch.zeros((ctx.ns,) + tuple(wl["n"]), dtype=torch.float32)
    wts[:, -1] = torch.as_tensor(w * np.maximum(dirs[:, 0], 0.0), dtype=torch.float32)[:, None, None]
    wts = wts.reshape(ctx.ns, -1).to(dev)

    def once():
        k = ka.clone().requires_grad_(True)
        j = jj.clone().requires_grad_(True)
        IN = RTSteps.apply(ctx, I0, k, j, T, wl["dt"], wl["steps"], wl["checkpoint"], opac)
        (IN * wts).sum().backward()
        return k.grad

    once()
    torch.cuda.synchronize()
    ctx.set_debug(2)
    ctx.kernel_times()
    t0 = time.perf_counter()
    g = once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.kernel_times()
    ctx.set_debug(0)
    n_adj, ms_adj = kt["adjoint"]
    ns, nc = ctx.ns, ctx.nc
    ctx.close()
    t = ms_adj / n_adj / 1e3
    ab = algorithmic_bytes("adjoint", 4, ns, nc)
    # the dominant kernel of a reverse step (the transport adjoint, two launches
    # per step) from the committed counters of the current adjoint sources
    cnt = counters_for("adjoint64", "tr_adjoint", 4) or {}
    dom = None
    if cnt:
        ts = cnt["avg_ms"] / 1e3
        dom = {"kernel": "k_tr_adj", "avg_ms": cnt["avg_ms"], "traffic": cnt["bytes"],
               "hbm_busy": cnt["bytes"] / ts / 1e9 / HBM_PEAK_GBS,
               "valu_busy": cnt["valu_insts"] * VALU_CYCLES / (SIMDS * CLOCK_HZ * ts)}
    return {"workload": "flat 64^3 x 162, FP32, fixed emissivity, 20 steps, checkpoints every 5, "
                        "gradient of the +x outgoing flux w.r.t. kappa_a and j",
            "forward_backward_ms": wall * 1e3,
            "adjoint_steps": n_adj,
            "adjoint_ms_per_step": t * 1e3,
            "adjoint_cell_direction_steps_per_s": ns * nc / t,
            "roofline": {"bound": "hbm", "achieved": ab / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ab / t / 1e9 / HBM_PEAK_GBS, "traffic": None, "kernel": "adjoint step",
                         "algorithmic_bytes": ab, "dominant_kernel": dom},
            "finite": bool(torch.isfinite(g).all().item())}


def run_only(which, steps, warmup, torch, P, W):
    """One of the secondary lines: the Kerr-Schild torus with donor-cell or
    MAPR angular states, the turbulent torus with 642 directions, the adjoint
    workload, the emitting ball, or the multi-group workload."""
    if which == "torus":
        # curved geometry: the a = 0.9 Kerr-Schild torus, FP32 transport form
        print(f"bench: torus_ks fp32 256x128x64 x 162, {steps} steps", file=sys.stderr, flush=True)
        tr = run_form(W.torus_ks(), "fp32", steps, warmup, torch, P, per_call=True)
        return line_entry("Kerr-Schild a=0.9 torus, (ln r, theta, phi) 256x128x64 x 162 directions, "
                          "Keplerian flow, Method 2, FP32 transport, donor-cell angular states",
                          "torus256", tr, steps)
    if which == "mapr":
        # the same torus with MAPR angular edge states (two kernels in place of
        # the donor-cell angular kernel)
        print(f"bench: torus_ks mapr fp32 256x128x64 x 162, {steps} steps", file=sys.stderr, flush=True)
        mr = run_form(dict(W.torus_ks(), angular_recon="mapr"), "fp32", steps, warmup, torch, P, per_call=True)
        return line_entry("Kerr-Schild a=0.9 torus, 256x128x64 x 162 directions, MAPR angular states, "
                          "FP32 transport", "torus256mapr", mr, steps)
    if which == "bigtorus":
        # the largest configuration: 6.1e9 cell-directions, 24 GB per FP32 intensity copy
        print(f"bench: turbulent torus fp32 384x192x128 x 642, {warmup} warmup + {steps} timed steps",
              file=sys.stderr, flush=True)
        bw = W.torus_ks(n=(384, 192, 128), generation=3, sigma_ln=0.7, scattering=True)
        br = run_form(bw, "fp32", steps, warmup, torch, P, per_call=True)
        return line_entry("Kerr-Schild a=0.9 turbulent torus (lognormal sigma_ln 0.7, scattering), "
                          "(ln r, theta, phi) 384x192x128 x 642 directions, FP32 transport",
                          "torus384g3", br, steps)
    if which == "adjoint":
        print("bench: adjoint 64^3 x 162 fp32, 20 steps, checkpoints every 5", file=sys.stderr, flush=True)
        return run_adjoint(torch, P)
    if which == "multigroup":
        # frequency bins: the flat recipe with 4 bins (5.4 GB per FP32 intensity copy)
        print(f"bench: multigroup fp32 128^3 x 162 x 4 bins, {steps} steps", file=sys.stderr, flush=True)
        mw = W.multigroup_flat()
        mr = run_form(mw, "fp32", steps, warmup, torch, P, per_call=True)
        out = line_entry("flat 128^3 x 162 directions x 4 frequency bins [0,1,3,9,inf), lognormal rho, "
                         "alpha^a_g = rho^2 (3, 1, 0.3, 0.1), alpha^s = rho, coupled temperature, FP32 "
                         "transport", "multigroup128", mr, steps)
        out["unit"] = "cell-direction-bin updates/s"
        return out
    if which == "sphere":
        # the curved-coordinate validation workload at the torus line's size
        print(f"bench: bright sphere fp32 256x128x64 x 162, {steps} steps", file=sys.stderr, flush=True)
        sw = W.bright_sphere(n=(256, 128, 64), generation=2)
        sr = run_form(sw, "fp32", steps, warmup, torch, P, per_call=True)
        return line_entry("emitting ball in flat space, (ln r, theta, phi) 256x128x64 x 162 directions, "
                          "fixed emissivity, FP32 transport", "sphere256", sr, steps)
    raise KeyError(which)


def accuracy_record():
    """Per-field error of the FP32 form against the FP64 oracle, as measured by
    tests/test_gpu_accuracy.py (RT_ACCURACY_OUT) and committed with its
    sources' hash; None when absent or taken on other sources."""
    try:
        with open(ACCURACY_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    rec["current_sources"] = rec.get("sources_sha256") == sources_sha256()
    return rec


# ---------------------------------------------------------------------------
# rocprofv3 summaries: the kernel-trace statistics and the counters of the
# same command (one counter set per run), per kernel, with the HBM bytes
# scaled by the plain-copy calibration.  The per-launch figures of the hot-path
# kernels are merged into profiles/traffic.json with the hash of their sources.
# ---------------------------------------------------------------------------
def _kernel_short(name):
    name = name.replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*$", "", name).replace("void ", "").strip()


def _kernel_kind(name):
    """(kind, fp32?) of a library kernel, or (None, None)."""
    f32 = "<float" in name or "_f32" in name
    if "k_stage<" in name:
        parts = [x.strip() for x in name.split("<", 1)[1].rstrip(">").split(",")]
        return ("stage2" if parts[3] == "true" else "stage1"), parts[0] == "float"
    for key, kind in (("k_materialize", "materialize"), ("k_moments", "moments"), ("k_angular", "angular"),
                      ("k_mapr", "angular"), ("k_mg_solve", "mg_solve"), ("k_tr_adj", "tr_adjoint")):
        if key in name:
            return kind, f32
    return None, None


def _read_profile(d):
    import csv
    import glob
    dur, cnt = {}, {}
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            dur[_kernel_short(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]) / 1e6,
                                             float(r["TotalDurationNs"]) / 1e6)
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            cnt.setdefault(_kernel_short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    return dur, {k: {n: sum(v) / len(v) for n, v in c.items()} for k, c in cnt.items()}


def summarize_profile(d, wkey, copy_dir, fp32_run):
    """Text summary of one profiled command (directory d: its kernel trace and
    counter runs) and the per-launch record of its library kernels."""
    # the per-kind source hashes the profiled run printed (its sources, not the tree's now)
    import glob
    logged = None
    for f in sorted(glob.glob(os.path.join(d, "*.log"))):
        for line in open(f, errors="replace"):
            if line.startswith("bench: sources "):
                logged = json.loads(line[len("bench: sources "):])
    if logged is None:
        raise SystemExit(f"no 'bench: sources' line in the logs of {d}")
    _, ccnt = _read_profile(copy_dir)
    cp = ccnt["__amd_rocclr_copyBuffer"]
    nbytes = float(1 << 30)
    ff, wf = nbytes / (cp["FETCH_SIZE"] * 1024), nbytes / (cp["WRITE_SIZE"] * 1024)
    dur, cnt = _read_profile(d)
    lines = [f"HBM byte scaling from a plain 1 GiB device copy: FETCH_SIZE x {ff:.3f}, WRITE_SIZE x {wf:.3f}", ""]
    per = {}
    for k in sorted(set(dur) | set(cnt), key=lambda k: -dur.get(k, (0, 0, 0))[2]):
        kind, f32 = _kernel_kind(k)
        if kind is None and dur.get(k, (0, 0, 0))[2] < 0.01 * sum(v[2] for v in dur.values()):
            continue  # small framework kernels
        c = cnt.get(k, {})
        lines.append(k)
        if k in dur:
            lines.append(f"    calls {dur[k][0]}  average {dur[k][1]:.4f} ms  total {dur[k][2]:.3f} ms")
        for n in sorted(c):
            lines.append(f"    {n:<16s} {c[n]:.5g}")
        if "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            rb, wb = c["FETCH_SIZE"] * 1024 * ff, c["WRITE_SIZE"] * 1024 * wf
            lines.append(f"    HBM bytes per launch (scaled): read {rb / 1e9:.4f} GB, written {wb / 1e9:.4f} GB")
            if "SQ_INSTS_VALU" in c and k in dur:
                busy = c["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * CLOCK_HZ * dur[k][1] / 1e3)
                lines.append(f"    VALU busy {busy:.3f}, HBM busy {(rb + wb) / (dur[k][1] / 1e3) / 1e9 / HBM_PEAK_GBS:.3f}"
                             " (of the trace's average duration)")
            if kind and kind not in logged:
                lines.append(f"    (no source hash of kind {kind} in the run's log: no per-launch record)")
            elif kind:
                key = f"{wkey}/{kind}_{'fp32' if (f32 or (kind in ('mg_solve', 'tr_adjoint') and fp32_run)) else 'fp64'}"
                e = per.setdefault(key, {"bytes": 0.0, "valu_insts": 0.0, "avg_ms": 0.0,
                                         "sources_sha256": logged[kind]})
                e["bytes"] += rb + wb
                e["valu_insts"] += c.get("SQ_INSTS_VALU", 0.0)
                e["avg_ms"] += dur.get(k, (0, 0.0, 0))[1]
        lines.append("")
    return "\n".join(lines), per, (ff, wf)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp32,fp64")
    ap.add_argument("--no-per-call", action="store_true",
                    help="skip the extra line with K steps advanced by one rt_step call")
    ap.add_argument("--no-torus", action="store_true",
                    help="skip the Kerr-Schild torus line (256x128x64 x 162, FP32)")
    ap.add_argument("--no-mapr", action="store_true",
                    help="skip the torus line with MAPR angular states (256x128x64 x 162, FP32)")
    ap.add_argument("--no-big-torus", action="store_true",
                    help="skip the large turbulent-torus line (384x192x128 x 642, FP32, 5 steps)")
    ap.add_argument("--no-sphere", action="store_true",
                    help="skip the curved-coordinate validation line (bright sphere 256x128x64 x 162, FP32)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint line (64^3 x 162 FP32, 20 steps, checkpoints every 5)")
    ap.add_argument("--no-multigroup", action="store_true",
                    help="skip the multi-group line (128^3 x 162 x 4 frequency bins, FP32)")
    ap.add_argument("--only", choices=["torus", "mapr", "bigtorus", "adjoint", "sphere", "multigroup"],
                    help="run only that line (for profiling) and print it as one JSON object")
    ap.add_argument("--moments-only", action="store_true",
                    help="only time rt_moments on the 128^3 x 162 field (FP32 and FP64) and print it")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print the summary of a profiled command's rocprofv3 output in DIR (no GPU) "
                         "and merge its per-launch counters into profiles/traffic.json; needs "
                         "--wkey and --copy-profile")
    ap.add_argument("--wkey", help="workload key of --summarize-profile")
    ap.add_argument("--copy-profile", metavar="DIR",
                    help="rocprofv3 output of the --calibrate-copy run (FETCH_SIZE and WRITE_SIZE)")
    ap.add_argument("--fp32-run", action="store_true", help="the profiled command ran the FP32 form")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.summarize_profile:
        text, per, factors = summarize_profile(args.summarize_profile, args.wkey, args.copy_profile,
                                               args.fp32_run)
        print(text)
        try:
            with open(TRAFFIC_FILE) as f:
                rec = json.load(f)
        except (OSError, ValueError):
            rec = {}
        rec["fetch_factor"], rec["write_factor"] = factors
        rec.setdefault("per_launch", {}).update(per)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
        return
    # the sources of every kernel kind, for the counter records of profiled runs
    print("bench: sources " + json.dumps({k: sources_sha256(v) for k, v in KERNEL_SOURCES.items()}),
          file=sys.stderr, flush=True)
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is designed but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2508_15532_amd as P
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    wl = W.brems_flat()
    forms = args.forms.split(",")
    if args.moments_only:
        print(json.dumps({"moments": [run_moments(wl, prec, 10, 2, torch, P) for prec in forms]}))
        return
    if args.only:
        print(json.dumps(run_only(args.only, args.steps, args.warmup, torch, P, W)))
        return
    res = {}
    for prec in forms:
        print(f"bench: {prec} 128^3 x 162, {args.warmup} warmup + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        res[prec] = run_form(wl, prec, args.steps, args.warmup, torch, P, per_call=True)
    multi = None
    if not args.no_per_call and "fp32" in forms:
        print("bench: fp32, all timed steps in one rt_step call", file=sys.stderr, flush=True)
        multi = run_form(wl, "fp32", args.steps, args.warmup, torch, P)
    head = "fp32" if "fp32" in res else forms[0]
    r = res[head]
    cd_per_step = r["ns"] * r["nc"]
    value = cd_per_step * args.steps / r["wall"]
    ms_per_step = 1e3 * r["wall"] / args.steps
    out = {
        "metric": "cell-direction updates/s for rt_step (FP32 vs FP64) + % HBM roofline",
        "value": value,
        "unit": "cell-direction updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "flat 128^3 x 162 directions (geodesic g2), lognormal rho, "
                               "T~U[0.5,2], alpha^a=rho^2 T^-3.5, alpha^s=rho, Method 2, periodic",
                   "form": "fp32 transport + fp64 interaction/moments" if head == "fp32" else "fp64",
                   "cells": r["nc"], "directions": r["ns"],
                   "step": "one rt_step call per step: predictor-corrector step incl. R^(ab) "
                           "and the 4-force of the new intensity",
                   "parallelism": "single GPU"},
        "roofline": roofline_block("flat128", r),
        "step_hbm_frac": step_frac(r, args.steps),
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in r["ktimes"].items() if v[0]},
    }
    for prec, rr in res.items():
        out[f"value_{prec}"] = rr["ns"] * rr["nc"] * args.steps / rr["wall"]
        out[f"ms_per_step_{prec}"] = 1e3 * rr["wall"] / args.steps
        out[f"roofline_{prec}"] = roofline_block("flat128", rr)
        out[f"step_hbm_frac_{prec}"] = step_frac(rr, args.steps)
        if not rr["finite"]:
            out["error"] = f"non-finite moments in the {prec} run"
    if multi is not None:
        # the interaction map of intermediate steps stays lazy, R only for the last
        out["value_fp32_k_steps_one_call"] = multi["ns"] * multi["nc"] * args.steps / multi["wall"]
        out["ms_per_step_fp32_k_steps_one_call"] = 1e3 * multi["wall"] / args.steps
    if "fp32" in res and "fp64" in res:
        out["speedup_fp32_over_fp64"] = out["value_fp32"] / out["value_fp64"]
    if not args.no_torus:
        out["torus_ks"] = run_only("torus", args.steps, args.warmup, torch, P, W)
    if not args.no_mapr:
        out["torus_ks_mapr"] = run_only("mapr", min(args.steps, 5), 1, torch, P, W)
    if not args.no_big_torus:
        try:
            out["torus_ks_384x192x128_g3"] = run_only("bigtorus", args.steps, 1, torch, P, W)
        except Exception as e:  # reported in the line, the headline stands
            out["torus_ks_384x192x128_g3"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_adjoint:
        out["adjoint"] = run_only("adjoint", 0, 0, torch, P, W)
    if not args.no_sphere:
        out["bright_sphere"] = run_only("sphere", min(args.steps, 10), 2, torch, P, W)
    if not args.no_multigroup:
        out["multigroup"] = run_only("multigroup", min(args.steps, 10), 2, torch, P, W)
    # the standalone moment contraction (inside rt_step R is formed in the
    # materialisation pass instead)
    print("bench: rt_moments 128^3 x 162", file=sys.stderr, flush=True)
    out["moments"] = [run_moments(wl, prec, 10, 2, torch, P) for prec in forms]
    out["device_copy_ceiling"] = copy_ceiling(torch)
    acc = accuracy_record()
    if acc is not None:
        out["accuracy_fp32_vs_oracle"] = acc
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
