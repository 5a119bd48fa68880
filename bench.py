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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
MFMA_F64_PEAK_TFS = 78.6       # MI355X published dense FP64 matrix-core rate
CSRC = os.path.join(ROOT, "paper_2508_15532_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def algorithmic_bytes(kind, elem, ns, nc):
    """Bytes a launch of each kernel must move at minimum (its inputs read once
    and its outputs written once), per launch over the whole grid."""
    cd = ns * nc
    if kind == "stage1":       # read I^n, write I~; per cell: map, T, rho in; T*, map out
        return 2 * elem * cd + 56 * nc
    if kind == "stage2":       # read I*, I^n, write I~; per cell: 2 maps, T, T*, rho in; T, map, R out
        return 3 * elem * cd + 160 * nc
    if kind == "materialize":  # read I~, write I; per cell: map
        return 2 * elem * cd + 16 * nc
    if kind == "moments":      # read I, write 10 components
        return elem * cd + 80 * nc
    raise KeyError(kind)


def step_algorithmic_bytes(elem, ns, nc):
    """Per step, what the method itself must move: stage 1 reads I^n and writes
    I*, stage 2 reads I* and I^n and writes I^(n+1) (5 intensity transfers per
    cell-direction), plus R (80 B per cell)."""
    return 5 * elem * ns * nc + 80 * nc


def make_inputs(wl, ctx, torch):
    dev = torch.device("cuda", 0)

    def t(x):
        return None if x is None else torch.as_tensor(x, dtype=torch.float64).reshape(-1).to(dev)
    rho, T, u = t(wl["rho"]), t(wl["T"]), t(wl.get("u"))
    ctx.set_opacities(wl["model"], rho, u=u, gamma=wl["gamma"], C_a=wl["C_a"], C_s=wl["C_s"])
    if wl.get("metric") == "kerr_schild":
        I0 = torch.as_tensor(wl["I0_iso"], dtype=torch.float64).reshape(-1).to(dev)
    else:
        I0 = T ** 4 / (4 * math.pi)
    I = I0.reshape(1, -1).expand(ctx.ns, -1).to(ctx.intensity_dtype).contiguous()
    R = torch.empty((10, ctx.nc), dtype=torch.float64, device=dev)
    G = torch.empty((4, ctx.nc), dtype=torch.float64, device=dev)
    return (rho, u, G), I, T, R


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
    ns, nc = ctx.ns, ctx.nc
    ctx.close()
    del I, T, R, G, keep
    torch.cuda.empty_cache()
    return dict(wall=wall, ktimes=ktimes, ns=ns, nc=nc, finite=ok,
                elem=4 if precision == "fp32" else 8)


def sources_sha256():
    """Hash of every kernel and host source of the library (sorted by name)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp", ".hpp")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def traffic_for(kernel, elem):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        if rec.get("sources_sha256") != sources_sha256():
            return None
        return rec["per_launch_bytes"].get(f"{kernel}_{'fp32' if elem == 4 else 'fp64'}")
    except (OSError, KeyError, ValueError):
        return None


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
                    help="skip the large turbulent-torus line (384x192x128 x 642, FP32, 3 steps)")
    ap.add_argument("--moments-only", action="store_true",
                    help="only time rt_moments on the 128^3 x 162 field (FP32 and FP64) and print it")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
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
    # roofline of the dominant kernel, from HIP events over the timed region
    kt = {k: v for k, v in r["ktimes"].items() if v[0] > 0}
    dom = max(kt, key=lambda k: kt[k][1])
    launches, tot_ms = kt[dom]
    avg_s = tot_ms / launches / 1e3
    abytes = algorithmic_bytes(dom, r["elem"], r["ns"], r["nc"])
    achieved = abytes / avg_s / 1e9
    traffic = traffic_for(dom, r["elem"])
    step_bytes = step_algorithmic_bytes(r["elem"], r["ns"], r["nc"])
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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                     "kernel_avg_ms": avg_s * 1e3,
                     "step_frac": step_bytes * args.steps / r["wall"] / 1e9 / HBM_PEAK_GBS},
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in r["ktimes"].items() if v[0]},
    }
    for prec, rr in res.items():
        out[f"value_{prec}"] = rr["ns"] * rr["nc"] * args.steps / rr["wall"]
        out[f"ms_per_step_{prec}"] = 1e3 * rr["wall"] / args.steps
        if not rr["finite"]:
            out["error"] = f"non-finite moments in the {prec} run"
    if multi is not None:
        # the interaction map of intermediate steps stays lazy, R only for the last
        out["value_fp32_k_steps_one_call"] = multi["ns"] * multi["nc"] * args.steps / multi["wall"]
        out["ms_per_step_fp32_k_steps_one_call"] = 1e3 * multi["wall"] / args.steps
    if "fp32" in res and "fp64" in res:
        out["speedup_fp32_over_fp64"] = out["value_fp32"] / out["value_fp64"]
    if not args.no_torus:
        # curved geometry: the a = 0.9 Kerr-Schild torus, FP32 transport form
        print("bench: torus_ks fp32 256x128x64 x 162", file=sys.stderr, flush=True)
        tw = W.torus_ks()
        tr = run_form(tw, "fp32", args.steps, args.warmup, torch, P, per_call=True)
        out["torus_ks"] = {
            "workload": "Kerr-Schild a=0.9 torus, (ln r, theta, phi) 256x128x64 x 162 directions, "
                        "Keplerian flow, Method 2, FP32 transport",
            "value": tr["ns"] * tr["nc"] * args.steps / tr["wall"],
            "unit": "cell-direction updates/s",
            "ms_per_step": 1e3 * tr["wall"] / args.steps,
            "kernels_ms_per_step": {k: v[1] / args.steps for k, v in tr["ktimes"].items() if v[0]},
            "finite": tr["finite"]}
    if not args.no_mapr:
        # the same torus with MAPR angular edge states (two kernels in place of the
        # donor-cell angular kernel); algorithmic HBM bytes of the pair per
        # cell-direction: slope pass reads I, writes the 2-component slope; flux
        # pass reads I and both slope components, writes D (neighbour rows are
        # cache reuse, the per-(r, theta) coefficient rows are shared along phi)
        msteps = min(args.steps, 5)
        print(f"bench: torus_ks mapr fp32 256x128x64 x 162, {msteps} steps", file=sys.stderr, flush=True)
        mw = dict(W.torus_ks(), angular_recon="mapr")
        mr = run_form(mw, "fp32", msteps, 1, torch, P, per_call=True)
        kms = {k: v[1] / msteps for k, v in mr["ktimes"].items() if v[0]}
        entry = {
            "workload": "Kerr-Schild a=0.9 torus, 256x128x64 x 162 directions, MAPR angular states, "
                        "FP32 transport",
            "value": mr["ns"] * mr["nc"] * msteps / mr["wall"],
            "unit": "cell-direction updates/s",
            "ms_per_step": 1e3 * mr["wall"] / msteps,
            "kernels_ms_per_step": kms,
            "finite": mr["finite"]}
        n_ang, ms_ang = mr["ktimes"].get("angular", (0, 0.0))
        if n_ang:
            per_launch_ms = ms_ang / n_ang          # one evaluation per stage
            entry["angular_mapr_ms_per_launch"] = per_launch_ms
            entry["angular_mapr_hbm_GBps"] = 7 * mr["elem"] * mr["ns"] * mr["nc"] / (per_launch_ms * 1e-3) / 1e9
        out["torus_ks_mapr"] = entry
    if not args.no_big_torus:
        # the largest configuration: 6.1e9 cell-directions, 24 GB per FP32 intensity copy
        print("bench: turbulent torus fp32 384x192x128 x 642, 1 warmup + 3 timed steps",
              file=sys.stderr, flush=True)
        try:
            bw = W.torus_ks(n=(384, 192, 128), generation=3, sigma_ln=0.7, scattering=True)
            br = run_form(bw, "fp32", 3, 1, torch, P, per_call=True)
            out["torus_ks_384x192x128_g3"] = {
                "workload": "Kerr-Schild a=0.9 turbulent torus (lognormal sigma_ln 0.7, scattering), "
                            "(ln r, theta, phi) 384x192x128 x 642 directions, FP32 transport",
                "value": br["ns"] * br["nc"] * 3 / br["wall"],
                "unit": "cell-direction updates/s",
                "ms_per_step": 1e3 * br["wall"] / 3,
                "kernels_ms_per_step": {k: v[1] / 3 for k, v in br["ktimes"].items() if v[0]},
                "finite": br["finite"]}
        except Exception as e:  # reported in the line, the headline stands
            out["torus_ks_384x192x128_g3"] = {"error": f"{type(e).__name__}: {e}"}
    # the standalone moment contraction (inside rt_step R is formed in the
    # materialisation pass instead)
    print("bench: rt_moments 128^3 x 162", file=sys.stderr, flush=True)
    out["moments"] = [run_moments(wl, prec, 10, 2, torch, P) for prec in forms]
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
