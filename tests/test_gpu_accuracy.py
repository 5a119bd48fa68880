"""Error of the FP32 transport form against the FP64 oracle, per field, over
long runs of the benchmark recipes at reduced size.

The FP32 form keeps intensities and transport arithmetic in FP32 and the
interaction solve and all angular sums in FP64.  Its error against the FP64
oracle is stated per field as rel-L2 = ||x - x_ref||_2 / ||x_ref||_2 for J and
T, and for each component of R^(ab) as ||dR^(ab)||_2 / ||R^00_ref||_2, with the
1e-5 bar of the accuracy target.  The plain FP64 form is measured beside it.
With RT_ACCURACY_OUT set, the measured errors are written there as JSON.
"""
import json
import math
import os

import pytest
import torch

import workloads as W
from runners import J_of, gpu_run, oracle_run, rel_l2

pytestmark = pytest.mark.gpu
COMP = ["00", "01", "02", "03", "11", "12", "13", "22", "23", "33"]
_RECORD = {}


def _say(msg):
    print(msg, flush=True)


def _errors(g, o):
    ref = torch.linalg.vector_norm(o["R"][0]).item()
    out = {"J": rel_l2(J_of(g["R"]), J_of(o["R"])), "T": rel_l2(g["T"], o["T"])}
    for k, name in enumerate(COMP):
        out["R" + name] = torch.linalg.vector_norm(g["R"][k] - o["R"][k]).item() / ref
    out["max_abs_J_rel"] = float((J_of(g["R"]) - J_of(o["R"])).abs().max() / J_of(o["R"]).abs().max())
    return out


def _record(name, entry):
    from bench import sources_sha256
    _RECORD[name] = entry
    _RECORD["sources_sha256"] = sources_sha256()
    path = os.environ.get("RT_ACCURACY_OUT")
    if path:
        with open(path, "w") as f:
            json.dump(_RECORD, f, indent=1, sort_keys=True)


def _measure(name, wl, steps, desc):
    _say(f"{name}: {desc}, {steps} steps: oracle")
    o = oracle_run(wl, steps)
    _say(f"{name}: FP32 and FP64 forms on the GPU")
    e32 = _errors(gpu_run(wl, steps, precision="fp32"), o)
    e64 = _errors(gpu_run(wl, steps, precision="fp64"), o)
    _record(name, {"workload": desc, "steps": steps, "fp32_vs_oracle": e32, "fp64_vs_oracle": e64})
    _say(f"{name}: FP32 rel-L2 J {e32['J']:.2e} T {e32['T']:.2e} "
         f"R max {max(e32['R' + c] for c in COMP):.2e}; FP64 J {e64['J']:.2e}")
    for field in ["J", "T"] + ["R" + c for c in COMP]:
        assert e32[field] < 1e-5, (field, e32[field])
        assert e64[field] < 1e-10, (field, e64[field])
    return e32


def test_fp32_error_flat_brems_100_steps():
    """The flat bremsstrahlung recipe (lognormal rho, T ~ U[0.5, 2], Method 2,
    scattering, periodic) on 20^3 cells x 162 directions, 100 steps."""
    wl = W.brems_flat(n=20, generation=2)
    _measure("flat_brems_20^3_g2", wl, 100,
             "flat 20^3 x 162, lognormal rho, T~U[0.5,2], alpha^a=rho^2 T^-3.5, alpha^s=rho, periodic")


@pytest.mark.parametrize("recon", ["donor", "mapr"])
def test_fp32_error_torus(recon):
    """The a = 0.9 Kerr-Schild torus recipe (Keplerian flow, Method 2, I0 = 0,
    zero-incoming outside, rows next to the axis zeroed) on 32x16x8 cells x 162
    directions: 50 steps with donor-cell angular states, 10 with MAPR (the
    oracle takes the FP32 form's tie band for the FP32 comparison; the FP64
    comparison uses the FP64 band)."""
    wl = W.torus_ks(n=(32, 16, 8), generation=2)
    wl["angular_recon"] = recon
    from oracle.setup import build_ks
    wl["dt"] = build_ks(wl)[3]
    steps = 50 if recon == "donor" else 10
    desc = f"Kerr-Schild a=0.9 torus 32x16x8 x 162, {recon} angular states"
    if recon == "donor":
        _measure(f"torus_{recon}_32x16x8_g2", wl, steps, desc)
        return
    _say(f"torus mapr: {steps} steps: oracle (FP32 and FP64 tie bands)")
    o32 = oracle_run(dict(wl, mapr_tie_rtol=1e-4), steps)
    o64 = oracle_run(wl, steps)
    e32 = _errors(gpu_run(wl, steps, precision="fp32"), o32)
    e64 = _errors(gpu_run(wl, steps, precision="fp64"), o64)
    _record(f"torus_{recon}_32x16x8_g2", {"workload": desc, "steps": steps, "fp32_vs_oracle": e32,
                                         "fp64_vs_oracle": e64})
    _say(f"torus mapr: FP32 rel-L2 J {e32['J']:.2e} T {e32['T']:.2e}; FP64 J {e64['J']:.2e}")
    for field in ["J", "T"] + ["R" + c for c in COMP]:
        assert e32[field] < 1e-5, (field, e32[field])
        assert e64[field] < 1e-10, (field, e64[field])
    assert math.isfinite(e32["max_abs_J_rel"])
