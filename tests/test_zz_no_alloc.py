"""rt_step_noalloc (the entry point that allocates nothing: its step scratch is
the library's static per-device array) against rt_step on the same inputs.

Both entry points run the same kernels in the same order, and a stage's
results do not depend on the order its tiles run in, so the outputs must be
bitwise equal.  Two calls in a row on one device, the second with a smaller
grid (the scratch keeps the first call's contents), then a grid too large for
the scratch, which must be rejected before any device work.
"""
import numpy as np
import pytest
import torch

import workloads as W
from runners import gpu_context, gpu_initial

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _say(msg):
    print(msg, flush=True)


def _run(wl, steps, noalloc, precision, I0=None):
    ctx = gpu_context(wl, precision)
    I, T = gpu_initial(ctx, wl, I0)
    R = torch.zeros((10, ctx.nc), dtype=F64, device=I.device)
    G = torch.zeros((4, ctx.nc), dtype=F64, device=I.device)
    dt = wl.get("dt") or ctx.dt_max
    if noalloc:
        ctx.step_noalloc(I, T, dt, steps, G=G, R=R)
        ctx.step_noalloc(I, T, dt, 1, G=G, R=R)
    else:
        ctx.step(I, T, dt, steps, G=G, R=R)
        ctx.step(I, T, dt, 1, G=G, R=R)
    torch.cuda.synchronize()
    out = dict(I=I.cpu(), T=T.cpu(), R=R.cpu(), G=G.cpu())
    ctx.close()
    return out


def _same(a, b, what):
    for k in a:
        assert torch.equal(a[k], b[k]), (what, k, float((a[k].double() - b[k].double()).abs().max()))


def _torus_mapr():
    wl = W.torus_ks(n=(12, 16, 8), a=0.9, generation=1)
    wl["pole_rows"] = 2
    wl["angular_recon"] = "mapr"
    return wl, W.random_intensity(42, (12, 16, 8), 11, 0.5, 1.5)


def test_noalloc_matches_rt_step_two_calls_second_smaller():
    # call 1: flat 24^3 x 162 FP32 (about 10 MB of scratch), fluid at rest,
    # bremsstrahlung opacities
    flat = W.brems_flat(n=24, generation=2, seed=31)
    _say("noalloc call 1: flat 24^3 x 162 fp32, 2 steps + 1")
    a = _run(flat, 2, True, "fp32")
    b = _run(flat, 2, False, "fp32")
    _same(a, b, "flat fp32")
    # call 2: a smaller curved grid, FP64 with MAPR angular states (intensity,
    # angular divergence and slopes in the scratch)
    wl, I0 = _torus_mapr()
    _say("noalloc call 2: torus 12x16x8 x 42 fp64 mapr, 2 steps + 1")
    a = _run(wl, 2, True, "fp64", I0)
    b = _run(wl, 2, False, "fp64", I0)
    _same(a, b, "torus fp64 mapr")


def test_noalloc_rejects_grid_beyond_the_scratch():
    from paper_2508_15532_amd import RTError
    big = W.brems_flat(n=(64, 64, 64), generation=2, seed=32)   # ~185 MB of FP32 scratch
    ctx = gpu_context(big, "fp32")
    I, T = gpu_initial(ctx, big)
    with pytest.raises(RTError) as e:
        ctx.step_noalloc(I, T, big["dt"], 1)
    assert e.value.status == -1 and "static scratch" in str(e.value)
    ctx.close()
