"""Hand-written adjoint (rt_step_adjoint, RTSteps autograd.Function) against
the oracle's reference gradient and FP64 finite differences."""
import numpy as np
import pytest
import torch

import workloads as W
from runners import gpu_context, gpu_grad, gpu_initial, oracle_grad

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _say(msg):
    print(msg, flush=True)


ADJ_CASES = [
    # bc, limiter, scattering
    (("zero_incoming",) * 3, "mc", False),
    (("zero_incoming",) * 3, "mc", True),
    (("periodic", "outflow", "zero_incoming"), "minmod", True),
    (("periodic",) * 3, "mc", False),
]


@pytest.mark.parametrize("case", range(len(ADJ_CASES)))
def test_adjoint_matches_oracle_gradient(case):
    """FP64 adjoint of 3 steps on a ragged 6x5x7 box vs autograd through the
    oracle, for L = sum(weights * I_N): dL/dI0, dL/dkappa_a, dL/dj."""
    bc, lim, scat = ADJ_CASES[case]
    n = (6, 5, 7)
    rng = np.random.default_rng(10 + case)
    wl = W.adjoint_flat(n=n, generation=1, seed=20 + case)
    wl["bc"] = bc
    if scat:
        wl["kappa_s"] = rng.uniform(0.0, 0.8, n)
    I0 = W.random_intensity(42, n, 30 + case, 0.0, 0.4)
    wts = rng.uniform(-1.0, 1.0, (42,) + n)
    _say(f"adjoint case {case}: {bc} {lim} scattering={scat}")
    gI, gk, gj = gpu_grad(wl, 3, I0, wts, limiter=lim)
    oI, ok, oj = oracle_grad(wl, 3, I0, wts, limiter={"mc": 0, "minmod": 1}[lim])
    for name, a, b in (("I", gI, oI), ("kappa_a", gk, ok), ("j", gj, oj)):
        err = (a - b).abs().max().item() / max(b.abs().max().item(), 1e-300)
        assert err < 1e-10, (name, err)


@pytest.mark.parametrize("n, bc", [((2, 3, 9), ("periodic", "periodic", "zero_incoming")),
                                   ((1, 5, 3), ("outflow", "periodic", "outflow")),
                                   ((9, 2, 5), ("zero_incoming", "periodic", "periodic"))])
def test_adjoint_short_lines_match_oracle_gradient(n, bc):
    """Lines shorter than a stencil (periodic lines of 2 and 3 cells wrap a face
    onto itself; a clamped line of one cell is its own ghost on both sides) and
    segments of the transport adjoint with a ragged end, FP64 against the
    oracle's autograd."""
    rng = np.random.default_rng(sum(n))
    wl = W.adjoint_flat(n=n, generation=1, seed=sum(n))
    wl["bc"] = bc
    wl["kappa_s"] = rng.uniform(0.0, 0.8, n)
    I0 = W.random_intensity(42, n, 3 + sum(n), 0.0, 0.4)
    wts = rng.uniform(-1.0, 1.0, (42,) + n)
    _say(f"adjoint short lines {n} {bc}")
    gI, gk, gj = gpu_grad(wl, 2, I0, wts)
    oI, ok, oj = oracle_grad(wl, 2, I0, wts)
    for name, a, b in (("I", gI, oI), ("kappa_a", gk, ok), ("j", gj, oj)):
        err = (a - b).abs().max().item() / max(b.abs().max().item(), 1e-300)
        assert err < 1e-10, (name, err)


def test_adjoint_fp32_matches_oracle_gradient():
    n = (6, 5, 7)
    rng = np.random.default_rng(5)
    wl = W.adjoint_flat(n=n, generation=1, seed=5)
    I0 = W.random_intensity(42, n, 6, 0.0, 0.4)
    wts = rng.uniform(0.0, 1.0, (42,) + n)
    gI, gk, gj = gpu_grad(wl, 3, I0, wts, precision="fp32")
    oI, ok, oj = oracle_grad(wl, 3, I0, wts)
    for name, a, b in (("I", gI, oI), ("kappa_a", gk, ok), ("j", gj, oj)):
        err = (a - b).abs().max().item() / max(b.abs().max().item(), 1e-300)
        assert err < 1e-5, (name, err)


def _outgoing_weights(ctx, n):
    """dL/dI_N of L = sum_(i2,i3) sum_s w_s max(n^x_s, 0) I_N(N1-1, i2, i3, s):
    the flux through the +x face read from the last interior layer."""
    dirs, w, _ = ctx.grid()
    wts = np.zeros((ctx.ns,) + tuple(n))
    wts[:, -1, :, :] = (w * np.maximum(dirs[:, 0], 0.0))[:, None, None]
    return wts


def test_adjoint_fd_full_size_checkpointed():
    """64^3 x 162, 20 steps, FP32 forward and adjoint through RTSteps (checkpoint
    every 5 steps) against FP64 central finite differences of the outgoing
    +x flux on 32 seeded cells near the +x face (relative 1e-4)."""
    from paper_2508_15532_amd.autograd import RTSteps
    wl = W.adjoint_flat()
    n = wl["n"]
    # FP32 gradient through the autograd Function
    ctx = gpu_context(wl, "fp32")
    I0, T = gpu_initial(ctx, wl)
    ka = torch.as_tensor(wl["kappa_a"], dtype=F64).reshape(-1).cuda().requires_grad_(True)
    jj = torch.as_tensor(wl["j"], dtype=F64).reshape(-1).cuda().requires_grad_(True)
    wts = torch.as_tensor(_outgoing_weights(ctx, n), dtype=torch.float32).reshape(ctx.ns, -1).cuda()
    opac = dict(rho=torch.as_tensor(wl["rho"], dtype=F64).reshape(-1).cuda(),
                kappa_s=torch.zeros(ctx.nc, dtype=F64, device="cuda"))
    _say("adjoint 64^3 fp32: forward + backward (20 steps, checkpoints every 5)")
    IN = RTSteps.apply(ctx, I0, ka, jj, T, wl["dt"], wl["steps"], wl["checkpoint"], opac)
    L = (IN * wts).sum()
    L.backward()
    gk, gj = ka.grad.cpu().reshape(n), jj.grad.cpu().reshape(n)
    ctx.close()
    # FP64 finite differences
    ctx = gpu_context(wl, "fp64")
    w64 = torch.as_tensor(_outgoing_weights(ctx, n), dtype=F64).reshape(ctx.ns, -1).cuda()

    def loss(kappa, j):
        ctx.set_opacities("fixed_emissivity", opac["rho"], kappa_a=kappa, kappa_s=opac["kappa_s"], j=j)
        I, T = gpu_initial(ctx, wl)
        ctx.step(I, T, wl["dt"], wl["steps"])
        return float((I * w64).sum().item())

    base_k = torch.as_tensor(wl["kappa_a"], dtype=F64).reshape(-1).cuda()
    base_j = torch.as_tensor(wl["j"], dtype=F64).reshape(-1).cuda()
    errs = []
    scale_k = scale_j = 0.0
    fds = []
    _say("adjoint 64^3: FP64 central differences on 32 cells")
    for (i1, i2, i3) in wl["probes"]:
        c = (int(i1) * n[1] + int(i2)) * n[2] + int(i3)
        # steps of 1e-6: at 1e-4 the perturbation crosses switch points of the
        # slope limiter in a few probe cells (the loss is only piecewise smooth)
        hk = 1e-6 * float(base_k[c])
        kp, km = base_k.clone(), base_k.clone()
        kp[c] += hk
        km[c] -= hk
        fk = (loss(kp, base_j) - loss(km, base_j)) / (2 * hk)
        jp, jm = base_j.clone(), base_j.clone()
        jp[c] += 1e-6
        jm[c] -= 1e-6
        fj = (loss(base_k, jp) - loss(base_k, jm)) / 2e-6
        fds.append((fk, fj, float(gk[i1, i2, i3]), float(gj[i1, i2, i3])))
        scale_k = max(scale_k, abs(fk))
        scale_j = max(scale_j, abs(fj))
    ctx.close()
    cell_rel = []
    for fk, fj, ak, aj in fds:
        errs.append(max(abs(ak - fk) / scale_k, abs(aj - fj) / scale_j))
        cell_rel.append((abs(ak - fk) / max(abs(fk), 1e-300), abs(aj - fj) / max(abs(fj), 1e-300), fk, fj))
    _say(f"max adjoint-vs-FD error over 32 cells, relative to the largest FD: {max(errs):.2e}")
    for k, (rk, rj, fk, fj) in enumerate(cell_rel):
        _say(f"  probe {k}: dL/dkappa {fk:+.4e} rel err {rk:.2e}; dL/dj {fj:+.4e} rel err {rj:.2e}")
    assert scale_k > 0 and scale_j > 0
    assert max(errs) < 1e-4
    # per cell: within 1e-4 of its own finite difference wherever the gradient
    # is at least 1% of the largest one; below that the FP32 rounding of the
    # forward and adjoint runs (about 2e-6 of the largest gradient) sets the
    # floor, and the bar is 1e-5 of the largest gradient in absolute terms
    for rk, rj, fk, fj in cell_rel:
        for rel, f, scale in ((rk, fk, scale_k), (rj, fj, scale_j)):
            if abs(f) >= 1e-2 * scale:
                assert rel < 1e-4, (rel, f, scale)
            else:
                assert rel * abs(f) < 1e-5 * scale, (rel, f, scale)
