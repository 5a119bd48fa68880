"""Shared drivers for the parity tests: run one workload through the HIP
library (via the Python binding) and through the oracle, from the same
seeded inputs."""
import math

import numpy as np
import torch

import workloads as W

F64 = torch.float64


def gpu_context(wl, precision="fp64", limiter="mc", cfl=0.4):
    import paper_2508_15532_amd as P
    if wl.get("metric") == "kerr_schild":
        ctx = P.RTContext(wl["n"], wl["xlo"], wl["xhi"], wl["generation"], weights=wl["weights"],
                          precision=precision, bc=wl["bc"], bc_hi=wl.get("bc_hi"), limiter=limiter,
                          coords="logr_theta_phi", pole_zero_rows=wl["pole_rows"],
                          n0_cut=wl["n0_cut"], angular_recon=wl.get("angular_recon", "donor"))
        ctx.set_metric("kerr_schild", M=wl["M"], a=wl["a"], cfl=wl.get("cfl", cfl))
    else:
        ctx = P.RTContext(wl["n"], wl["xlo"], wl["xhi"], wl["generation"], weights=wl["weights"],
                          precision=precision, bc=wl["bc"], bc_hi=wl.get("bc_hi"), limiter=limiter)
        ctx.set_metric("flat", cfl=cfl)
    dev = torch.device("cuda", 0)

    def t(x):
        return None if x is None else torch.as_tensor(np.ascontiguousarray(x), dtype=F64).to(dev)

    ctx.set_opacities(wl["model"], t(wl["rho"]), u=t(wl.get("u")), kappa_a=t(wl.get("kappa_a")),
                      kappa_s=t(wl.get("kappa_s")), j=t(wl.get("j")), gamma=wl["gamma"],
                      C_a=wl.get("C_a", 1.0), C_s=wl.get("C_s", 1.0),
                      newton_max_iter=wl.get("newton_max_iter", 50))
    return ctx


def gpu_initial(ctx, wl, I0=None):
    dev = torch.device("cuda", 0)
    if I0 is None:
        iso = torch.as_tensor(np.ascontiguousarray(wl["I0_iso"]), dtype=F64, device=dev)
        I = iso.reshape(1, -1).expand(ctx.ns, -1).to(ctx.intensity_dtype).contiguous()
    else:
        I = torch.as_tensor(np.ascontiguousarray(I0), dtype=F64).reshape(ctx.ns, -1).to(dev)
        I = I.to(ctx.intensity_dtype).contiguous()
    T = torch.as_tensor(np.ascontiguousarray(wl["T"]), dtype=F64, device=dev).reshape(-1).contiguous()
    return I, T


def gpu_run(wl, steps, precision="fp64", I0=None, limiter="mc", want_G=False):
    ctx = gpu_context(wl, precision, limiter)
    I, T = gpu_initial(ctx, wl, I0)
    G = torch.zeros((4, ctx.nc), dtype=F64, device=I.device) if want_G else None
    for _ in range(steps):
        ctx.step(I, T, wl["dt"], 1, G=G)
    R = ctx.moments(I)
    torch.cuda.synchronize()
    shape = tuple(wl["n"])
    out = dict(I=I.double().cpu().reshape((ctx.ns,) + shape), T=T.cpu().reshape(shape),
               R=R.cpu().reshape((10,) + shape))
    if want_G:
        out["G"] = G.cpu().reshape((4,) + shape)
    ctx.close()
    return out


def oracle_problem(wl, limiter=0):
    from oracle.setup import build_flat, build_ks
    if wl.get("metric") == "kerr_schild":
        pb, I, T, _ = build_ks(wl, limiter=limiter)
        return pb, I, T
    return build_flat(wl, limiter=limiter)


def oracle_run(wl, steps, I0=None, limiter=0, want_G=False):
    from oracle import step as st
    pb, I, T = oracle_problem(wl, limiter)
    if I0 is not None:
        I = torch.as_tensor(I0, dtype=F64).reshape(I.shape).clone()
    G = None
    for _ in range(steps):
        if want_G:
            I, T, G = st.step(pb, I, T, wl["dt"], want_G=True)
        else:
            I, T = st.step(pb, I, T, wl["dt"])
    g = pb.geo.grid
    out = dict(I=I, T=T, R=st.moments(I, g.n, g.w))
    if want_G:
        out["G"] = G
    out["failed"] = sum(pb.failed)
    return out


def rel_l2(a, b):
    return float(torch.linalg.vector_norm(a - b) / max(torch.linalg.vector_norm(b).item(), 1e-300))


def rel_max(a, b):
    return float((a - b).abs().max() / max(b.abs().max().item(), 1e-300))


def moments_error(Ra, Rb):
    """max over the 10 components of ||dR^(ab)||_2 / ||R^00_ref||_2."""
    ref = torch.linalg.vector_norm(Rb[0]).item()
    return max(torch.linalg.vector_norm(Ra[k] - Rb[k]).item() for k in range(10)) / ref


def J_of(R):
    return R[0] / (4 * math.pi)


def moving_fluid(shape, seed, vmax=0.3):
    """Random subluminal coordinate 4-velocity u^mu [4, *shape] (flat space)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1, 1, (3,) + tuple(shape))
    v *= vmax / np.maximum(np.sqrt((v ** 2).sum(0)), 1e-12) * rng.uniform(0, 1, tuple(shape))
    g = 1.0 / np.sqrt(1 - (v ** 2).sum(0))
    return np.concatenate([g[None], g[None] * v])


def patch(field, center, radius):
    """Periodic cube of side 2*radius+1 around `center` from a [..., n1, n2, n3] array."""
    idx = [np.arange(c - radius, c + radius + 1) % n for c, n in zip(center, field.shape[-3:])]
    return field[..., idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]


def gpu_run_mg(wl, steps, precision="fp64", per_call=1, noalloc=False):
    """Multi-group workload on the GPU: I [G, Ns, *n], T, R and G (summed over
    the bins) of the last step; `per_call` steps per rt_step call."""
    ctx = gpu_context(wl, precision)
    dev = torch.device("cuda", 0)
    kag = torch.as_tensor(np.ascontiguousarray(wl["kappa_a_groups"]), dtype=F64, device=dev)
    ctx.set_groups(wl["group_edges"], kag)
    G_ = kag.shape[0]
    iso = torch.as_tensor(np.ascontiguousarray(wl["I0_iso_groups"]), dtype=F64, device=dev).reshape(G_, 1, -1)
    I = iso.expand(G_, ctx.ns, ctx.nc).to(ctx.intensity_dtype).contiguous()
    T = torch.as_tensor(np.ascontiguousarray(wl["T"]), dtype=F64, device=dev).reshape(-1).contiguous()
    R = torch.zeros((10, ctx.nc), dtype=F64, device=dev)
    Gf = torch.zeros((4, ctx.nc), dtype=F64, device=dev)
    step = ctx.step_noalloc if noalloc else ctx.step
    done = 0
    while done < steps:
        k = min(per_call, steps - done)
        step(I, T, wl["dt"], k, G=Gf, R=R)
        done += k
    torch.cuda.synchronize()
    shape = tuple(wl["n"])
    out = dict(I=I.double().cpu().reshape((G_, ctx.ns) + shape), T=T.cpu().reshape(shape),
               R=R.cpu().reshape((10,) + shape), G=Gf.cpu().reshape((4,) + shape),
               fail=ctx.newton_failures())
    ctx.close()
    return out


def oracle_run_mg(wl, steps):
    """The oracle's multi-group steps; R and the 4-force of the last step's
    second interaction, summed over the bins."""
    from oracle import multigroup as mg
    from oracle.setup import build_flat_mg
    pb, ka, edges, I, T = build_flat_mg(wl)
    g = pb.geo.grid
    for _ in range(steps):
        I, T, It = mg.step_mg(pb, ka, edges, I, T, wl["dt"])
    R = mg.moments_mg(I, g.n, g.w)
    Gf = -(R[0:4] - mg.moments_mg(It, g.n, g.w)[0:4]) / wl["dt"]
    return dict(I=I, T=T, R=R, G=Gf, failed=sum(pb.failed))


__all__ = ["W", "gpu_context", "gpu_initial", "gpu_run", "oracle_run", "rel_l2", "rel_max",
           "moments_error", "J_of", "moving_fluid", "patch", "gpu_run_mg", "oracle_run_mg"]


def oracle_grad(wl, steps, I0, weights, limiter=0):
    """Reference gradient by torch autograd through the FP64 oracle:
    L = sum(weights * I_N); returns (dL/dI0, dL/dkappa_a, dL/dj)."""
    from oracle import step as st
    from oracle.setup import build_flat
    pb, _, T = build_flat(wl, limiter=limiter)
    ka = pb.kappa_a.clone().requires_grad_(True)
    jj = pb.j.clone().requires_grad_(True)
    pb.kappa_a, pb.j = ka, jj
    I = torch.as_tensor(I0, dtype=F64).reshape((pb.geo.grid.ns,) + tuple(wl["n"])).clone()
    I.requires_grad_(True)
    X = I
    for _ in range(steps):
        X, T = st.step(pb, X, T, wl["dt"])
    L = (torch.as_tensor(weights, dtype=F64).reshape(X.shape) * X).sum()
    gI, gk, gj = torch.autograd.grad(L, [I, ka, jj])
    return gI, gk, gj


def gpu_grad(wl, steps, I0, weights, precision="fp64", limiter="mc"):
    """dL/dI0, dL/dkappa_a, dL/dj from the HIP adjoint, for L = sum(weights * I_N)."""
    ctx = gpu_context(wl, precision, limiter)
    I, T = gpu_initial(ctx, wl, I0)
    states = []
    for _ in range(steps):
        states.append(I.clone())
        ctx.step(I, T, wl["dt"], 1)
    g = torch.as_tensor(np.ascontiguousarray(weights), dtype=F64).reshape(ctx.ns, -1)
    g = g.to(ctx.intensity_dtype).cuda().contiguous()
    gk = torch.zeros(ctx.nc, dtype=F64, device="cuda")
    gj = torch.zeros(ctx.nc, dtype=F64, device="cuda")
    for I_k in reversed(states):
        g = ctx.step_adjoint(I_k, T, wl["dt"], g, g, g_kappa_a=gk, g_j=gj)
    torch.cuda.synchronize()
    shape = tuple(wl["n"])
    out = (g.double().cpu().reshape((ctx.ns,) + shape), gk.cpu().reshape(shape), gj.cpu().reshape(shape))
    ctx.close()
    return out


def oracle_grad_thermal(wl, steps, I0, wI, wT, limiter=0):
    """Reference gradient by torch autograd through the FP64 oracle for the
    bremsstrahlung model: L = sum(wI * I_N) + sum(wT * T_N); returns
    (dL/dI0, dL/dT0, dL/dkappa_a) with kappa_a the per-cell opacity factor."""
    from oracle import step as st
    from oracle.setup import build_flat
    pb, _, T0 = build_flat(wl, limiter=limiter)
    ka = (pb.kappa_a if pb.kappa_a is not None else pb.kappa_default()).clone().requires_grad_(True)
    pb.kappa_a = ka
    I = torch.as_tensor(I0, dtype=F64).reshape((pb.geo.grid.ns,) + tuple(wl["n"])).clone().requires_grad_(True)
    T = T0.clone().requires_grad_(True)
    X, Tx = I, T
    for _ in range(steps):
        X, Tx = st.step(pb, X, Tx, wl["dt"])
    L = (torch.as_tensor(wI, dtype=F64).reshape(X.shape) * X).sum() + \
        (torch.as_tensor(wT, dtype=F64).reshape(Tx.shape) * Tx).sum()
    return torch.autograd.grad(L, [I, T, ka])


def gpu_grad_thermal(wl, steps, I0, wI, wT, precision="fp64", limiter="mc"):
    """(dL/dI0, dL/dT0, dL/dkappa_a) from the HIP adjoint of the bremsstrahlung
    step, for L = sum(wI * I_N) + sum(wT * T_N)."""
    ctx = gpu_context(wl, precision, limiter)
    I, T = gpu_initial(ctx, wl, I0)
    states = []
    for _ in range(steps):
        states.append((I.clone(), T.clone()))
        ctx.step(I, T, wl["dt"], 1)
    gI = torch.as_tensor(np.ascontiguousarray(wI), dtype=F64).reshape(ctx.ns, -1).to(ctx.intensity_dtype)
    gI = gI.cuda().contiguous()
    gT = torch.as_tensor(np.ascontiguousarray(wT), dtype=F64).reshape(-1).cuda().contiguous()
    gk = torch.zeros(ctx.nc, dtype=F64, device="cuda")
    for I_k, T_k in reversed(states):
        gI, gT = ctx.step_adjoint_thermal(I_k, T_k, wl["dt"], gI, gT, gI_n=gI, g_kappa_a=gk)
    torch.cuda.synchronize()
    shape = tuple(wl["n"])
    out = (gI.double().cpu().reshape((ctx.ns,) + shape), gT.cpu().reshape(shape), gk.cpu().reshape(shape))
    ctx.close()
    return out
