"""torch.autograd.Functions around rt_step and its hand-written adjoints, with
step checkpointing.

RTSteps.apply(rt, I0, kappa_a, j, T, dt, nsteps, every, opac) advances I0 by
nsteps steps with the fixed-emissivity model (fluid at rest) and returns I_N;
backward returns dL/dI0, dL/dkappa_a and dL/dj (rt_step_adjoint).
RTStepsThermal.apply(rt, I0, T0, kappa_a, dt, nsteps, every, opac) does the same
for the bremsstrahlung model, returning (I_N, T_N) and, backward, dL/dI0,
dL/dT0 and dL/dkappa_a (rt_step_adjoint_thermal).
Memory: the state is kept every `every` steps (nsteps/every checkpoints);
during the backward pass one segment of `every` states is recomputed at a
time.  All work runs in the HIP library; torch only holds the buffers.
"""
import torch


class RTSteps(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rt, I0, kappa_a, j, T, dt, nsteps, every, opac):
        rt.set_opacities("fixed_emissivity", kappa_a=kappa_a.detach().contiguous(),
                         j=j.detach().contiguous(), **opac)
        I = I0.detach().clone()
        T = T.detach().clone()
        ckpts = []
        for k in range(nsteps):
            if k % every == 0:
                ckpts.append(I.clone())
            rt.step(I, T, dt, 1)
        fctx.rt, fctx.dt, fctx.nsteps, fctx.every = rt, dt, nsteps, every
        fctx.save_for_backward(T, *ckpts)
        return I

    @staticmethod
    def backward(fctx, gI):
        rt, dt, nsteps, every = fctx.rt, fctx.dt, fctx.nsteps, fctx.every
        T, *ckpts = fctx.saved_tensors
        g = gI.detach().to(rt.intensity_dtype).contiguous().clone()
        gk = torch.zeros(rt.nc, dtype=torch.float64, device=g.device)
        gj = torch.zeros(rt.nc, dtype=torch.float64, device=g.device)
        for seg in reversed(range(len(ckpts))):
            k0 = seg * every
            k1 = min(nsteps, k0 + every)
            states = [ckpts[seg]]
            Tw = T.clone()
            for _ in range(k0, k1 - 1):
                I = states[-1].clone()
                rt.step(I, Tw, dt, 1)
                states.append(I)
            for I_k in reversed(states):
                g = rt.step_adjoint(I_k, T, dt, g, g, g_kappa_a=gk, g_j=gj)
        return None, g, gk, gj, None, None, None, None, None


class RTStepsThermal(torch.autograd.Function):
    """RTStepsThermal.apply(rt, I0, T0, kappa_a, dt, nsteps, every, opac) advances
    (I0, T0) by nsteps steps of the bremsstrahlung model (fluid at rest; kappa_a
    is the per-cell factor of its absorption opacity) and returns (I_N, T_N).
    Backward returns dL/dI0, dL/dT0 and dL/dkappa_a through rt_step_adjoint_thermal;
    (I, T) are kept every `every` steps and each segment is recomputed once."""

    @staticmethod
    def forward(fctx, rt, I0, T0, kappa_a, dt, nsteps, every, opac):
        rt.set_opacities("brems", kappa_a=kappa_a.detach().contiguous(), **opac)
        I = I0.detach().clone()
        T = T0.detach().clone()
        ckpts = []
        for k in range(nsteps):
            if k % every == 0:
                ckpts.extend([I.clone(), T.clone()])
            rt.step(I, T, dt, 1)
        fctx.rt, fctx.dt, fctx.nsteps, fctx.every = rt, dt, nsteps, every
        fctx.save_for_backward(*ckpts)
        return I, T

    @staticmethod
    def backward(fctx, gI, gT):
        rt, dt, nsteps, every = fctx.rt, fctx.dt, fctx.nsteps, fctx.every
        saved = fctx.saved_tensors
        g = gI.detach().to(rt.intensity_dtype).contiguous().clone()
        gt = (torch.zeros(rt.nc, dtype=torch.float64, device=g.device) if gT is None
              else gT.detach().to(torch.float64).contiguous().clone())
        gk = torch.zeros(rt.nc, dtype=torch.float64, device=g.device)
        nseg = len(saved) // 2
        for seg in reversed(range(nseg)):
            k0 = seg * every
            k1 = min(nsteps, k0 + every)
            states = [(saved[2 * seg], saved[2 * seg + 1])]
            for _ in range(k0, k1 - 1):
                I, T = states[-1][0].clone(), states[-1][1].clone()
                rt.step(I, T, dt, 1)
                states.append((I, T))
            for I_k, T_k in reversed(states):
                g, gt = rt.step_adjoint_thermal(I_k, T_k, dt, g, gt, gI_n=g, g_kappa_a=gk)
        return None, g, gt, gk, None, None, None, None
