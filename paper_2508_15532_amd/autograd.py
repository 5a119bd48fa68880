"""torch.autograd.Function around rt_step / rt_step_adjoint with step checkpointing.

RTSteps.apply(rt, I0, kappa_a, j, T, dt, nsteps, every, opac) advances I0 by
nsteps steps with the fixed-emissivity model (fluid at rest) and returns I_N.
Backward returns dL/dI0, dL/dkappa_a and dL/dj.  Memory: the intensity is
kept every `every` steps (nsteps/every checkpoints); during the backward pass
one segment of `every` states is recomputed at a time.  All work runs in the
HIP library; torch only holds the buffers.
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
