"""Differentiable FLB run: torch.autograd.Function over the HIP forward and
hand-written adjoint kernels.

    rho_N = FLBRun.apply(delta_f0, rate_shear, kT, params, nsteps, checkpoint_every)

runs ``nsteps`` steps from the shifted populations ``delta_f0`` at a fixed
noise seed and returns the density after the final streaming,
rho_N(x) = rho0 + sum_i delta S_{N,i}(x - c_i), as an FP64 tensor.  The backward pass seeds
dL/dS_N from dL/drho_N, then walks the checkpoints (one every
``checkpoint_every`` steps) from last to first: it recomputes the states of a
segment with the forward kernel and applies the adjoint step kernel to each in
reverse, regenerating the same Philox noise (one library call; the recompute
of a segment runs beside the reverse sweep of the next on a second stream).  It returns dL/d(delta_f0),
dL/d(rate_shear) and dL/d(kT); the bulk and ghost rate derivatives are kept in
``FLBRun.last_grads``.
"""

import numpy as np
import torch

from .sim import Simulation


class FLBRun(torch.autograd.Function):
    last_grads = None

    @staticmethod
    def forward(ctx, delta_f0, rate_shear, kT, params, nsteps, checkpoint_every=20):
        p = params.with_(rate_shear=float(rate_shear), kT=float(kT), step0=0)
        sim = Simulation(p, device=delta_f0.device)
        sim.load_state(delta_f0.detach())
        ck = int(checkpoint_every)
        ckpts = []
        for k0 in range(0, nsteps, ck):
            ckpts.append(sim.state().clone())
            sim.step(min(ck, nsteps - k0))
        # delta rho is exact to the storage precision; rho0 is added in FP64
        rho = sim.density(sim.state()).double() + p.rho0
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.nsteps = nsteps
        ctx.ck = ck
        ctx.dtype = delta_f0.dtype
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        sim, ck, N = ctx.sim, ctx.ck, ctx.nsteps
        abar = sim.adjoint_seed(grad_rho.to(sim.params.dtype).contiguous())
        g = np.zeros(4)
        # one library call for all segments: the recompute of each earlier
        # segment overlaps the reverse sweep of the later one
        sim.adjoint_run(ctx.ckpts, abar, ck, N, grad=g)
        FLBRun.last_grads = dict(rate_shear=g[0], kT=g[1], rate_bulk=g[2], rate_ghost=g[3])
        dev = grad_rho.device
        # a parameter passed as a plain number (or a tensor without
        # requires_grad) gets no gradient
        need = ctx.needs_input_grad
        g_f0 = abar.to(ctx.dtype) if need[0] else None
        g_rs = torch.tensor(g[0], dtype=torch.float64, device=dev) if need[1] else None
        g_kT = torch.tensor(g[1], dtype=torch.float64, device=dev) if need[2] else None
        return g_f0, g_rs, g_kT, None, None, None


def final_density(delta_f0, rate_shear, kT, params, nsteps, checkpoint_every=20):
    """Functional form of FLBRun.apply."""
    return FLBRun.apply(delta_f0, rate_shear, kT, params, nsteps, checkpoint_every)
