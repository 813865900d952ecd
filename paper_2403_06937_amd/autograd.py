"""torch.autograd.Function around the forward run and tc_evolve_backward.

    loss = TCMLoss.apply(g, delta, n, c, rho0, dt, steps, checkpoint_every, mode, sectors)

g, delta: float64 CPU tensors of length n (couplings g_i and detunings delta_i,
w_a,i = 1 + delta_i).  rho0: the initial density matrix on the GPU (complex64 or
complex128).  The forward forms H and U = exp(-i H dt) on the GPU, steps rho
(rotating frame, lab-frame checkpoints) with checkpoints every `checkpoint_every` steps and returns the
final sum_i <s_i^+ s_i^-> as a 0-d float64 tensor; backward runs the adjoint
sweep of tc_evolve_backward (sectors: both by excitation-sector blocks).  Only
marshalling happens here.
"""
from __future__ import annotations

import torch

from . import (Model, TC_C128, TC_C64, TC_FRAME_LAB, TC_FRAME_ROTATING, TC_GEMM_F64,
               make_opts, tc_evolve_backward)
from . import pipeline


class TCMLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, delta, n, c, rho0, dt, steps, checkpoint_every, mode=TC_GEMM_F64,
                sectors=False):
        g64 = g.detach().to(torch.float64).cpu()
        d64 = delta.detach().to(torch.float64).cpu()
        model = Model(int(n), int(c), g64.tolist(), (1.0 + d64).tolist())
        H, U = pipeline.propagator(model, float(dt), device=rho0.device)
        rho = rho0.clone()
        # rotating frame: in reduced precision only the small U~ - I is rounded;
        # checkpoints are stored as lab-frame states either way
        pop, _, ck = pipeline.evolve(model, U, rho, int(steps), float(dt), mode,
                                     TC_FRAME_ROTATING, 0, int(steps) if steps > 0 else 1,
                                     int(checkpoint_every), sectors=bool(sectors))
        ctx.model, ctx.H, ctx.U, ctx.ck = model, H, U, ck
        ctx.opts = make_opts(int(steps), float(dt), mode,
                             TC_C128 if rho0.dtype == torch.complex128 else TC_C64,
                             TC_FRAME_LAB, 0, 1, int(checkpoint_every), sectors=int(bool(sectors)))
        return pop[-1].detach().cpu()

    @staticmethod
    def backward(ctx, grad_out):
        dev = ctx.U.device
        n = ctx.model.n
        gg = torch.zeros(n, dtype=torch.float64, device=dev)
        gd = torch.zeros(n, dtype=torch.float64, device=dev)
        tc_evolve_backward(ctx.model, ctx.H, ctx.U, ctx.opts, ctx.ck, None, gg, gd)
        go = grad_out.to(torch.float64).cpu()
        return (gg.cpu() * go, gd.cpu() * go, None, None, None, None, None, None, None, None)
