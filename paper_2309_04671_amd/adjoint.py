"""Velocity gradient of a receiver misfit: torch.autograd.Function over the
library's forward and adjoint leapfrog kernels, with sqrt(N) checkpointing.

Forward: N leapfrog steps (paper Eq. 2, Algorithm 1) from zero wavefields,
recording the receiver traces; every C steps the pair (u^{n-1}, u^n) is
copied aside (C = ceil(sqrt(N)) by default).
Backward: for each segment, last first, the C forward states are recomputed
from its checkpoint (sp_wave_run_states) and the adjoint is stepped back over
the segment (sp_wave_adjoint_step), accumulating the FP64 gradient sum;
sp_grad_finish turns it into dL/dv.  dt and dx are held fixed.

Memory: 2 fields per checkpoint (N/C of them) + C+1 recompute fields + 2
adjoint fields + the FP64 sum, against N fields for storing every state.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import fields, lib


class WaveProblem:
    """Fixed (non-differentiable) part of a forward-modelling run."""

    def __init__(self, nx, ny, nz, coeffs, dt, dx, nsteps, src, amp, rec, ckpt=None,
                 device="cuda"):
        self.g = lib.grid_init(nx, ny, nz, lib.SP_F32)
        self.shape = (nz, ny, nx)
        self.co = lib.coeffs(coeffs)
        self.dt, self.dx, self.nsteps = float(dt), float(dx), int(nsteps)
        self.src_xyz = np.asarray(src, np.int32).reshape(-1, 3)
        amp = torch.as_tensor(np.asarray(amp, np.float32)).reshape(self.nsteps, len(self.src_xyz))
        self.amp = amp.to(device).contiguous()
        self.rec_xyz = np.asarray(rec, np.int32).reshape(-1, 3)
        self.rec_d = torch.as_tensor(self.rec_xyz).to(device).contiguous()
        self.nrec = len(self.rec_xyz)
        self.ckpt = int(ckpt) if ckpt else max(1, math.ceil(math.sqrt(self.nsteps)))
        self.device = device

    def sources(self):
        if len(self.src_xyz) == 0:
            return None
        return lib.make_sources(self.src_xyz, self.amp.data_ptr(), len(self.src_xyz))

    def receivers(self, traces, row0=0):
        return lib.make_receivers(self.nrec, self.rec_d.data_ptr(),
                                  traces[row0:].data_ptr(), self.nrec)


class WaveOp(torch.autograd.Function):
    """traces = WaveOp.apply(v, problem); v: (nz, ny, nx) FP32 CUDA tensor."""

    @staticmethod
    def forward(ctx, v, prob: WaveProblem):
        g, N, C = prob.g, prob.nsteps, prob.ckpt
        V = fields.Field(g, prob.device).set_interior(v.detach())
        ws = fields.WaveState(g, prob.device)
        traces = torch.zeros((N, prob.nrec), dtype=torch.float32, device=prob.device)
        src = prob.sources()
        ckpts = []
        for n0 in range(0, N, C):
            if n0 > 0:
                ckpts.append((ws.prev().buf.clone(), ws.cur().buf.clone()))
            L = min(C, N - n0)
            lib.sp_wave_step(g, prob.co, prob.dt, prob.dx, g, V.ptr, ws.st, L, src=src,
                             rec=prob.receivers(traces, n0) if prob.nrec else None)
        ctx.prob = prob
        ctx.V = V
        ctx.ckpts = ckpts
        return traces

    @staticmethod
    def backward(ctx, gtr):
        prob, V = ctx.prob, ctx.V
        g, N, C = prob.g, prob.nsteps, prob.ckpt
        gtr = gtr.detach().to(torch.float32).contiguous()
        G = torch.zeros(int(g.elems), dtype=torch.float64, device=prob.device)
        adj = fields.WaveState(g, prob.device)
        adj.st.step = N
        zeros = (fields.Field(g, prob.device), fields.Field(g, prob.device))
        ring = [fields.Field(g, prob.device) for _ in range(C)]
        src = prob.sources()
        rec = lib.make_receivers(prob.nrec, prob.rec_d.data_ptr(), gtr.data_ptr(), prob.nrec)
        starts = list(range(0, N, C))
        for j in reversed(range(len(starts))):
            n0 = starts[j]
            L = min(C, N - n0)
            if j == 0:
                first = [zeros[0].ptr, zeros[1].ptr]
            else:
                first = [ctx.ckpts[j - 1][0].data_ptr(), ctx.ckpts[j - 1][1].data_ptr()]
            states = first + [f.ptr for f in ring[:L - 1]]          # u^{n0-1} .. u^{n0+L-1}
            if L > 1:
                lib.sp_wave_run_states(g, prob.co, prob.dt, prob.dx, g, V.ptr, states, n0, L - 1,
                                       src=src)
            u_hist = [states[L - i] for i in range(L)]             # u^{k-1}, k = n0+L .. n0+1
            lib.sp_wave_adjoint_step(g, prob.co, prob.dt, prob.dx, g, V.ptr, adj.st, u_hist, L,
                                     src, rec if prob.nrec else None, G.data_ptr())
        out = fields.Field(g, prob.device)
        lib.sp_grad_finish(g, V.ptr, G.data_ptr(), out.ptr)
        return out.interior().contiguous(), None


def misfit_gradient(v, prob: WaveProblem, d_obs):
    """J = 1/2 sum (traces - d_obs)^2 and dJ/dv for a velocity tensor v."""
    v = v.detach().clone().requires_grad_(True)
    tr = WaveOp.apply(v, prob)
    J = 0.5 * ((tr.double() - d_obs.double()) ** 2).sum()
    J.backward()
    return float(J.detach()), v.grad
