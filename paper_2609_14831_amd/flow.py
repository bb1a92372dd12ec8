"""Differentiable coflow: torch.autograd.Function over cut_flow_integrate /
cut_flow_adjoint (argument marshalling only).

forward:  z(end) = RK4 flow of z0 (Sec. 2.1 Eq. coflow), checkpoints every
          ``ckpt_every`` steps kept on the device;
backward: dL/dz0 by the exact adjoint of the discrete RK4 map, recomputing each
          checkpoint block (graph-level adjoint of Sec. 2.4 plus the induced
          generator variation of Eq. directional-derivative).
"""
from __future__ import annotations

import torch

from . import _lib as L


class FlowFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z0: torch.Tensor, graph: int, n_steps, generator: int, ds: float, delta: float,
                ckpt_every: int, precision: int):
        assert z0.is_cuda and z0.dtype == torch.float64 and z0.dim() == 3 and z0.is_contiguous()
        N, nops, nsets = z0.shape
        T = max(int(v) for v in n_steps) if len(n_steps) else 0
        nck = (T + ckpt_every - 1) // ckpt_every if T else 0
        ckpt = torch.empty((max(nck, 1), N, nops, nsets), dtype=torch.float64, device=z0.device)
        z = z0.clone()
        p = L.flow_params(generator, precision, ds, delta, ckpt_every)
        L.cut_flow_integrate(graph, p, nsets, nops, list(n_steps), z, ckpt)
        ctx.save_for_backward(ckpt)
        ctx.cfg = (graph, list(n_steps), generator, ds, delta, ckpt_every, nsets, nops)
        return z

    @staticmethod
    def backward(ctx, gz: torch.Tensor):
        (ckpt,) = ctx.saved_tensors
        graph, n_steps, generator, ds, delta, ckpt_every, nsets, nops = ctx.cfg
        lam = gz.contiguous().clone()
        p = L.flow_params(generator, L.CUT_F64, ds, delta, ckpt_every, flags=0)
        L.cut_flow_adjoint(graph, p, nsets, nops, n_steps, ckpt, lam)
        return lam, None, None, None, None, None, None, None


def flow(z0, graph, n_steps, generator=L.CUT_GEN_G2, ds=5e-3, delta=0.5, ckpt_every=16,
         precision=L.CUT_F64):
    return FlowFn.apply(z0, graph, n_steps, generator, ds, delta, ckpt_every, precision)
