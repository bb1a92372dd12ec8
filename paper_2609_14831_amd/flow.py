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


def _gen_rows(graph: int) -> int:
    """Generator rows of a loaded graph (Pauli-boson graphs are real-split)."""
    d = L.cut_graph_info(graph)
    return (2 if d["algebra"] == L.CUT_ALG_PAULI_BOSON else 1) * (d["n_gen_ops"] or d["n_ops"])


class ActionFn(torch.autograd.Function):
    """One projected action F(h, x) = L(eta(h)) x (Sec. 2.4), differentiable in
    both arguments: backward through cut_graph_vjp (the adjoint traversals and
    the generator VJP), forward mode through cut_graph_jvp (Eq.
    directional-derivative).  h [rows, nsets], x [rows, nops, nsets], both
    float64 contiguous on the device; the result has the layout of x."""

    @staticmethod
    def forward(h, x, graph: int, generator: int, delta: float, precision: int):
        assert h.is_cuda and x.is_cuda and h.dtype == x.dtype == torch.float64
        assert h.dim() == 2 and x.dim() == 3 and h.is_contiguous() and x.is_contiguous()
        N, nops, nsets = x.shape
        eta = torch.empty((_gen_rows(graph), nsets), dtype=torch.float64, device=h.device)
        L.cut_generator(graph, generator, delta, nsets, h, eta)
        y = torch.empty_like(x)
        xa = x.view(N, nops * nsets)
        if precision != L.CUT_F64:
            eta, xa = eta.float(), xa.float()
        L.cut_graph_apply(graph, L.CUT_GRAPH_FLOW, precision, nsets, nops, eta, xa, y.view(N, nops * nsets))
        return y

    @staticmethod
    def setup_context(ctx, inputs, output):
        h, x, graph, generator, delta, precision = inputs
        ctx.save_for_backward(h, x)
        ctx.save_for_forward(h, x)
        ctx.cfg = (graph, generator, delta, precision)

    @staticmethod
    def backward(ctx, gy):
        h, x = ctx.saved_tensors
        graph, generator, delta, precision = ctx.cfg
        N, nops, nsets = x.shape
        g_h = torch.empty_like(h)
        g_x = torch.empty_like(x)
        L.cut_graph_vjp(graph, generator, delta, precision, nsets, nops, h, x.view(N, nops * nsets),
                        gy.contiguous().view(N, nops * nsets), g_h, g_x.view(N, nops * nsets))
        return g_h, g_x, None, None, None, None

    @staticmethod
    def jvp(ctx, dh, dx, *_):
        h, x = ctx.saved_tensors
        graph, generator, delta, precision = ctx.cfg
        N, nops, nsets = x.shape
        dy = torch.empty_like(x)
        L.cut_graph_jvp(graph, generator, delta, precision, nsets, nops, h,
                        None if dh is None else dh.contiguous(), x.view(N, nops * nsets),
                        None if dx is None else dx.contiguous().view(N, nops * nsets), None,
                        dy.view(N, nops * nsets))
        return dy


def action(h, x, graph, generator=L.CUT_GEN_G2, delta=0.5, precision=L.CUT_F64):
    return ActionFn.apply(h, x, graph, generator, delta, precision)
