"""Derivatives of one projected action (FP64).

Test infrastructure (see the package docstring).

The projected action of Sec. 2.4 is F(h, x) = L(h) x = apply(eta(h), x): the
generator is built from the Hamiltonian coefficients h [N, nsets] and the graph
acts on the operand x [N, nops, nsets] (op 0 is often h itself, but here h and x
are independent inputs).

* action_jvp   the directional derivative of Eq. directional-derivative:
               dF = apply(eta'(h) dh, x) + apply(eta(h), dx); the first term is the
               induced generator variation, the second the linear response.
* action_vjp   its transpose: for a cotangent w of F,
               g_x = adjoint_x(eta(h), w) and g_h = eta'(h)^T adjoint_eta(w, x)
               (the adjoint traversals of Sec. 2.4, then the generator VJP).
* pairing_defect   <w, dF> - (<g_h, dh> + <g_x, dx>), zero for an exact
               transpose pair (the forward-adjoint pairing check of Sec. 3.3).
* fd_scan      centred finite differences of F along (dh, 0) or (0, dx) at the
               given steps, each compared with action_jvp in the relative
               max-norm (the scan of Sec. 3.3, Fig. execution-consistency a).
"""
from __future__ import annotations

from typing import Callable, Dict, Iterable, Tuple

import numpy as np

from . import graph as G
from .algebra import Graph


def action(g: Graph, gen: Callable, h: np.ndarray, x: np.ndarray) -> np.ndarray:
    return G.apply(g, gen(h), x)


def action_jvp(g: Graph, gen: Callable, gen_jvp: Callable, h: np.ndarray, x: np.ndarray,
               dh: np.ndarray, dx: np.ndarray) -> np.ndarray:
    return G.apply(g, gen_jvp(h, dh), x) + G.apply(g, gen(h), dx)


def action_vjp(g: Graph, gen: Callable, gen_vjp: Callable, h: np.ndarray, x: np.ndarray,
               w: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Returns (g_h [N, nsets], g_x [N, nops, nsets])."""
    g_x = G.adjoint_x(g, gen(h), w)
    g_h = gen_vjp(h, G.adjoint_eta(g, w, x))
    return g_h, g_x


def pairing_defect(g: Graph, gen: Callable, gen_jvp: Callable, gen_vjp: Callable,
                   h: np.ndarray, x: np.ndarray, dh: np.ndarray, dx: np.ndarray,
                   w: np.ndarray) -> Tuple[float, float]:
    """(absolute defect, scale) where scale = |<w, dF>| + |<g_h, dh>| + |<g_x, dx>|."""
    df = action_jvp(g, gen, gen_jvp, h, x, dh, dx)
    g_h, g_x = action_vjp(g, gen, gen_vjp, h, x, w)
    lhs = float(np.sum(w * df))
    a, b = float(np.sum(g_h * dh)), float(np.sum(g_x * dx))
    return lhs - (a + b), abs(lhs) + abs(a) + abs(b)


def fd_scan(g: Graph, gen: Callable, gen_jvp: Callable, h: np.ndarray, x: np.ndarray,
            d: np.ndarray, direction: str, steps: Iterable[float]) -> Dict[float, float]:
    """max|FD - JVP| / max|JVP| per step for the direction 'h' or 'x'."""
    zero_h, zero_x = np.zeros_like(h), np.zeros_like(x)
    if direction == "h":
        exact = action_jvp(g, gen, gen_jvp, h, x, d, zero_x)
    elif direction == "x":
        exact = action_jvp(g, gen, gen_jvp, h, x, zero_h, d)
    else:
        raise ValueError(direction)
    out = {}
    for eps in steps:
        if direction == "h":
            fp, fm = action(g, gen, h + eps * d, x), action(g, gen, h - eps * d, x)
        else:
            fp, fm = action(g, gen, h, x + eps * d), action(g, gen, h, x - eps * d)
        fd = (fp - fm) / (2.0 * eps)
        out[float(eps)] = float(np.max(np.abs(fd - exact)) / np.max(np.abs(exact)))
    return out
