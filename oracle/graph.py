"""Graph actions: forward action and its two adjoint traversals (FP64).

Test infrastructure (see the package docstring).  Operand layout: eta[N, nsets],
x / w / y [N, nops, nsets]; op and set columns are independent except that every
operand column of a set uses that set's eta.

* apply        F_k = sum_{e in E(k)} c_e eta_{i_e} x_{j_e}        (Eq. graph-actions,
               Sec. 2.2; L(h)x of Sec. 2.4)
* adjoint_x    g_x[j] = sum_{e : j_e = j} c_e eta_{i_e} w_{k_e}   (the adjoint
               traversal accumulates into the input coordinate, Sec. 2.4)
* adjoint_eta  g_eta[i] = sum_{e : i_e = i} c_e sum_op w_{k_e} x_{j_e}
* apply_outside  C_q = sum_{e in E_C(q)} c_e eta_{i_e} x_{j_e}   (the optional
               outside-space action, Eq. graph-actions third line)

All factors are real, so the conjugation of the adjoint is the identity.
"""
from __future__ import annotations

import numpy as np

from .algebra import Graph


def _scatter(index: np.ndarray, vals: np.ndarray, N: int) -> np.ndarray:
    """out[r] = sum of vals[e] over e with index[e] == r (vals is [E, ...])."""
    flat = vals.reshape(vals.shape[0], -1)
    out = np.empty((N, flat.shape[1]))
    for col in range(flat.shape[1]):
        out[:, col] = np.bincount(index, weights=flat[:, col], minlength=N)
    return out.reshape((N,) + vals.shape[1:])


def apply(g: Graph, eta: np.ndarray, x: np.ndarray) -> np.ndarray:
    contrib = g.c[:, None, None] * eta[g.i][:, None, :] * x[g.j]
    return _scatter(g.k, contrib, g.N)


def adjoint_x(g: Graph, eta: np.ndarray, w: np.ndarray) -> np.ndarray:
    contrib = g.c[:, None, None] * eta[g.i][:, None, :] * w[g.k]
    return _scatter(g.j, contrib, g.N)


def adjoint_eta(g: Graph, w: np.ndarray, x: np.ndarray) -> np.ndarray:
    contrib = g.c[:, None] * np.sum(w[g.k] * x[g.j], axis=1)
    return _scatter(g.i, contrib, g.N)


def apply_outside(og, eta: np.ndarray, x: np.ndarray) -> np.ndarray:
    """C [n_out, nops, nsets] for an OutsideGraph ``og``."""
    contrib = og.c[:, None, None] * eta[og.i][:, None, :] * x[og.j]
    return _scatter(og.k, contrib, og.n_out)


def apply_rows(g: Graph, eta: np.ndarray, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Forward action evaluated only at the given target rows (for sampling).

    ``g`` may hold the records of just those targets (see majorana_graph with
    ``targets``); the result is [len(rows), nops, nsets].
    """
    out = np.zeros((len(rows),) + x.shape[1:])
    for t, r in enumerate(rows):
        sel = g.k == r
        out[t] = np.sum(g.c[sel, None, None] * eta[g.i[sel]][:, None, :] * x[g.j[sel]],
                        axis=0)
    return out
