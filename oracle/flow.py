"""Classic RK4 coflow and its exact discrete adjoint (FP64).

Test infrastructure (see the package docstring).

State z[N, nops, nsets]: op 0 is the Hamiltonian h, ops 1.. are coflowed
operators X (Eq. coflow, Sec. 2.1; Eq. forward-coeff, Sec. 2.4).  Right-hand side:
    f(z) = L(eta(h)) z,   i.e.  f_op = apply(eta(h), z_op)   for every op.
The paper does not name its integrator; the classic fourth-order Runge-Kutta
scheme with a fixed step is used.  Set b advances n_b whole steps, then freezes.

The reverse direction is the exact adjoint of the discrete RK4 map (what central
finite differences of the discrete flow measure).  For one step with stage
states Z1..Z4 and cotangent lam' of the step output:
    u4 = J(Z4)^T [ds/6 lam']
    u3 = J(Z3)^T [ds/3 lam' + ds u4]
    u2 = J(Z2)^T [ds/3 lam' + ds/2 u3]
    u1 = J(Z1)^T [ds/6 lam' + ds/2 u2]
    lam = lam' + u1 + u2 + u3 + u4
with J(Z)^T mu = (adjoint_x(eta, mu) for every op) + e_h * eta'(h)^T
adjoint_eta(mu, Z): the graph-level adjoint of Sec. 2.4 plus the induced
generator variation of Eq. directional-derivative.
"""
from __future__ import annotations

from typing import Callable, List, Optional, Tuple

import numpy as np

from . import graph as G
from .algebra import Graph


def rhs(g: Graph, gen: Callable, z: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    eta = gen(z[:, 0, :])
    return G.apply(g, eta, z), eta


def rk4_step(g: Graph, gen: Callable, z: np.ndarray, ds: float,
             active: np.ndarray) -> np.ndarray:
    k1, _ = rhs(g, gen, z)
    k2, _ = rhs(g, gen, z + 0.5 * ds * k1)
    k3, _ = rhs(g, gen, z + 0.5 * ds * k2)
    k4, _ = rhs(g, gen, z + ds * k3)
    znew = z + (ds / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return np.where(active[None, None, :], znew, z)


RK4_WEIGHTS = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


def integrate_outside(g: Graph, gen: Callable, og, z0: np.ndarray, ds: float,
                      n_steps) -> Tuple[np.ndarray, np.ndarray]:
    """The flow of ``integrate`` plus the outside-space diagnostic (Eq.
    projected-flow: C_X = (I - P)[eta, X] never feeds the flow).  Returns
    (z_end, leak[nops, nsets]) with leak = sum over the steps each set takes of
    sum_s b_s ds sum_q C_q(Z_s)^2: the RK4 quadrature, over the same stage
    states, of the integral of |C_X|^2 (b = 1/6, 1/3, 1/3, 1/6; Z_s the stage
    states, C evaluated with the stage generator eta(Z_s,h))."""
    n_steps = np.asarray(n_steps)
    z = z0.copy()
    leak = np.zeros(z0.shape[1:])
    for t in range(int(n_steps.max()) if n_steps.size else 0):
        active = n_steps > t
        stage, ks = z, []
        for s, b in enumerate(RK4_WEIGHTS):
            k, eta = rhs(g, gen, stage)
            C = G.apply_outside(og, eta, stage)
            leak += np.where(active[None, :], b * ds * np.sum(C * C, axis=0), 0.0)
            ks.append(k)
            if s < 3:
                stage = z + (0.5 if s < 2 else 1.0) * ds * k
        znew = z + (ds / 6.0) * (ks[0] + 2.0 * ks[1] + 2.0 * ks[2] + ks[3])
        z = np.where(active[None, None, :], znew, z)
    return z, leak


def integrate(g: Graph, gen: Callable, z0: np.ndarray, ds: float, n_steps,
              ckpt_every: int = 0) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Flows every set for its own n_b steps; returns (z_end, checkpoints).

    Checkpoints hold z at steps 0, c, 2c, ... (global step counter) when
    ckpt_every = c > 0.
    """
    n_steps = np.asarray(n_steps)
    z = z0.copy()
    ck = []
    for t in range(int(n_steps.max()) if n_steps.size else 0):
        if ckpt_every and t % ckpt_every == 0:
            ck.append(z.copy())
        z = rk4_step(g, gen, z, ds, n_steps > t)
    return z, ck


def jt(g: Graph, gen: Callable, gen_vjp: Callable, Z: np.ndarray,
       mu: np.ndarray) -> np.ndarray:
    """J(Z)^T mu for f(Z) = apply(eta(Z_h), Z)."""
    h = Z[:, 0, :]
    eta = gen(h)
    out = G.adjoint_x(g, eta, mu)
    geta = G.adjoint_eta(g, mu, Z)
    out[:, 0, :] += gen_vjp(h, geta)
    return out


def step_adjoint(g, gen, gen_vjp, z, ds, lam, active):
    """Pulls lam back through one RK4 step taken from state z."""
    k1, _ = rhs(g, gen, z)
    Z2 = z + 0.5 * ds * k1
    k2, _ = rhs(g, gen, Z2)
    Z3 = z + 0.5 * ds * k2
    k3, _ = rhs(g, gen, Z3)
    Z4 = z + ds * k3
    u4 = jt(g, gen, gen_vjp, Z4, (ds / 6.0) * lam)
    u3 = jt(g, gen, gen_vjp, Z3, (ds / 3.0) * lam + ds * u4)
    u2 = jt(g, gen, gen_vjp, Z2, (ds / 3.0) * lam + 0.5 * ds * u3)
    u1 = jt(g, gen, gen_vjp, z, (ds / 6.0) * lam + 0.5 * ds * u2)
    new = lam + u1 + u2 + u3 + u4
    return np.where(active[None, None, :], new, lam)


def flow_adjoint(g: Graph, gen: Callable, gen_vjp: Callable, z0: np.ndarray, ds: float,
                 n_steps, lam_end: np.ndarray, ckpt_every: int = 16) -> np.ndarray:
    """dL/dz0 given dL/dz_end, recomputing each checkpoint block forward."""
    n_steps = np.asarray(n_steps)
    T = int(n_steps.max()) if n_steps.size else 0
    _, ck = integrate(g, gen, z0, ds, n_steps, ckpt_every=ckpt_every)
    lam = lam_end.copy()
    nblk = len(ck)
    for b in range(nblk - 1, -1, -1):
        t0 = b * ckpt_every
        t1 = min(T, t0 + ckpt_every)
        states = [ck[b]]
        for t in range(t0, t1 - 1):
            states.append(rk4_step(g, gen, states[-1], ds, n_steps > t))
        for t in range(t1 - 1, t0 - 1, -1):
            lam = step_adjoint(g, gen, gen_vjp, states[t - t0], ds, lam, n_steps > t)
    return lam
