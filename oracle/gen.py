"""Generators eta(h) and their vector-Jacobian products (FP64).

Test infrastructure (see the package docstring).  h and eta are [N, nsets].

* wegner_graph: the block generator eta = [H_d, H_od] (Eq. block-generator,
  Sec. 2.1) evaluated as a graph pass over E_eta (Eq. graph-actions, first line):
  eta_k = s_g * sum_{e in E_eta(k)} c_e (Dh)_{i_e} h_{j_e}, where s_g converts the
  operator-basis bracket into generator-basis coefficients (+1 for E_pq, whose
  generator basis is the operator basis; -1 for Majorana strings, whose generator
  basis is i*Gamma: [Gamma_A, Gamma_B] = -i [iGamma_A, Gamma_B]).
* g2: normalised Wegner generator for Majorana strings (the reading taken here
  of a White-type generator built from the diagonal pair energies): with
  pair energies eps_a = h_{P_a} and the pair-flip set F(S),
      N_S = -sum_{a in F(S)} c(S, P_a, S^P_a) eps_a h_{S^P_a}
      Q_S = 4 sum_{a in F(S)} eps_a^2 + delta^2,     eta_S = N_S / Q_S,
  and eta = 0 on block-diagonal strings.  N is the Wegner generator of the
  quadratic diagonal part H_0 = sum_a eps_a Gamma_{P_a}; Q_S is the diagonal of
  ad_{H_0}^2 in the orthonormal string basis, regularised by delta^2.
* g1: the literal reading of a White-type generator from the diagonal pair
  energies, eta_S = h_S / D_S with D_S = 2 sum_{a in F(S)} |eps_a| + delta
  (delta >= 0 regularises D_S = 0), eta = 0 on block-diagonal strings.
"""
from __future__ import annotations

import numpy as np

from .algebra import Graph, MajoranaRegistry, bracket_coeff, _popcount


def wegner_graph(g: Graph, h: np.ndarray) -> np.ndarray:
    ge = g.eta_records()
    dh = np.where(g.diag[:, None], h, 0.0)       # (Dh)
    odh = np.where(g.diag[:, None], 0.0, h)      # ((I-D)h)
    contrib = ge.c[:, None] * dh[ge.i] * odh[ge.j]
    out = np.zeros_like(h)
    for s in range(h.shape[1]):
        out[:, s] = np.bincount(ge.k, weights=contrib[:, s], minlength=g.N)
    return g.gen_sign * out


def wegner_graph_jvp(g: Graph, h: np.ndarray, dh: np.ndarray) -> np.ndarray:
    """Directional derivative of wegner_graph along dh.  The generator is a
    bilinear function of (Dh, (I-D)h), so by the product rule (the derivative of
    the generator that Eq. directional-derivative calls for) it is
    W(D dh, (I-D)h) + W(Dh, (I-D) dh)."""
    ge = g.eta_records()
    dmask = g.diag[:, None]
    a0, b0 = np.where(dmask, h, 0.0), np.where(dmask, 0.0, h)
    a1, b1 = np.where(dmask, dh, 0.0), np.where(dmask, 0.0, dh)
    contrib = ge.c[:, None] * (a1[ge.i] * b0[ge.j] + a0[ge.i] * b1[ge.j])
    out = np.zeros_like(h)
    for s in range(h.shape[1]):
        out[:, s] = np.bincount(ge.k, weights=contrib[:, s], minlength=g.N)
    return g.gen_sign * out


def wegner_graph_vjp(g: Graph, h: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    ge = g.eta_records()
    dmask = g.diag.astype(float)
    gh = np.zeros_like(h)
    for s in range(h.shape[1]):
        w = g.gen_sign * ge.c * gbar[ge.k, s]
        gh[:, s] += dmask * np.bincount(ge.i, weights=w * (1 - dmask[ge.j]) * h[ge.j, s],
                                        minlength=g.N)
        gh[:, s] += (1 - dmask) * np.bincount(ge.j, weights=w * dmask[ge.i] * h[ge.i, s],
                                              minlength=g.N)
    return gh


class G2:
    """Per-pair stencil of the normalised Wegner generator (built once per m)."""

    def __init__(self, m: int, delta: float):
        reg = MajoranaRegistry(m)
        self.reg = reg
        self.delta = float(delta)
        self.stencil = []   # per pair a: (S rows, partner rows, c)
        for a in range(m // 2):
            pm = reg.pair_masks[a]
            flips = _popcount(reg.masks & pm) == 1
            S = np.nonzero(flips)[0].astype(np.int64)
            partner_mask = reg.masks[S] ^ pm
            partner = reg.index_of(partner_mask)
            assert np.all(partner >= 0)
            # coefficient of Gamma_S in [i Gamma_{P_a}, Gamma_partner]
            c = bracket_coeff(np.full(S.size, pm, dtype=np.uint64), partner_mask, m)
            assert np.all(np.abs(c) == 2.0)
            self.stencil.append((S, partner, c))

    def _nq(self, h):
        N = np.zeros_like(h)
        Qs = np.zeros_like(h)
        for a, (S, P, c) in enumerate(self.stencil):
            eps = h[self.reg.pairs[a]][None, :]
            N[S] += -c[:, None] * eps * h[P]
            Qs[S] += 4.0 * eps * eps
        Q = Qs + self.delta ** 2
        return N, Q

    def __call__(self, h: np.ndarray) -> np.ndarray:
        N, Q = self._nq(h)
        eta = N / Q
        eta[self.reg.diag] = 0.0
        return eta

    def jvp(self, h: np.ndarray, dh: np.ndarray) -> np.ndarray:
        """Directional derivative of eta along dh by the quotient rule:
        d eta_S = (dN_S Q_S - N_S dQ_S) / Q_S^2 with
        dN_S = -sum_a c (d eps_a h_partner + eps_a dh_partner) and
        dQ_S = 8 sum_a eps_a d eps_a; zero on block-diagonal strings."""
        N, Q = self._nq(h)
        dN = np.zeros_like(h)
        dQ = np.zeros_like(h)
        for a, (S, P, c) in enumerate(self.stencil):
            pa = self.reg.pairs[a]
            eps, deps = h[pa][None, :], dh[pa][None, :]
            dN[S] += -c[:, None] * (deps * h[P] + eps * dh[P])
            dQ[S] += 8.0 * eps * deps
        out = (dN * Q - N * dQ) / (Q * Q)
        out[self.reg.diag] = 0.0
        return out

    def vjp(self, h: np.ndarray, gbar: np.ndarray) -> np.ndarray:
        """d/dh of sum(gbar * eta(h)) by the product and quotient rules."""
        N, Q = self._nq(h)
        gb = np.where(self.reg.diag[:, None], 0.0, gbar)
        gh = np.zeros_like(h)
        for a, (S, P, c) in enumerate(self.stencil):
            pa = self.reg.pairs[a]
            eps = h[pa][None, :]
            w = gb[S] / Q[S]
            # d eta_S / d h_partner = -c eps / Q
            np.add.at(gh, P, -c[:, None] * eps * w)
            # d eta_S / d eps_a = -c h_partner / Q - N_S * 8 eps / Q^2
            d_eps = -c[:, None] * h[P] * w - gb[S] * N[S] * 8.0 * eps / (Q[S] ** 2)
            gh[pa] += d_eps.sum(axis=0)
        return gh


class G1:
    """eta_S = h_S / (2 sum_{a in F(S)} |h_{P_a}| + delta) on off-diagonal S.

    F(S) = pairs a = (2a, 2a+1) that S holds exactly one mode of; stored as a
    0/1 matrix flips[S, a]."""

    def __init__(self, m: int, delta: float):
        reg = MajoranaRegistry(m)
        self.reg = reg
        self.delta = float(delta)
        self.flips = np.stack([_popcount(reg.masks & pm) == 1 for pm in reg.pair_masks], axis=1).astype(float)
        self.off = ~reg.diag

    def _d(self, h):
        return 2.0 * self.flips @ np.abs(h[self.reg.pairs]) + self.delta

    def __call__(self, h: np.ndarray) -> np.ndarray:
        return np.where(self.off[:, None], h / self._d(h), 0.0)

    def jvp(self, h: np.ndarray, dh: np.ndarray) -> np.ndarray:
        """d eta_S = dh_S / D_S - h_S dD_S / D_S^2, dD_S = 2 sum_{a in F(S)} sign(eps_a) d eps_a."""
        D = self._d(h)
        dD = 2.0 * self.flips @ (np.sign(h[self.reg.pairs]) * dh[self.reg.pairs])
        return np.where(self.off[:, None], dh / D - h * dD / (D * D), 0.0)

    def vjp(self, h: np.ndarray, gbar: np.ndarray) -> np.ndarray:
        D = self._d(h)
        gb = np.where(self.off[:, None], gbar, 0.0)
        gh = gb / D
        geps = -2.0 * np.sign(h[self.reg.pairs]) * (self.flips.T @ (gb * h / (D * D)))
        np.add.at(gh, self.reg.pairs, geps)
        return gh


def make_generator(g: Graph, kind: str, delta: float = 0.5):
    """Returns (eta(h), vjp(h, gbar)) for the named generator."""
    if kind == "wegner_graph":
        return (lambda h: wegner_graph(g, h)), (lambda h, gb: wegner_graph_vjp(g, h, gb))
    if kind in ("g2", "g1"):
        gen = (G2 if kind == "g2" else G1)(g.size, delta)
        return gen, gen.vjp
    raise ValueError(kind)


def make_generator_jvp(g: Graph, kind: str, delta: float = 0.5):
    """Returns jvp(h, dh) = eta'(h) dh for the named generator."""
    if kind == "wegner_graph":
        return lambda h, dh: wegner_graph_jvp(g, h, dh)
    if kind in ("g2", "g1"):
        return (G2 if kind == "g2" else G1)(g.size, delta).jvp
    raise ValueError(kind)
