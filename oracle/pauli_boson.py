"""Pauli-boson operator algebra and its compiled records (exact arithmetic).

Test infrastructure (see the package docstring).

Sec. 2.1, Eq. monomial: operator labels B_{tau,c,a} = sigma_tau prod_m
(b_m^dagger)^{c_m} b_m^{a_m}, tau in {I, x, y, z}, c, a in N_0^M.  The complete
degree-p registry holds every label with |c| + |a| <= p; its size is
4 C(2M + p, p) (Eq. basis-size).  Products are evaluated in the full bosonic
algebra and normal ordered before membership in the registry is tested.  The
block-diagonal coordinates (mask D) are the I and sigma_z labels with c = a
(joint sigma_z / boson-number blocks).

Sec. 2.2, Eq. graph-actions: with the generator eta = [H_d, H_od] (Eq.
block-generator) expanded exactly,
  E_eta: xi_a = sum alpha (Dh)_i ((I-D)h)_j   over i in D, j not in D,
         [B_i, B_j] = sum_a alpha B_a  (a ranges over the generator registry:
         every label that occurs);
  E_L:   F_k = sum beta xi_a x_j    over the generator registry a and the
         registry j, [B_a, B_j] = sum_k beta B_k with k in the registry;
  E_C:   the same terms with k outside the registry (optional diagnostic).
Factors are Gaussian integers (sigma products contribute powers of i, normal
ordering contributes k! C(a, k) C(c', k) per mode); they are kept exact as
(re, im) pairs of Python ints.

Canonical orders (a reading; the paper does not print one): every registry is
sorted by (total bosonic degree, tau, c_1, a_1, ..., c_M, a_M); records within
a target by (left input index, right input index).
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache
from typing import Dict, List, Tuple

Label = Tuple[int, Tuple[int, ...], Tuple[int, ...]]      # (tau, c, a)
GInt = Tuple[int, int]                                     # re, im

# sigma_t sigma_u = phase * sigma_w, phase = i**e; tau 0 = I, 1 = x, 2 = y, 3 = z
_CYCLIC = {(1, 2), (2, 3), (3, 1)}


def pauli_mul(t: int, u: int) -> Tuple[int, int]:
    """(w, e) with sigma_t sigma_u = i**e sigma_w."""
    if t == 0:
        return u, 0
    if u == 0:
        return t, 0
    if t == u:
        return 0, 0
    w = 6 - t - u
    return w, (1 if (t, u) in _CYCLIC else 3)


@lru_cache(maxsize=None)
def mode_product(c1: int, a1: int, c2: int, a2: int) -> Tuple[Tuple[int, int, int], ...]:
    """Normal ordering of (b^+)^c1 b^a1 (b^+)^c2 b^a2 for one mode:
    sum_k k! C(a1, k) C(c2, k) (b^+)^(c1+c2-k) b^(a1+a2-k)  (Wick contractions of
    the a1 annihilators with the c2 creators).  Returns ((c, a, coeff), ...)."""
    out = []
    for k in range(min(a1, c2) + 1):
        out.append((c1 + c2 - k, a1 + a2 - k, math.factorial(k) * math.comb(a1, k) * math.comb(c2, k)))
    return tuple(out)


def boson_product(cA, aA, cB, aB) -> List[Tuple[Tuple[int, ...], Tuple[int, ...], int]]:
    """Normal-ordered product of two multi-mode monomials (modes commute)."""
    terms = [((), (), 1)]
    for m in range(len(cA)):
        nxt = []
        for c, a, f in terms:
            for cc, aa, g in mode_product(cA[m], aA[m], cB[m], aB[m]):
                nxt.append((c + (cc,), a + (aa,), f * g))
        terms = nxt
    return terms


_IPOW = [(1, 0), (0, 1), (-1, 0), (0, -1)]


def commutator(A: Label, B: Label) -> Dict[Label, GInt]:
    """[B_A, B_B] as {label: Gaussian-integer coefficient}, zeros dropped."""
    out: Dict[Label, List[int]] = {}
    for (X, Y, sign) in ((A, B, 1), (B, A, -1)):
        w, e = pauli_mul(X[0], Y[0])
        pr, pi = _IPOW[e]
        for c, a, f in boson_product(X[1], X[2], Y[1], Y[2]):
            acc = out.setdefault((w, c, a), [0, 0])
            acc[0] += sign * pr * f
            acc[1] += sign * pi * f
    return {k: (v[0], v[1]) for k, v in out.items() if v[0] != 0 or v[1] != 0}


def degree(L: Label) -> int:
    return sum(L[1]) + sum(L[2])


def sort_key(L: Label):
    key = [degree(L), L[0]]
    for m in range(len(L[1])):
        key += [L[1][m], L[2][m]]
    return tuple(key)


def registry(M: int, p: int) -> List[Label]:
    """The complete degree-p registry in canonical order."""
    out = []
    for exps in itertools.product(range(p + 1), repeat=2 * M):
        if sum(exps) > p:
            continue
        c, a = tuple(exps[0::2]), tuple(exps[1::2])
        for tau in range(4):
            out.append((tau, c, a))
    return sorted(out, key=sort_key)


def registry_size(M: int, p: int) -> int:
    """Eq. basis-size."""
    return 4 * math.comb(2 * M + p, p)


def is_diagonal(L: Label) -> bool:
    return L[0] in (0, 3) and L[1] == L[2]


class PBGraph:
    """Registries and record lists (k, i, j, (re, im)) of one (M, p)."""

    def __init__(self, M: int, p: int, outside: bool = False):
        self.M, self.p = M, p
        self.labels = registry(M, p)
        self.index = {L: n for n, L in enumerate(self.labels)}
        self.N = len(self.labels)
        self.diag = [is_diagonal(L) for L in self.labels]
        D = [n for n in range(self.N) if self.diag[n]]
        OD = [n for n in range(self.N) if not self.diag[n]]
        # E_eta: products of a diagonal and an off-diagonal coordinate
        raw = []
        for i in D:
            for j in OD:
                for L, f in commutator(self.labels[i], self.labels[j]).items():
                    raw.append((L, i, j, f))
        self.gen_labels = sorted({r[0] for r in raw}, key=sort_key)
        self.gen_index = {L: n for n, L in enumerate(self.gen_labels)}
        self.NG = len(self.gen_labels)
        self.eta = sorted((self.gen_index[L], i, j, f) for L, i, j, f in raw)
        # E_L and E_C: generator coordinate x registry coordinate
        rec_l, rec_c = [], []
        for a, A in enumerate(self.gen_labels):
            for j, B in enumerate(self.labels):
                for L, f in commutator(A, B).items():
                    k = self.index.get(L)
                    if k is not None:
                        rec_l.append((k, a, j, f))
                    elif outside:
                        rec_c.append((L, a, j, f))
        self.flow = sorted(rec_l)
        if outside:
            self.out_labels = sorted({r[0] for r in rec_c}, key=sort_key)
            oi = {L: n for n, L in enumerate(self.out_labels)}
            self.outside = sorted((oi[L], a, j, f) for L, a, j, f in rec_c)

    # ---------------------------------------------------------------- actions
    def generator(self, h):
        """xi = sum alpha (Dh)_i ((I-D)h)_j over E_eta (complex h of length N)."""
        import numpy as np
        xi = np.zeros(self.NG, dtype=complex)
        for a, i, j, f in self.eta:
            xi[a] += complex(*f) * h[i] * h[j]
        return xi

    def action(self, xi, x):
        """F_k = sum beta xi_a x_j over E_L (complex vectors)."""
        import numpy as np
        y = np.zeros(self.N, dtype=complex)
        for k, a, j, f in self.flow:
            y[k] += complex(*f) * xi[a] * x[j]
        return y


def generator_registry(M: int, p: int) -> List[Label]:
    """Every label the brackets [B_i, B_j] (i block-diagonal, j not) of the
    degree-p registry reach (the generator registry of Eq. graph-actions),
    canonical order."""
    labels = registry(M, p)
    D = [L for L in labels if is_diagonal(L)]
    OD = [L for L in labels if not is_diagonal(L)]
    out = set()
    for A in D:
        for B in OD:
            out.update(commutator(A, B))
    return sorted(out, key=sort_key)


def target_terms(labels: List[Label], gen_labels: List[Label], T: Label):
    """The terms of target label T in [B_a, B_j] over generator labels a and
    registry labels j, as sorted (a, j, (re, im)): the records of T in E_L when
    T is in the registry, in E_C when it is not, found without enumerating
    every pair.  Per mode, a product of (b^+)^cA b^aA and (b^+)^cB b^aB in
    either order reaches (b^+)^cT b^aT only through a contraction of order
    k >= 0 with cT = cA + cB - k and aT = aA + aB - k, and sigma_A sigma_B is
    proportional to sigma_T only for one tau_A; so for every registry label B
    the candidates A are cA = cT - cB + k, aA = aT - aB + k over k >= 0 (degree
    bounded by the generator registry's), and each candidate's bracket gives
    the exact factor."""
    gen_index = {L: n for n, L in enumerate(gen_labels)}
    dmax = max(degree(L) for L in gen_labels)
    M = len(T[1])
    out = []
    for j, B in enumerate(labels):
        # sigma_A = sigma_T sigma_B up to phase (the Pauli group is abelian
        # modulo phases, so one tau serves both orders)
        tau_a = pauli_mul(T[0], B[0])[0]
        base_c = [T[1][m] - B[1][m] for m in range(M)]
        base_a = [T[2][m] - B[2][m] for m in range(M)]
        kmin = [max(0, -base_c[m], -base_a[m]) for m in range(M)]
        slack = dmax - sum(base_c[m] + base_a[m] + 2 * kmin[m] for m in range(M))
        if slack < 0:
            continue
        for extra in itertools.product(range(slack // 2 + 1), repeat=M):
            if 2 * sum(extra) > slack:
                continue
            k = [kmin[m] + extra[m] for m in range(M)]
            A = (tau_a, tuple(base_c[m] + k[m] for m in range(M)), tuple(base_a[m] + k[m] for m in range(M)))
            a = gen_index.get(A)
            if a is None:
                continue
            f = commutator(A, B).get(T)
            if f is not None:
                out.append((a, j, f))
    return sorted(out)


def _streamed_part(args):
    labels, gen_slice, xi_slice, X = args
    import numpy as np
    index = {L: n for n, L in enumerate(labels)}
    F = np.zeros((len(labels),) + X.shape[1:], dtype=complex)
    S = np.zeros(F.shape)
    n = np.zeros(len(labels), dtype=np.int64)
    aX = np.abs(X.real) + np.abs(X.imag)
    for A, xa in zip(gen_slice, xi_slice):
        axa = np.abs(xa.real) + np.abs(xa.imag)
        for j, B in enumerate(labels):
            for L, f in commutator(A, B).items():
                k = index.get(L)
                if k is not None:
                    F[k] += complex(*f) * xa * X[j]
                    S[k] += abs(complex(*f)) * axa * aX[j]
                    n[k] += 1
    return F, S, n


def streamed_action(M: int, p: int, h, X, workers: int = 1):
    """The generator and retained action of ``PBGraph`` (E_eta, then E_L of
    Eq. graph-actions) for registries too large to hold their records: xi =
    sum alpha (Dh)_i ((I-D)h)_j over the diagonal / off-diagonal pairs, the
    generator registry being every label those brackets reach, then F_k = sum
    beta xi_a X_j over every (generator label, registry label) pair, each
    bracket expanded as it is needed.  h is complex [N, sets] (one Hamiltonian
    per set), X complex [N, nops, sets]; the pairs are dealt over ``workers``
    processes by generator label and the partial sums added.  Returns a dict:
    labels, gen_labels, xi [NG, sets], F [N, nops, sets], and for the rounding
    error of any evaluation order, per output coordinate, the number of terms
    (xi_n, F_n) and the sums of their absolute sizes (xi_abs: |alpha| |h_i|
    |h_j|; F_abs: |beta| |xi_a| |X_j|, with |v| = |Re v| + |Im v|)."""
    import numpy as np
    labels = registry(M, p)
    diag = [is_diagonal(L) for L in labels]
    D = [n for n in range(len(labels)) if diag[n]]
    OD = [n for n in range(len(labels)) if not diag[n]]
    h = np.asarray(h, dtype=complex)
    ah = np.abs(h.real) + np.abs(h.imag)
    acc: Dict[Label, list] = {}
    for i in D:
        for j in OD:
            for L, f in commutator(labels[i], labels[j]).items():
                e = acc.setdefault(L, [0, 0, 0])
                e[0] = e[0] + complex(*f) * h[i] * h[j]
                e[1] = e[1] + abs(complex(*f)) * ah[i] * ah[j]
                e[2] += 1
    gen_labels = sorted(acc, key=sort_key)
    xi = np.stack([acc[L][0] for L in gen_labels]).astype(complex)
    X = np.asarray(X, dtype=complex)
    xi_b = xi[:, None, :]
    parts = [(labels, gen_labels[w::workers], xi_b[w::workers], X) for w in range(workers)]
    if workers == 1:
        out = [_streamed_part(parts[0])]
    else:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            out = pool.map(_streamed_part, parts)
    F, S, n = (sum(o[q] for o in out) for q in range(3))
    return {"labels": labels, "gen_labels": gen_labels, "xi": xi,
            "xi_abs": np.stack([acc[L][1] for L in gen_labels]).astype(float),
            "xi_n": np.array([acc[L][2] for L in gen_labels], dtype=np.int64),
            "F": F, "F_abs": S, "F_n": n}


def adjoint(g: "PBGraph", xi, x, w):
    """Reverse traversal of E_L (Sec. 2.4: the stored factor, accumulated back
    into the input coordinates with conjugation): with F_k = sum beta xi_a x_j,
    g_x[j] = sum conj(beta xi_a) w_k and g_xi[a] = sum conj(beta x_j) w_k, the
    gradients of Re <w, F> = Re sum conj(w_k) F_k with respect to x and xi
    (complex vectors).  Returns (g_x, g_xi)."""
    import numpy as np
    gx = np.zeros(g.N, dtype=complex)
    gxi = np.zeros(g.NG, dtype=complex)
    for k, a, j, f in g.flow:
        c = complex(*f)
        gx[j] += np.conj(c * xi[a]) * w[k]
        gxi[a] += np.conj(c * x[j]) * w[k]
    return gx, gxi


def outside_action(g: "PBGraph", xi, x):
    """C_q = sum gamma xi_a x_j over E_C (the graph must hold outside records)."""
    import numpy as np
    y = np.zeros(len(g.out_labels), dtype=complex)
    for q, a, j, f in g.outside:
        y[q] += complex(*f) * xi[a] * x[j]
    return y


def flow_outside(g: "PBGraph", z0, ds: float, steps: int):
    """The flow of ``flow`` plus the outside-space diagnostic: every stage
    state Z_s of every step adds b_s ds sum_q |C_q(Z_s)|^2 per operand
    (b = 1/6, 1/3, 1/3, 1/6), C evaluated with the stage generator."""
    import numpy as np
    z = np.array(z0, dtype=complex)
    leak = np.zeros(z.shape[1])
    b = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
    for _ in range(steps):
        stage, ks = z, []
        for s in range(4):
            xi = g.generator(stage[:, 0])
            for o in range(z.shape[1]):
                c = outside_action(g, xi, stage[:, o])
                leak[o] += b[s] * ds * float(np.sum(np.abs(c) ** 2))
            ks.append(np.stack([g.action(xi, stage[:, o]) for o in range(z.shape[1])], axis=1))
            if s < 3:
                stage = z + (0.5 if s < 2 else 1.0) * ds * ks[-1]
        z = z + (ds / 6.0) * (ks[0] + 2 * ks[1] + 2 * ks[2] + ks[3])
    return z, leak


def flow(g: "PBGraph", z0, ds: float, steps: int):
    """Classic RK4 of the coflow (Eq. coflow): z[:, 0] = H, z[:, 1:] = operators,
    dz/ds = P[eta(H), z] with eta = [H_d, H_od] from E_eta and P[.,.] from E_L
    (complex coefficients; the integrator reading of the Majorana flow)."""
    import numpy as np
    z = np.array(z0, dtype=complex)

    def rhs(u):
        xi = g.generator(u[:, 0])
        return np.stack([g.action(xi, u[:, o]) for o in range(u.shape[1])], axis=1)

    for _ in range(steps):
        k1 = rhs(z)
        k2 = rhs(z + 0.5 * ds * k1)
        k3 = rhs(z + 0.5 * ds * k2)
        k4 = rhs(z + ds * k3)
        z = z + (ds / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return z
