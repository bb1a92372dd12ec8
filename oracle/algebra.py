"""Operator registries and contribution records, built from the operator algebra.

Test infrastructure (see the package docstring).  A record (k, i, j, c) states
that the commutator of the i-th generator basis element with the j-th operator
basis element contributes c times the k-th operator basis element (Sec. 2.2,
Eq. graph-actions): dh_k/ds = sum_e c_e * eta_{i_e} * h_{j_e}.  Records are
grouped by target k and, within a target, ordered by (i, j).

Two algebras are provided:

* One-body fermion operators E_pq = a+_p a_q, registry index p*n+q, with
  [E_pq, E_rs] = delta_qr E_ps - delta_ps E_rq.  The generator basis is the
  operator basis itself.  Diagonal mask: p == q.
* Majorana strings over m = 2n modes, gamma_a^2 = 1, {gamma_a, gamma_b} = 0 for
  a != b.  Hermitian basis Gamma_S = phi(|S|) gamma_{s1} ... gamma_{sd} with
  phi(d) = i^{d(d-1)/2} (orthonormal under Tr(.)/2^n); generator basis
  i*Gamma_S (anti-Hermitian).  Registry: every 2-subset, then every 4-subset,
  each in lexicographic order (projection P keeps degree <= 4, Sec. 2.1,
  Eq. projected-flow).  Diagonal mask: S is a union of pairs {2a, 2a+1}.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Graph:
    """Records grouped by target (k-sorted, then (i, j)), plus registry metadata."""

    algebra: str
    size: int
    N: int
    k: np.ndarray           # int64 [E]
    i: np.ndarray           # int64 [E]
    j: np.ndarray           # int64 [E]
    c: np.ndarray           # float64 [E]
    diag: np.ndarray        # bool [N], block-diagonal coordinates (mask D)
    pairs: np.ndarray       # int64 [n]: registry index of the n diagonal quadratics
    gen_sign: float         # eta_k = gen_sign * sum c (Dh)_i h_j for Wegner
    masks: Optional[np.ndarray] = None   # uint64 [N] (Majorana)

    @property
    def E(self) -> int:
        return int(self.k.size)

    def offsets(self) -> np.ndarray:
        cnt = np.bincount(self.k, minlength=self.N)
        return np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)

    def eta_records(self) -> "Graph":
        """E_eta: the records whose left input is a block-diagonal coordinate.

        The block generator eta = [H_d, H_od] (Eq. block-generator) expands into
        exactly these terms; records with both inputs diagonal vanish because the
        diagonal coordinates commute in both algebras.
        """
        sel = self.diag[self.i]
        return dataclasses.replace(self, k=self.k[sel], i=self.i[sel], j=self.j[sel],
                                   c=self.c[sel])


# ----------------------------------------------------------------------------
# One-body fermion operators E_pq
# ----------------------------------------------------------------------------

def epq_graph(n: int) -> Graph:
    """All records of [E_pq, E_rs] = delta_qr E_ps - delta_ps E_rq over the registry.

    Every ordered pair of registry elements is expanded; identical (k, i, j) are
    merged by summing and zero factors are dropped ("every nonzero term",
    Sec. 2.2).
    """
    acc: Dict[Tuple[int, int, int], int] = {}
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    i, j = p * n + q, r * n + s
                    if q == r:
                        key = (p * n + s, i, j)
                        acc[key] = acc.get(key, 0) + 1
                    if p == s:
                        key = (r * n + q, i, j)
                        acc[key] = acc.get(key, 0) - 1
    recs = sorted((key, v) for key, v in acc.items() if v != 0)
    k = np.array([r[0][0] for r in recs], dtype=np.int64)
    i = np.array([r[0][1] for r in recs], dtype=np.int64)
    j = np.array([r[0][2] for r in recs], dtype=np.int64)
    c = np.array([r[1] for r in recs], dtype=np.float64)
    diag = np.zeros(n * n, dtype=bool)
    diag[[p * n + p for p in range(n)]] = True
    pairs = np.array([p * n + p for p in range(n)], dtype=np.int64)
    return Graph("epq", n, n * n, k, i, j, c, diag, pairs, 1.0)


# ----------------------------------------------------------------------------
# Majorana strings
# ----------------------------------------------------------------------------

def majorana_subsets(m: int) -> List[Tuple[int, ...]]:
    """Canonical registry order: 2-subsets then 4-subsets, lexicographic."""
    return list(itertools.combinations(range(m), 2)) + list(itertools.combinations(range(m), 4))


def majorana_masks(m: int) -> np.ndarray:
    subs = majorana_subsets(m)
    out = np.zeros(len(subs), dtype=np.uint64)
    for t, S in enumerate(subs):
        v = 0
        for a in S:
            v |= 1 << a
        out[t] = v
    return out


def _popcount(x: np.ndarray) -> np.ndarray:
    return np.bitwise_count(x.astype(np.uint64)).astype(np.int64)


def _tri(d: np.ndarray) -> np.ndarray:
    """Exponent of i in phi(d) = i^{d(d-1)/2}, reduced mod 4."""
    return (d * (d - 1) // 2) % 4


def inversions(A: np.ndarray, B: np.ndarray, m: int) -> np.ndarray:
    """#{(a, b) in A x B : a > b} for bitmask arrays (plain count over b)."""
    A = A.astype(np.uint64)
    B = B.astype(np.uint64)
    inv = np.zeros(A.shape, dtype=np.int64)
    for b in range(m):
        has_b = ((B >> np.uint64(b)) & np.uint64(1)).astype(bool)
        above = A >> np.uint64(b + 1)
        inv += np.where(has_b, _popcount(above), 0)
    return inv


def bracket_coeff(A: np.ndarray, B: np.ndarray, m: int) -> np.ndarray:
    """c with [i*Gamma_A, Gamma_B] = c * Gamma_{A xor B}; 0 when they commute.

    Reordering gamma_A gamma_B into sorted order costs (-1)^{inv(A,B)} (each
    transposition of distinct modes anticommutes, equal modes square to 1), so
    Gamma_A Gamma_B = phi(|A|) phi(|B|) (-1)^inv / phi(|C|) * Gamma_C.  For even
    strings they anticommute iff |A & B| is odd, and then
    [i Gamma_A, Gamma_B] = 2 i Gamma_A Gamma_B.
    """
    A = np.asarray(A, dtype=np.uint64)
    B = np.asarray(B, dtype=np.uint64)
    C = A ^ B
    anti = (_popcount(A & B) % 2) == 1
    e = (1 + _tri(_popcount(A)) + _tri(_popcount(B)) - _tri(_popcount(C))
         + 2 * inversions(A, B, m)) % 4
    if np.any(anti & (e % 2 == 1)):
        raise AssertionError("non-real structure constant")
    c = np.where(e == 0, 2.0, -2.0)
    return np.where(anti, c, 0.0)


class MajoranaRegistry:
    def __init__(self, m: int):
        self.m = m
        self.masks = majorana_masks(m)
        self.N = self.masks.size
        self.order = np.argsort(self.masks, kind="stable")
        self.sorted_masks = self.masks[self.order]
        pm = np.array([(1 << (2 * a)) | (1 << (2 * a + 1)) for a in range(m // 2)],
                      dtype=np.uint64)
        self.pair_masks = pm
        self.pairs = self.index_of(pm)
        # diagonal: every member's partner in its pair is also a member
        lo = np.uint64(int("01" * 32, 2) & ((1 << m) - 1))   # even bits 0, 2, 4, ...
        ev = self.masks & lo
        od = (self.masks >> np.uint64(1)) & lo
        self.diag = ev == od

    def index_of(self, q: np.ndarray) -> np.ndarray:
        q = np.asarray(q, dtype=np.uint64)
        pos = np.searchsorted(self.sorted_masks, q)
        pos = np.minimum(pos, self.N - 1)
        ok = self.sorted_masks[pos] == q
        out = np.where(ok, self.order[pos], -1)
        return out.astype(np.int64)

    def records_for_target(self, t: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """All (i, j, c) with [iGamma_i, Gamma_j] having a nonzero Gamma_t component.

        Brute force over the left input: j is forced to A xor target; the pair is
        kept when that string is in the registry (degree 2 or 4) and the two
        strings anticommute.  Ascending i, hence ascending (i, j).
        """
        kmask = self.masks[t]
        A = self.masks
        B = A ^ kmask
        dB = _popcount(B)
        keep = ((dB == 2) | (dB == 4)) & ((_popcount(A & B) % 2) == 1)
        ii = np.nonzero(keep)[0].astype(np.int64)
        jj = self.index_of(B[ii])
        assert np.all(jj >= 0)
        cc = bracket_coeff(A[ii], B[ii], self.m)
        return ii, jj, cc


def majorana_graph(m: int, targets: Optional[np.ndarray] = None) -> Graph:
    """Full k-sorted record list (or the records of the given targets only)."""
    reg = MajoranaRegistry(m)
    tl = np.arange(reg.N) if targets is None else np.asarray(targets, dtype=np.int64)
    ks, is_, js, cs = [], [], [], []
    for t in tl:
        ii, jj, cc = reg.records_for_target(int(t))
        ks.append(np.full(ii.size, t, dtype=np.int64))
        is_.append(ii)
        js.append(jj)
        cs.append(cc)
    k = np.concatenate(ks)
    i = np.concatenate(is_)
    j = np.concatenate(js)
    c = np.concatenate(cs)
    return Graph("majorana", m, reg.N, k, i, j, c, reg.diag.copy(), reg.pairs.copy(),
                 -1.0, masks=reg.masks)


def majorana_closed_form_counts(m: int) -> Tuple[int, int, int]:
    """(records per quadratic target, per quartic target, total) from counting.

    Quadratic target {a,b}: quad x quad with one shared mode (2(m-2) ordered
    pairs) and quartic x quartic sharing three modes (2*C(m-2,3)).  Quartic
    target: quad x quartic and quartic x quad sharing one mode (8(m-4)).
    """
    from math import comb
    q = 2 * (m - 2) + 2 * comb(m - 2, 3)
    f = 8 * (m - 4)
    return q, f, comb(m, 2) * q + comb(m, 4) * f


# ----------------------------------------------------------------------------
# Outside-space records E_C (Majorana strings)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class OutsideGraph:
    """Records of the outside-space action C (Eq. projected-flow, C_X =
    (I - P)[eta, X]; Eq. graph-actions, third line): target q indexes the
    outside registry (here every 6-subset, lexicographic), inputs i and j the
    operator registry.  Grouped by q, then (i, j)."""

    size: int
    N: int                  # operator registry size (inputs)
    n_out: int              # outside registry size (targets)
    k: np.ndarray
    i: np.ndarray
    j: np.ndarray
    c: np.ndarray
    masks: np.ndarray       # uint64 [n_out]

    @property
    def E(self) -> int:
        return int(self.k.size)

    def offsets(self) -> np.ndarray:
        cnt = np.bincount(self.k, minlength=self.n_out)
        return np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)


def majorana_outside_masks(m: int) -> np.ndarray:
    """Every 6-subset of the m modes as a bitmask, lexicographic."""
    out = []
    for S in itertools.combinations(range(m), 6):
        v = 0
        for a in S:
            v |= 1 << a
        out.append(v)
    return np.array(out, dtype=np.uint64)


def majorana_outside_graph(m: int, targets: Optional[np.ndarray] = None) -> OutsideGraph:
    """The degree-6 part of [i Gamma_A, Gamma_B] over all registry pairs.

    Brute force per outside target Q over the left input A: B = A xor Q must be
    a registry string that anticommutes with A, and the factor is the bracket
    coefficient.  Two even strings of degree <= 4 reach degree 6 only as two
    quartics sharing one mode, so every stored pair is of that kind; the test
    suite checks the completeness against dense commutators.
    """
    reg = MajoranaRegistry(m)
    omasks = majorana_outside_masks(m)
    tl = np.arange(omasks.size) if targets is None else np.asarray(targets, dtype=np.int64)
    ks, is_, js, cs = [], [], [], []
    A = reg.masks
    for t in tl:
        B = A ^ omasks[t]
        dB = _popcount(B)
        keep = ((dB == 2) | (dB == 4)) & ((_popcount(A & B) % 2) == 1)
        ii = np.nonzero(keep)[0].astype(np.int64)
        jj = reg.index_of(B[ii])
        assert np.all(jj >= 0)
        ks.append(np.full(ii.size, t, dtype=np.int64))
        is_.append(ii)
        js.append(jj)
        cs.append(bracket_coeff(A[ii], B[ii], m))
    cat = (lambda parts, dt: np.concatenate(parts).astype(dt) if parts else np.zeros(0, dt))
    return OutsideGraph(m, reg.N, int(omasks.size), cat(ks, np.int64), cat(is_, np.int64),
                        cat(js, np.int64), cat(cs, np.float64), omasks)


def majorana_outside_count(m: int) -> int:
    """|E_C| by counting: a 6-subset Q splits into an ordered pair of triples
    (T1, T2) in C(6,3) = 20 ways, and the shared mode s is any of the m - 6
    modes outside Q: records (T1+s, T2+s)."""
    from math import comb
    return 20 * (m - 6) * comb(m, 6)


def graph_for(algebra: str, size: int) -> Graph:
    if algebra == "epq":
        return epq_graph(size)
    return majorana_graph(size)
