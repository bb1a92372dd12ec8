"""Pins of the oracle's registries, records and graph actions (CPU only).

Each test checks the oracle against something other than itself: dense matrix
commutators (Jordan-Wigner Majorana matrices, one-body unit matrices), closed
form counts, and exact record identities.
"""
import itertools
import math

import numpy as np
import pytest

import brute
from oracle import algebra as A
from oracle import graph as G


def _rec_dict(g):
    return {(int(k), int(i), int(j)): float(c) for k, i, j, c in zip(g.k, g.i, g.j, g.c)}


# ---------------------------------------------------------------- Majorana ----

@pytest.mark.parametrize("m", [4, 6, 8])
def test_majorana_records_match_dense_jw(m):
    """Every record equals Tr(Gamma_k [i Gamma_i, Gamma_j]) / 2^n, and every
    nonzero in-registry component of every commutator is a record."""
    subs, mats = brute.dense_strings(m)
    g = A.majorana_graph(m)
    assert [tuple(np.nonzero([(int(x) >> b) & 1 for b in range(m)])[0]) for x in g.masks] == subs
    rec = _rec_dict(g)
    N = len(subs)
    M = 1j * (np.einsum("axy,byz->abxz", mats, mats) - np.einsum("bxy,ayz->abxz", mats, mats))
    coef = brute.project(mats, M)          # [a, b, k]
    assert np.max(np.abs(coef.imag)) < 1e-12
    coef = coef.real
    found = 0
    for a in range(N):
        for b in range(N):
            for k in np.nonzero(np.abs(coef[a, b]) > 1e-9)[0]:
                assert rec[(int(k), a, b)] == pytest.approx(coef[a, b, k], abs=1e-12)
                found += 1
    assert found == len(rec)


def test_majorana_phase_convention_hermitian_orthonormal():
    subs, mats = brute.dense_strings(8)
    dim = mats.shape[-1]
    for M in mats:
        assert np.allclose(M, M.conj().T)
    gram = np.einsum("axy,byx->ab", mats, mats) / dim
    assert np.allclose(gram, np.eye(len(subs)))


@pytest.mark.parametrize("m", [8, 12, 16, 24])
def test_majorana_counts_closed_form(m):
    g = A.majorana_graph(m)
    nq = math.comb(m, 2)
    per_q = 2 * (m - 2) + 2 * math.comb(m - 2, 3)
    per_f = 8 * (m - 4)
    cnt = np.bincount(g.k, minlength=g.N)
    assert np.all(cnt[:nq] == per_q)
    assert np.all(cnt[nq:] == per_f)
    assert g.E == nq * per_q + math.comb(m, 4) * per_f
    if m == 24:
        assert g.E == 2_562_384
    # records sorted by (k, i, j) with no duplicates
    key = (g.k * g.N + g.i) * g.N + g.j
    assert np.all(np.diff(key) > 0)
    assert set(np.unique(g.c)) <= {-2.0, 2.0}


@pytest.mark.parametrize("m,expect_total", [(40, 39_539_760), (64, 457_720_704)])
def test_majorana_sampled_target_counts(m, expect_total):
    reg = A.MajoranaRegistry(m)
    nq = math.comb(m, 2)
    per_q = 2 * (m - 2) + 2 * math.comb(m - 2, 3)
    per_f = 8 * (m - 4)
    assert nq * per_q + math.comb(m, 4) * per_f == expect_total
    rng = np.random.default_rng(3)
    for t in list(rng.integers(0, nq, 3)) + list(rng.integers(nq, reg.N, 3)):
        ii, jj, cc = reg.records_for_target(int(t))
        assert ii.size == (per_q if t < nq else per_f)
        assert np.all(reg.masks[ii] ^ reg.masks[jj] == reg.masks[t])


@pytest.mark.parametrize("m", [8, 12])
def test_majorana_record_antisymmetry(m):
    """ad of an anti-Hermitian basis element is antisymmetric in an orthonormal
    Hermitian basis: c(k, i, j) = -c(j, i, k)."""
    rec = _rec_dict(A.majorana_graph(m))
    for (k, i, j), c in rec.items():
        assert rec[(j, i, k)] == -c


def test_majorana_apply_matches_dense_commutator():
    m = 8
    subs, mats = brute.dense_strings(m)
    g = A.majorana_graph(m)
    rng = np.random.default_rng(11)
    N = len(subs)
    eta = rng.normal(size=(N, 2))
    x = rng.normal(size=(N, 3, 2))
    y = G.apply(g, eta, x)
    for s in range(2):
        etaop = np.einsum("a,axy->xy", 1j * eta[:, s], mats)
        for op in range(3):
            X = np.einsum("a,axy->xy", x[:, op, s], mats)
            ref = brute.project(mats, etaop @ X - X @ etaop)
            assert np.max(np.abs(ref.imag)) < 1e-12
            np.testing.assert_allclose(y[:, op, s], ref.real, atol=1e-12)


def test_majorana_diag_and_pairs():
    m = 8
    reg = A.MajoranaRegistry(m)
    subs = A.majorana_subsets(m)
    for t, S in enumerate(subs):
        is_union = all(((a ^ 1) in S) for a in S)
        assert bool(reg.diag[t]) == is_union
    assert [subs[p] for p in reg.pairs] == [(2 * a, 2 * a + 1) for a in range(m // 2)]
    # diagonal strings are diagonal matrices under Jordan-Wigner
    _, mats = brute.dense_strings(m)
    for t in np.nonzero(reg.diag)[0]:
        M = mats[t]
        assert np.allclose(M, np.diag(np.diag(M)))


# ---------------------------------------------------------------- E_pq -------

def test_epq_records_match_matrix_commutators():
    n = 4
    g = A.epq_graph(n)
    rec = _rec_dict(g)
    found = 0
    for (p, q), (r, s) in itertools.product(itertools.product(range(n), repeat=2), repeat=2):
        C = brute.epq_matrix(n, p, q) @ brute.epq_matrix(n, r, s) - \
            brute.epq_matrix(n, r, s) @ brute.epq_matrix(n, p, q)
        for a, b in zip(*np.nonzero(C)):
            assert rec[(a * n + b, p * n + q, r * n + s)] == C[a, b]
            found += 1
    assert found == len(rec)


def test_epq_counts():
    for n in (3, 5, 8):
        g = A.epq_graph(n)
        assert g.E == 2 * n ** 3 - 2 * n
        assert g.eta_records().E == 2 * n * n - 2 * n
    g = A.epq_graph(8)
    assert g.E == 1008 and g.eta_records().E == 112
    cnt = np.bincount(g.k, minlength=64)
    diag = np.array([p * 8 + p for p in range(8)])
    assert np.all(cnt[diag] == 14)
    assert np.all(np.delete(cnt, diag) == 16)


def test_epq_record_identity_transpose():
    """The adjoint of ad_{E_pq} is ad_{E_qp}: c(k, i, j) = c(j, tau(i), k)."""
    n = 5
    rec = _rec_dict(A.epq_graph(n))
    tau = lambda t: (t % n) * n + t // n
    for (k, i, j), c in rec.items():
        assert rec[(j, tau(i), k)] == c


def test_epq_apply_matches_matrix_commutator():
    n = 8
    g = A.epq_graph(n)
    rng = np.random.default_rng(5)
    eta = rng.normal(size=(n * n, 1))
    x = rng.normal(size=(n * n, 2, 1))
    y = G.apply(g, eta, x)
    E = eta[:, 0].reshape(n, n)
    for op in range(2):
        X = x[:, op, 0].reshape(n, n)
        np.testing.assert_allclose(y[:, op, 0], (E @ X - X @ E).ravel(), atol=1e-12)


# ------------------------------------------------------------- adjoints -----

@pytest.mark.parametrize("alg,size", [("majorana", 8), ("epq", 6)])
def test_adjoints_are_transposes(alg, size):
    """Both adjoint traversals equal the transposes of the dense linear maps."""
    g = A.graph_for(alg, size)
    N = g.N
    rng = np.random.default_rng(2)
    nops, nsets = 2, 3
    eta = rng.normal(size=(N, nsets))
    x = rng.normal(size=(N, nops, nsets))
    w = rng.normal(size=(N, nops, nsets))
    # dense map x -> apply(eta, x) for set 0, op 0 (one column)
    Lx = np.zeros((N, N))
    Le = np.zeros((N, N))
    for col in range(N):
        e = np.zeros((N, 1, 1)); e[col] = 1.0
        Lx[:, col] = G.apply(g, eta[:, :1], e)[:, 0, 0]
        ee = np.zeros((N, 1)); ee[col] = 1.0
        Le[:, col] = G.apply(g, ee, x[:, :1, :1])[:, 0, 0]
    gx = G.adjoint_x(g, eta, w)
    np.testing.assert_allclose(gx[:, 0, 0], Lx.T @ w[:, 0, 0], atol=1e-11)
    ge = G.adjoint_eta(g, w[:, :1, :1], x[:, :1, :1])
    np.testing.assert_allclose(ge[:, 0], Le.T @ w[:, 0, 0], atol=1e-11)
    # dot-product identity over all columns
    y = G.apply(g, eta, x)
    lhs = np.sum(w * y)
    assert np.sum(G.adjoint_x(g, eta, w) * x) == pytest.approx(lhs, rel=1e-12)
    assert np.sum(G.adjoint_eta(g, w, x) * eta) == pytest.approx(lhs, rel=1e-12)
