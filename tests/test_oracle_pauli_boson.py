"""Pins of the oracle's Pauli-boson algebra (Eq. monomial, Eq. basis-size,
Eq. projected-flow, Eq. graph-actions).

* registry sizes against Eq. basis-size;
* commutators against dense matrices on a truncated Fock space: sigma_tau (x)
  prod_m (b^+)^c b^a with b|n> = sqrt(n)|n-1>, compared on the input states whose
  occupations keep every intermediate state below the cutoff, where the
  truncated products are exact;
* the adjoint symmetry [A, B]^+ = [B^+, A^+] of the exact coefficients;
* record counts of the five-mode degree-4 graph against the numbers the paper
  prints (Sec. 3.2: 7,017,036 generator + retained-flow contributions and
  345,388,180 outside-space contributions), through the oracle's plain-C
  counter;
* the generator and action against dense commutators on a random Hamiltonian.
"""
import itertools
import json
import math
import os
from functools import reduce

import numpy as np
import pytest

from oracle import pauli_boson as PB

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_SIG = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1.0, -1.0])]


def _dense(L, nmax):
    tau, c, a = L
    b = np.diag(np.sqrt(np.arange(1, nmax + 1)), 1)
    mats = [np.linalg.matrix_power(b.T, c[m]) @ np.linalg.matrix_power(b, a[m]) for m in range(len(c))]
    return np.kron(_SIG[tau], reduce(np.kron, mats))


def _safe_columns(M, nmax, cmax):
    cols = []
    for occ in itertools.product(range(nmax + 1), repeat=M):
        if all(occ[m] <= nmax - cmax[m] for m in range(M)):
            idx = 0
            for m in range(M):
                idx = idx * (nmax + 1) + occ[m]
            cols.append(idx)
    dimb = (nmax + 1) ** M
    return [s * dimb + q for s in range(2) for q in cols]


@pytest.mark.parametrize("M,p", [(1, 1), (1, 4), (2, 3), (3, 2), (5, 4)])
def test_registry_size(M, p):
    assert len(PB.registry(M, p)) == PB.registry_size(M, p)
    assert PB.registry_size(5, 4) == 4004 and PB.registry_size(2, 4) == 280 and PB.registry_size(1, 24) == 1300


@pytest.mark.parametrize("M,p,nmax", [(1, 4, 14), (2, 3, 7)])
def test_commutators_match_dense_matrices(M, p, nmax):
    labels = PB.registry(M, p)
    rng = np.random.default_rng(M * 10 + p)
    pairs = [(labels[i], labels[j]) for i, j in rng.integers(0, len(labels), size=(60, 2))]
    # generator-registry products too (degree up to 2p on the left)
    g = PB.PBGraph(M, min(p, 2))
    pairs += [(g.gen_labels[i], labels[j]) for i, j in
              zip(rng.integers(0, g.NG, 20), rng.integers(0, len(labels), 20))]
    checked = 0
    for A, B in pairs:
        cmax = [A[1][m] + B[1][m] for m in range(M)]
        if any(x > nmax - 1 for x in cmax):
            continue
        cols = _safe_columns(M, nmax, cmax)
        DA, DB = _dense(A, nmax), _dense(B, nmax)
        ref = (DA @ DB - DB @ DA)[:, cols]
        got = np.zeros(ref.shape, dtype=complex)
        for L, f in PB.commutator(A, B).items():
            got += complex(*f) * _dense(L, nmax)[:, cols]
        assert np.allclose(got, ref, atol=1e-9 * max(1.0, np.abs(ref).max())), (A, B)
        checked += 1
    assert checked >= 40


def test_commutator_adjoint_symmetry():
    labels = PB.registry(2, 4)
    dag = lambda L: (L[0], L[2], L[1])
    rng = np.random.default_rng(1)
    for i, j in rng.integers(0, len(labels), size=(300, 2)):
        A, B = labels[i], labels[j]
        lhs = {dag(L): (f[0], -f[1]) for L, f in PB.commutator(A, B).items()}
        assert lhs == PB.commutator(dag(B), dag(A))


def test_generator_and_action_match_dense_commutators():
    """H Hermitian on the M = 1, p = 3 registry: xi = [H_d, H_od] and
    F = P[eta, X] agree with dense matrices on the safe columns (the outside part
    is what the projection drops, so only the retained labels are compared by
    projecting the dense commutator's expansion)."""
    M, p, nmax = 1, 3, 16
    g = PB.PBGraph(M, p, outside=True)
    rng = np.random.default_rng(3)
    h = np.zeros(g.N, dtype=complex)
    for n, L in enumerate(g.labels):           # Hermitian: h_{L^+} = conj(h_L)
        Ld = (L[0], L[2], L[1])
        m = g.index[Ld]
        if m == n:
            h[n] = rng.normal()
        elif m > n:
            h[n] = rng.normal() + 1j * rng.normal()
            h[m] = np.conj(h[n])
    x = rng.normal(size=g.N) + 1j * rng.normal(size=g.N)
    xi = g.generator(h)
    # eta as a dense matrix from the generator registry vs [H_d, H_od] densely
    dense = lambda coeffs, labs: sum(c * _dense(L, nmax) for c, L in zip(coeffs, labs))
    # the joint sigma_z / boson-number eigenspaces are single product states, so
    # the block-diagonal part of H is its diagonal in that basis
    Hfull = dense(h, g.labels)
    Hd = np.diag(np.diag(Hfull))
    Hod = Hfull - Hd
    cols = _safe_columns(M, nmax, [2 * p])
    eta_dense = (Hd @ Hod - Hod @ Hd)[:, cols]
    assert np.allclose(dense(xi, g.gen_labels)[:, cols], eta_dense, atol=1e-8)
    # retained + outside action equals the full commutator [eta, X]
    F = g.action(xi, x)
    C = np.zeros(len(g.out_labels), dtype=complex)
    for q, a, j, f in g.outside:
        C[q] += complex(*f) * xi[a] * x[j]
    cols = _safe_columns(M, nmax, [3 * p])
    Xd = dense(x, g.labels)
    E = dense(xi, g.gen_labels)
    full = (E @ Xd - Xd @ E)[:, cols]
    got = dense(F, g.labels)[:, cols] + dense(C, g.out_labels)[:, cols]
    assert np.allclose(got, full, atol=1e-7 * np.abs(full).max())


def test_five_mode_counts_match_the_paper():
    """Sec. 3.2: complete degree-four registry with five boson modes."""
    from oracle import native
    ref = json.load(open(os.path.join(GOLD, "pauli_boson_counts.json")))
    for case in ref["cases"]:
        got = native.pb_counts(case["M"], case["p"])
        for key in ("n_ops", "production", "outside"):
            if key in case:
                assert got[key] == case[key], (case, got)


def test_flow_outside_matches_plain_flow_and_dense_outside_norm():
    """One RK4 step on M = 1, p = 3: the flow with the outside-space diagnostic
    leaves the state as the plain flow does, and each stage's sum_q |C_q|^2 is
    the squared norm of the part of the dense [eta, X] outside the registry
    (orthonormality is not used: the outside part is rebuilt from the C_q and
    compared with the dense commutator minus the retained part)."""
    import workloads
    M, p, nmax = 1, 3, 16
    g = PB.PBGraph(M, p, outside=True)
    rng = np.random.default_rng(9)
    z0 = np.stack([workloads.pb_hermitian(g.labels, rng, 1.0, 0.05),
                   workloads.pb_hermitian(g.labels, rng, 1.0, 1.0)], axis=1)
    z1, leak = PB.flow_outside(g, z0, 1e-3, 1)
    np.testing.assert_array_equal(z1, PB.flow(g, z0, 1e-3, 1))
    assert np.all(leak > 0)
    xi = g.generator(z0[:, 0])
    dense = lambda coeffs, labs: sum(c * _dense(L, nmax) for c, L in zip(coeffs, labs))
    cols = _safe_columns(M, nmax, [3 * p])
    for o in range(2):
        E, X = dense(xi, g.gen_labels), dense(z0[:, o], g.labels)
        full = (E @ X - X @ E)[:, cols]
        outside = full - dense(g.action(xi, z0[:, o]), g.labels)[:, cols]
        C = PB.outside_action(g, xi, z0[:, o])
        assert np.allclose(dense(C, g.out_labels)[:, cols], outside, atol=1e-9 * np.abs(full).max())


def _pb_small():
    import workloads
    g = PB.PBGraph(1, 3, outside=True)
    rng = np.random.default_rng(21)
    z0 = np.stack([workloads.pb_hermitian(g.labels, rng, 1.0, 0.05),
                   workloads.pb_hermitian(g.labels, rng, 1.0, 1.0)], axis=1)
    return g, z0


def _columns(fn, n):
    """Matrix of a linear map given on unit vectors."""
    return np.stack([fn(np.eye(n, dtype=complex)[:, j]) for j in range(n)], axis=1)


def test_pb_rk4_step_is_fourth_order_taylor_with_fixed_generator():
    """With the generator held fixed the coflow right-hand side is the linear map
    L x = P[xi, x], so one classic RK4 step must equal the degree-4 Taylor
    polynomial sum_p (ds L)^p / p! applied to every column (Eq. coflow under
    the RK4 reading).  L is taken column by column from the action, which is
    pinned against dense truncated-Fock commutators above."""
    g, z0 = _pb_small()
    xi = g.generator(z0[:, 0])
    Lm = _columns(lambda e: g.action(xi, e), g.N)
    g.generator = lambda h: xi        # hold the generator fixed on this instance
    ds = 0.05
    z1 = PB.flow(g, z0, ds, 1)
    taylor = np.zeros_like(z0)
    term = z0.copy()
    for p in range(5):
        taylor += term
        term = ds * (Lm @ term) / (p + 1)
    np.testing.assert_allclose(z1, taylor, rtol=0, atol=1e-13 * np.abs(taylor).max())
    # the exponential differs at fifth order, so the step is not a trivially exact map
    from scipy.linalg import expm
    assert np.abs(expm(ds * Lm) @ z0 - z1).max() > 1e-12


def test_pb_flow_converges_at_fourth_order():
    """Self-consistent flow (generator from the stage Hamiltonian): the error
    at s = 0.1 against a 256-step reference falls by about 2^4 per halving of
    ds (the spectral radius of the action is about 6.4 here)."""
    g, z0 = _pb_small()
    T = 0.1
    ref = PB.flow(g, z0, T / 256, 256)
    errs = [np.abs(PB.flow(g, z0, T / n, n) - ref).max() for n in (16, 32)]
    assert 13.0 < errs[0] / errs[1] < 19.0, errs


def test_pb_outside_diagnostic_is_fourth_order_quadrature():
    """With the generator fixed, Z(s) = exp(sL) z0 and the diagnostic must be
    the RK4 quadrature of int_0^T sum_q |C_q(Z(s))|^2 ds: against that integral
    (Gauss-Legendre on the exact trajectory) its error falls by about 2^4 per
    halving of ds.  A wrong stage weight b_s leaves a first-order error."""
    from scipy.linalg import expm
    g, z0 = _pb_small()
    xi = g.generator(z0[:, 0])
    Lm = _columns(lambda e: g.action(xi, e), g.N)
    Cm = _columns(lambda e: PB.outside_action(g, xi, e), g.N)
    g.generator = lambda h: xi
    T = 0.2
    nodes, weights = np.polynomial.legendre.leggauss(40)
    exact = np.zeros(z0.shape[1])
    for u, wq in zip(nodes, weights):
        s = 0.5 * T * (u + 1.0)
        exact += 0.5 * T * wq * np.sum(np.abs(Cm @ (expm(s * Lm) @ z0)) ** 2, axis=0)
    errs = []
    for n in (8, 16):
        z, leak = PB.flow_outside(g, z0, T / n, n)
        np.testing.assert_array_equal(z, PB.flow(g, z0, T / n, n))
        errs.append(np.abs(leak - exact).max() / np.abs(exact).max())
    assert 13.0 < errs[0] / errs[1] < 19.0, errs
    assert errs[1] < 1e-6


def test_pb_adjoint_is_the_conjugate_transpose_of_the_action():
    """Sec. 2.4 reverse traversal: with the action's matrices in x (xi fixed)
    and in xi (x fixed) taken column by column, the oracle's adjoint must be
    g_x = A_x^H w and g_xi = A_xi^H w (the conjugation the paper names).  A
    missing conjugate or swapped input fails here."""
    g, z0 = _pb_small()
    rng = np.random.default_rng(8)
    xi = g.generator(z0[:, 0])
    x = z0[:, 1]
    w = rng.normal(size=g.N) + 1j * rng.normal(size=g.N)
    Ax = _columns(lambda e: g.action(xi, e), g.N)
    Axi = _columns(lambda e: g.action(e, x), g.NG)
    gx, gxi = PB.adjoint(g, xi, x, w)
    np.testing.assert_allclose(gx, Ax.conj().T @ w, rtol=0, atol=1e-12 * np.abs(gx).max())
    np.testing.assert_allclose(gxi, Axi.conj().T @ w, rtol=0, atol=1e-12 * np.abs(gxi).max())


def _normal_order_by_commutation(a, c):
    """b^a (b^+)^c normal ordered by moving one annihilator at a time through the
    creators with b (b^+)^x = (b^+)^x b + x (b^+)^(x-1): {(creators, annihilators):
    integer coefficient}."""
    poly = {(c, 0): 1}
    for _ in range(a):
        nxt = {}
        for (x, y), f in poly.items():
            nxt[(x, y + 1)] = nxt.get((x, y + 1), 0) + f
            if x:
                nxt[(x - 1, y)] = nxt.get((x - 1, y), 0) + x * f
        poly = nxt
    return poly


def test_wick_factors_at_degree_24_by_commutation():
    """The normal-ordering factors of the degree-24 one-mode registry (the
    registry of the paper's one-mode study, Sec. 3.1) leave int64 (24! ~ 6.2e23):
    the oracle's contraction formula must equal the exact integers obtained by
    commuting annihilators through creators one at a time, up to 24 of each,
    and the bracket [b^24, (b^+)^24] must hold 24! on the identity."""
    for a, c in ((24, 24), (24, 13), (7, 24), (17, 19)):
        ref = _normal_order_by_commutation(a, c)
        got = {(cc, aa): f for cc, aa, f in PB.mode_product(0, a, c, 0)}
        assert got == ref, (a, c)
    br = PB.commutator((0, (0,), (24,)), (0, (24,), (0,)))
    assert br[(0, (0,), (0,))] == (math.factorial(24), 0) and math.factorial(24) > 2 ** 63


@pytest.mark.parametrize("M,p,workers", [(1, 4, 1), (2, 2, 2), (1, 8, 3)])
def test_streamed_action_matches_the_record_graph(M, p, workers):
    """The streamed form (no stored records; used for registries too large to
    hold theirs) gives the generator registry, xi, F, the per-target term counts
    and absolute sums of the record graph."""
    import workloads
    g = PB.PBGraph(M, p)
    rng = np.random.default_rng(M * 100 + p)
    h = np.stack([workloads.pb_hermitian(g.labels, rng) for _ in range(2)], 1)
    X = rng.normal(size=(g.N, 3, 2)) + 1j * rng.normal(size=(g.N, 3, 2))
    r = PB.streamed_action(M, p, h, X, workers=workers)
    xi, F, S, n = r["xi"], r["F"], r["F_abs"], r["F_n"]
    assert r["labels"] == g.labels and r["gen_labels"] == g.gen_labels
    np.testing.assert_array_equal(r["xi_n"], np.bincount([e[0] for e in g.eta], minlength=g.NG))
    ah = np.abs(h.real) + np.abs(h.imag)
    Sx = np.zeros((g.NG, 2))
    for a, i, j, f in g.eta:
        Sx[a] += abs(complex(*f)) * ah[i] * ah[j]
    np.testing.assert_allclose(r["xi_abs"], Sx, rtol=1e-13)
    xi0 = np.stack([g.generator(h[:, s]) for s in range(2)], 1)
    np.testing.assert_allclose(xi, xi0, rtol=0, atol=1e-13 * np.abs(xi0).max())
    F0 = np.stack([np.stack([g.action(xi0[:, s], X[:, o, s]) for s in range(2)], 1) for o in range(3)], 1)
    np.testing.assert_allclose(F, F0, rtol=0, atol=1e-13 * np.abs(F0).max())
    np.testing.assert_array_equal(n, np.bincount([r[0] for r in g.flow], minlength=g.N))
    S0 = np.zeros(S.shape)
    ax, aX = np.abs(xi0.real) + np.abs(xi0.imag), np.abs(X.real) + np.abs(X.imag)
    for k, a, j, f in g.flow:
        S0[k] += abs(complex(*f)) * ax[a] * aX[j]
    np.testing.assert_allclose(S, S0, rtol=1e-13)


@pytest.mark.parametrize("M,p", [(1, 4), (2, 3), (3, 2)])
def test_target_terms_are_the_records_of_each_target(M, p):
    """The per-target expansion (used for targets of registries too large to
    expand whole, such as the five-mode graph) gives, for every retained and
    every outside target, exactly the records the whole-graph expansion files
    under it, factors included; and the generator registry matches."""
    from collections import defaultdict
    g = PB.PBGraph(M, p, outside=True)
    gl = PB.generator_registry(M, p)
    assert gl == g.gen_labels
    by_k, by_q = defaultdict(list), defaultdict(list)
    for k, a, j, f in g.flow:
        by_k[k].append((a, j, f))
    for q, a, j, f in g.outside:
        by_q[q].append((a, j, f))
    for k, T in enumerate(g.labels):
        assert PB.target_terms(g.labels, gl, T) == sorted(by_k[k]), k
    for q, T in enumerate(g.out_labels):
        assert PB.target_terms(g.labels, gl, T) == sorted(by_q[q]), q
