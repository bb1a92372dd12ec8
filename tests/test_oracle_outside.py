"""Pins of the oracle's outside-space records E_C (Majorana strings).

C_X = (I - P)[eta, X] (Eq. projected-flow) is checked against dense
Jordan-Wigner commutators: the full commutator of random eta (generator basis
i Gamma) and X must equal the retained action on the registry plus the
outside-space action on the 6-subsets, with nothing left over; record counts
against the closed form; the factor antisymmetry c(Q; A, B) = -c(Q; B, A).
"""
import numpy as np
import pytest

import brute
from oracle import algebra as A
from oracle import graph as G


@pytest.mark.parametrize("m", [8, 10])
def test_outside_action_completes_dense_commutator(m):
    subs, mats = brute.dense_strings(m)
    osubs, omats = brute.dense_strings_of_degree(m, 6)
    g = A.majorana_graph(m)
    og = A.majorana_outside_graph(m)
    assert og.n_out == len(osubs)
    rng = np.random.default_rng(m)
    eta = rng.normal(size=(len(subs), 1))
    x = rng.normal(size=(len(subs), 1, 1))
    etaop = np.einsum("a,axy->xy", 1j * eta[:, 0], mats)
    xop = np.einsum("a,axy->xy", x[:, 0, 0], mats)
    M = etaop @ xop - xop @ etaop
    F = G.apply(g, eta, x)[:, 0, 0]
    C = G.apply_outside(og, eta, x)[:, 0, 0]
    np.testing.assert_allclose(brute.project(omats, M).real, C, atol=1e-10)
    rebuilt = np.einsum("a,axy->xy", F, mats) + np.einsum("a,axy->xy", C, omats)
    assert np.max(np.abs(M - rebuilt)) < 1e-10


@pytest.mark.parametrize("m", [6, 8, 10, 12, 14])
def test_outside_counts_closed_form(m):
    og = A.majorana_outside_graph(m)
    assert og.E == A.majorana_outside_count(m)
    if og.n_out:
        per = np.diff(og.offsets())
        assert np.all(per == 20 * (m - 6))


def test_outside_records_structure_and_antisymmetry():
    m = 12
    og = A.majorana_outside_graph(m)
    reg = A.MajoranaRegistry(m)
    a, b = reg.masks[og.i], reg.masks[og.j]
    assert np.all(np.bitwise_count(a) == 4) and np.all(np.bitwise_count(b) == 4)
    assert np.all(np.bitwise_count(a & b) == 1)
    assert np.all((a ^ b) == og.masks[og.k])
    assert set(np.unique(og.c)) <= {-2.0, 2.0}
    key = {(int(k), int(i), int(j)): c for k, i, j, c in zip(og.k, og.i, og.j, og.c)}
    for (k, i, j), c in list(key.items())[:5000]:
        assert key[(k, j, i)] == -c


def test_flow_outside_diagnostic_matches_dense_commutators():
    """One RK4 step at m = 8: the leak equals sum_s b_s ds |(I - P)[eta_s, Z_s]|^2
    with the outside part taken from dense matrices as the full Frobenius norm
    (orthonormal string basis) minus the registry part, and the flowed state
    equals the plain integrator's."""
    from oracle import flow as OF
    from oracle import gen as OG
    m = 8
    subs, mats = brute.dense_strings(m)
    dim = mats.shape[-1]
    g = A.majorana_graph(m)
    og = A.majorana_outside_graph(m)
    gen, _ = OG.make_generator(g, "g2", 0.5)
    rng = np.random.default_rng(4)
    z0 = rng.normal(size=(g.N, 2, 2))
    ds = 0.05
    z1, leak = OF.integrate_outside(g, gen, og, z0, ds, [1, 1])
    zr, _ = OF.integrate(g, gen, z0, ds, [1, 1])
    np.testing.assert_array_equal(z1, zr)
    ref = np.zeros((2, 2))
    stage, ks = z0, []
    for s, b in enumerate(OF.RK4_WEIGHTS):
        k, eta = OF.rhs(g, gen, stage)
        for op in range(2):
            for st in range(2):
                etaop = np.einsum("a,axy->xy", 1j * eta[:, st], mats)
                xop = np.einsum("a,axy->xy", stage[:, op, st], mats)
                M = etaop @ xop - xop @ etaop
                total = np.sum(np.abs(M) ** 2) / dim
                inside = np.sum(np.abs(brute.project(mats, M)) ** 2)
                ref[op, st] += b * ds * (total - inside)
        ks.append(k)
        if s < 3:
            stage = z0 + (0.5 if s < 2 else 1.0) * ds * k
    assert np.max(ref) > 1e-3
    np.testing.assert_allclose(leak, ref, rtol=1e-10)


def test_flow_outside_zero_in_closed_quadratic_algebra():
    """Quadratic strings close under the bracket: with no quartic coefficients
    the flow never leaves degree 2 and the outside action vanishes."""
    from oracle import flow as OF
    from oracle import gen as OG
    m = 10
    g = A.majorana_graph(m)
    og = A.majorana_outside_graph(m)
    gen, _ = OG.make_generator(g, "g2", 0.5)
    rng = np.random.default_rng(5)
    z0 = np.zeros((g.N, 2, 3))
    nq = m * (m - 1) // 2
    z0[:nq] = rng.normal(size=(nq, 2, 3))
    _, leak = OF.integrate_outside(g, gen, og, z0, 0.02, [5, 3, 0])
    assert np.all(leak == 0.0)
