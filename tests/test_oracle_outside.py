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
