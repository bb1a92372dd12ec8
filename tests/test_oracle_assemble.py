"""Pins of the oracle's multi-operator assembly: the written-out definition on
small cases, exact selection, and the linearity of the transform (assembling
transformed sources equals transforming the assembled sources)."""
import numpy as np

import workloads
from oracle import algebra as A
from oracle import assemble as AS
from oracle import flow as OF
from oracle import gen as OG


def test_assemble_matches_definition():
    X = workloads.random_dense((7, 5), seed=1)
    W = workloads.random_dense((5, 9), seed=2)
    np.testing.assert_allclose(AS.assemble(X, W), AS.assemble_loops(X, W), rtol=1e-14, atol=1e-14)


def test_assemble_selection_is_exact():
    X = workloads.random_dense((11, 6), seed=3)
    W = np.zeros((6, 4))
    W[[5, 0, 3, 3], [0, 1, 2, 3]] = 1.0
    W[1, 3] = -1.0
    Y = AS.assemble(X, W)
    np.testing.assert_array_equal(Y[:, :3], X[:, [5, 0, 3]])
    np.testing.assert_array_equal(Y[:, 3], X[:, 3] - X[:, 1])


def test_assembly_commutes_with_the_transform():
    """Flow 6 source operators with one Hamiltonian (m = 8, G2, 10 RK4 steps);
    combining the flowed sources equals flowing the combined sources."""
    m, S, K = 8, 6, 5
    g = A.majorana_graph(m)
    gen, _ = OG.make_generator(g, "g2", 0.5)
    h = workloads.small_majorana(m, 1, 1, seed=4)[:, 0, 0]
    X0 = workloads.random_dense((g.N, S), seed=5)
    W = workloads.random_dense((S, K), seed=6)

    def transform(ops):
        z = np.zeros((g.N, 1 + ops.shape[1], 1))
        z[:, 0, 0] = h
        z[:, 1:, 0] = ops
        zt, _ = OF.integrate(g, gen, z, 0.01, [10])
        return zt[:, 1:, 0]

    XT = transform(X0)
    np.testing.assert_allclose(AS.assemble(XT, W), transform(AS.assemble(X0, W)), rtol=1e-11,
                               atol=1e-12 * np.abs(XT).max())
