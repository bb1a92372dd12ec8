"""Cross-check of the oracle's C engine against the (pinned) NumPy oracle."""
import numpy as np
import pytest

import workloads
from oracle import algebra as A
from oracle import flow as F
from oracle import gen as GEN
from oracle import graph as G
from oracle import native


@pytest.fixture(scope="module")
def maj10():
    return A.majorana_graph(10)


@pytest.mark.parametrize("m", [6, 10, 16])
def test_c_records_match_numpy_records(m):
    gc = native.majorana_graph(m)
    gp = A.majorana_graph(m)
    for f in ("k", "i", "j", "c"):
        np.testing.assert_array_equal(getattr(gc, f), getattr(gp, f))


def test_c_records_sampled_targets_m40():
    reg = A.MajoranaRegistry(40)
    t = np.array([0, 5, 779, 780, 50000, reg.N - 1])
    gc = native.majorana_graph(40, targets=t)
    gp = A.majorana_graph(40, targets=t)
    for f in ("k", "i", "j", "c"):
        np.testing.assert_array_equal(getattr(gc, f), getattr(gp, f))


def test_engine_actions_match_numpy(maj10):
    g = maj10
    eng = native.Engine(g, "g2", 0.5)
    rng = np.random.default_rng(1)
    eta = rng.normal(size=(g.N, 3))
    x = rng.normal(size=(g.N, 2, 3))
    w = rng.normal(size=(g.N, 2, 3))
    np.testing.assert_allclose(eng.apply(eta, x), G.apply(g, eta, x), rtol=0, atol=1e-12)
    np.testing.assert_allclose(eng.adjoint_x(eta, w), G.adjoint_x(g, eta, w), atol=1e-12)
    np.testing.assert_allclose(eng.adjoint_eta(w, x), G.adjoint_eta(g, w, x), atol=1e-12)


@pytest.mark.parametrize("alg,size,kind", [("majorana", 10, "g2"), ("epq", 5, "wegner_graph")])
def test_engine_flow_and_adjoint_match_numpy(alg, size, kind):
    g = A.graph_for(alg, size)
    eng = native.Engine(g, kind, 0.5)
    gen, vjp = GEN.make_generator(g, kind, 0.5)
    if alg == "majorana":
        z0 = workloads.small_majorana(size, 3, 2, seed=3)
        ns = np.array([11, 4, 0], dtype=np.int32)
    else:
        h = workloads.random_dense((size, size), seed=2)
        z0 = (h + h.T).reshape(-1, 1, 1)
        ns = np.array([11], dtype=np.int32)
    ds = 1e-2
    zc, ckc = eng.flow(z0, ds, ns, ckpt_every=4)
    zp, ckp = F.integrate(g, gen, z0, ds, ns, ckpt_every=4)
    np.testing.assert_allclose(zc, zp, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ckc, np.array(ckp), rtol=0, atol=1e-12)
    lam_end = workloads.random_dense(z0.shape, seed=9)
    lc = eng.flow_adjoint(z0, ds, ns, lam_end, ckpt_every=4)
    lp = F.flow_adjoint(g, gen, vjp, z0, ds, ns, lam_end, ckpt_every=4)
    np.testing.assert_allclose(lc, lp, rtol=0, atol=1e-11)
