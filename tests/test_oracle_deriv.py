"""Pins of the oracle's derivative functions (generator JVPs, action JVP/VJP).

The JVPs are checked against quantities that do not use them: the complex-step
derivative of the forward generator (exact to rounding for an analytic map),
the exactness of central differences for a quadratic map, second-order
convergence of finite differences of the forward action, and the pairing
<w, J v> = <J^T w, v> against the VJPs, which are pinned separately by finite
differences in test_oracle_flow.
"""
import numpy as np
import pytest

import workloads
from oracle import algebra as A
from oracle import deriv as D
from oracle import gen as GEN


def _graph(alg, size):
    return A.majorana_graph(size) if alg == "majorana" else A.epq_graph(size)


def _inputs(g, alg, size, nsets, nops, seed):
    if alg == "majorana":
        z = workloads.small_majorana(size, nsets, nops, seed=seed)
    else:
        z = workloads.random_dense((g.N, nops, nsets), seed=seed)
    return z[:, 0, :].copy(), z


def test_g2_jvp_matches_complex_step():
    m = 8
    gen = GEN.G2(m, 0.5)
    h = workloads.small_majorana(m, 3, 1, seed=4)[:, 0, :]
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.normal(size=h.shape)
        t = 1e-30
        cs = np.imag(gen(h + 1j * t * d)) / t
        np.testing.assert_allclose(gen.jvp(h, d), cs, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("alg,size", [("epq", 5), ("majorana", 8)])
def test_wegner_graph_jvp_is_exact_central_difference(alg, size):
    """The Wegner generator is quadratic in h, so (W(h+d) - W(h-d)) / 2 equals
    its derivative along d at any step length."""
    g = _graph(alg, size)
    h, _ = _inputs(g, alg, size, 2, 1, seed=6)
    d = workloads.random_dense(h.shape, seed=7)
    cd = 0.5 * (GEN.wegner_graph(g, h + d) - GEN.wegner_graph(g, h - d))
    jv = GEN.wegner_graph_jvp(g, h, d)
    assert np.max(np.abs(jv)) > 1e-3
    np.testing.assert_allclose(jv, cd, rtol=1e-12, atol=1e-12 * np.max(np.abs(cd)))


@pytest.mark.parametrize("alg,size,kind", [("majorana", 8, "g2"), ("majorana", 8, "wegner_graph"),
                                           ("epq", 5, "wegner_graph")])
def test_action_pairing_defect(alg, size, kind):
    """<w, dF(dh, dx)> = <g_h, dh> + <g_x, dx> with (g_h, g_x) = F'^T w."""
    g = _graph(alg, size)
    gen, vjp = GEN.make_generator(g, kind, 0.5)
    jvp = GEN.make_generator_jvp(g, kind, 0.5)
    h, x = _inputs(g, alg, size, 3, 2, seed=8)
    dh = workloads.random_dense(h.shape, seed=9)
    dx = workloads.random_dense(x.shape, seed=10)
    w = workloads.random_dense(x.shape, seed=11)
    defect, scale = D.pairing_defect(g, gen, jvp, vjp, h, x, dh, dx, w)
    assert scale > 1e-3
    assert abs(defect) < 1e-14 * scale
    # each half separately: the h and x directions
    zh, zx = np.zeros_like(h), np.zeros_like(x)
    for a, b in ((dh, zx), (zh, dx)):
        defect, scale = D.pairing_defect(g, gen, jvp, vjp, h, x, a, b, w)
        assert abs(defect) < 1e-14 * scale


def test_action_fd_scan_second_order_and_floor():
    """Centred differences of the forward action converge to the JVP at second
    order in the step (h direction) and are exact to rounding in the operand
    direction, where the action is linear."""
    m = 8
    g = A.majorana_graph(m)
    gen, _ = GEN.make_generator(g, "g2", 0.5)
    jvp = GEN.make_generator_jvp(g, "g2", 0.5)
    h, x = _inputs(g, "majorana", m, 2, 2, seed=12)
    steps = [1e-2, 1e-3, 1e-4, 1e-5]
    dh = workloads.random_dense(h.shape, seed=13)
    eh = D.fd_scan(g, gen, jvp, h, x, dh, "h", steps)
    # truncation error ~ eps^2 while it dominates rounding
    assert 50 < eh[1e-2] / eh[1e-3] < 200
    assert min(eh.values()) < 1e-9
    dx = workloads.random_dense(x.shape, seed=14)
    ex = D.fd_scan(g, gen, jvp, h, x, dx, "x", steps)
    assert max(ex.values()) < 1e-10


def test_action_jvp_matches_complex_step_of_action():
    """The action is linear in eta, so the complex step of F along (dh, dx) is
    apply(Im eta(h + i t dh) / t, x) + F(h, dx)."""
    from oracle import graph as G
    m = 8
    g = A.majorana_graph(m)
    gen = GEN.G2(m, 0.5)
    h, x = _inputs(g, "majorana", m, 2, 3, seed=15)
    dh = workloads.random_dense(h.shape, seed=16)
    dx = workloads.random_dense(x.shape, seed=17)
    t = 1e-30
    cs = G.apply(g, np.imag(gen(h + 1j * t * dh)) / t, x) + G.apply(g, gen(h), dx)
    jv = D.action_jvp(g, gen, gen.jvp, h, x, dh, dx)
    np.testing.assert_allclose(jv, cs, rtol=1e-12, atol=1e-13 * np.max(np.abs(cs)))
