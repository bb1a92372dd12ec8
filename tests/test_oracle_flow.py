"""Pins of the oracle's generators, RK4 coflow and discrete adjoint (CPU only)."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import brute
import workloads
from oracle import algebra as A
from oracle import flow as F
from oracle import gen as GEN
from oracle import graph as G


# ------------------------------------------------------------ generators ----

def test_epq_wegner_closed_form_and_dense():
    n = 8
    g = A.epq_graph(n)
    inp = workloads.make_inputs(1)
    h = inp.z0[:, 0, :]
    eta = GEN.wegner_graph(g, h)
    H = h[:, 0].reshape(n, n)
    closed = (np.diag(H)[:, None] - np.diag(H)[None, :]) * H
    np.fill_diagonal(closed, 0.0)
    np.testing.assert_allclose(eta[:, 0].reshape(n, n), closed, atol=1e-13)
    Hd = np.diag(np.diag(H))
    np.testing.assert_allclose(eta[:, 0].reshape(n, n), Hd @ (H - Hd) - (H - Hd) @ Hd,
                               atol=1e-13)
    assert np.allclose(closed, -closed.T)   # anti-Hermitian generator


def test_majorana_wegner_graph_matches_dense_block_generator():
    m = 8
    subs, mats = brute.dense_strings(m)
    g = A.majorana_graph(m)
    h = workloads.small_majorana(m, 1, 1, seed=4)[:, 0, :]
    Hd = np.einsum("a,axy->xy", np.where(g.diag, h[:, 0], 0.0), mats)
    Hod = np.einsum("a,axy->xy", np.where(g.diag, 0.0, h[:, 0]), mats)
    eta_op = Hd @ Hod - Hod @ Hd                      # anti-Hermitian
    coef = brute.project(mats, eta_op) / 1j           # coefficients of i*Gamma
    assert np.max(np.abs(coef.imag)) < 1e-12
    np.testing.assert_allclose(GEN.wegner_graph(g, h)[:, 0], coef.real, atol=1e-12)


def test_g2_numerator_is_quadratic_wegner_and_denominator_closed_form():
    m, delta = 8, 0.5
    subs, mats = brute.dense_strings(m)
    gen = GEN.G2(m, delta)
    h = workloads.small_majorana(m, 2, 1, seed=9)[:, 0, :]
    Nn, Q = gen._nq(h)
    for s in range(2):
        eps = [h[subs.index((2 * a, 2 * a + 1)), s] for a in range(m // 2)]
        H0 = sum(e * mats[subs.index((2 * a, 2 * a + 1))] for a, e in enumerate(eps))
        H = np.einsum("a,axy->xy", h[:, s], mats)
        coef = brute.project(mats, H0 @ H - H @ H0) / 1j
        np.testing.assert_allclose(Nn[:, s], coef.real, atol=1e-12)
        for t, S in enumerate(subs):
            flips = [a for a in range(m // 2) if ((2 * a) in S) != ((2 * a + 1) in S)]
            assert Q[t, s] == pytest.approx(4 * sum(eps[a] ** 2 for a in flips) + delta ** 2)
    eta = gen(h)
    assert np.all(eta[gen.reg.diag] == 0.0)


def test_g2_linearised_decay_rates_closed_form():
    """Around H0 = sum eps_a Gamma_{P_a}, the G2 flow of the off-diagonal strings
    is linear with eigenvalues -4 w^2 / Q_S, w running over the sums +-eps over
    the flipped pairs of S (the Bohr frequencies of ad_{H0} on that block)."""
    m, delta = 8, 0.5
    g = A.majorana_graph(m)
    gen = GEN.G2(m, delta)
    subs = A.majorana_subsets(m)
    eps = np.array([0.9, 0.4, -0.7, 0.25])
    h0 = np.zeros((g.N, 1))
    for a in range(m // 2):
        h0[subs.index((2 * a, 2 * a + 1)), 0] = eps[a]
    off = np.nonzero(~g.diag)[0]
    J = np.zeros((off.size, off.size))
    t = 1e-3
    for col, r in enumerate(off):
        v = np.zeros_like(h0); v[r, 0] = 1.0
        fp = G.apply(g, gen(h0 + t * v), (h0 + t * v)[:, None, :])[:, 0, 0]
        fm = G.apply(g, gen(h0 - t * v), (h0 - t * v)[:, None, :])[:, 0, 0]
        J[:, col] = ((fp - fm) / (2 * t))[off]
    ev = np.sort(np.linalg.eigvals(J).real)
    expect = []
    for S in (subs[r] for r in off):
        F_ = [a for a in range(m // 2) if ((2 * a) in S) != ((2 * a + 1) in S)]
        Q = 4 * sum(eps[a] ** 2 for a in F_) + delta ** 2
        # one string per block member; the block of 2^|F| strings carries the
        # 2^(|F|-1) frequencies |sum +-eps|, each twice
        expect.append((F_, Q))
    rates = []
    seen = {}
    for F_, Q in expect:
        seen.setdefault(tuple(F_), [0, Q])
        seen[tuple(F_)][0] += 1
    for F_, (count, Q) in seen.items():
        signs = np.array(np.meshgrid(*[[1, -1]] * len(F_))).reshape(len(F_), -1).T
        ws = [abs(np.dot(sg, eps[list(F_)])) for sg in signs]   # each w appears twice
        per = count // len(ws)
        for w in ws:
            rates += [-4 * w * w / Q] * per
    np.testing.assert_allclose(ev, np.sort(rates), atol=1e-9)
    assert ev.max() < 0


@pytest.mark.parametrize("kind", ["g2", "wegner_graph"])
def test_generator_vjp_matches_finite_differences(kind):
    m = 8
    g = A.majorana_graph(m)
    gen, vjp = GEN.make_generator(g, kind, 0.5)
    h = workloads.small_majorana(m, 2, 1, seed=1)[:, 0, :]
    gb = workloads.random_dense(h.shape, seed=3)
    gh = vjp(h, gb)
    rng = np.random.default_rng(8)
    for _ in range(4):
        v = rng.normal(size=h.shape)
        eps = 1e-6
        fd = (np.sum(gb * gen(h + eps * v)) - np.sum(gb * gen(h - eps * v))) / (2 * eps)
        assert np.sum(gh * v) == pytest.approx(fd, rel=1e-7, abs=1e-9)


# ---------------------------------------------------------------- RK4 --------

def test_rk4_step_is_fourth_order_taylor_of_linear_flow():
    """For a fixed generator the coflow is linear, dz/ds = L z; one classic RK4
    step equals sum_{p<=4} (ds L)^p / p! applied to z (L built from dense
    Jordan-Wigner commutators)."""
    m = 6
    subs, mats = brute.dense_strings(m)
    g = A.majorana_graph(m)
    N = len(subs)
    rng = np.random.default_rng(0)
    eta_fixed = rng.normal(size=(N, 1))
    etaop = np.einsum("a,axy->xy", 1j * eta_fixed[:, 0], mats)
    L = np.zeros((N, N))
    for col in range(N):
        L[:, col] = brute.project(mats, etaop @ mats[col] - mats[col] @ etaop).real
    z = rng.normal(size=(N, 2, 1))
    ds = 0.05
    z1 = F.rk4_step(g, lambda h: eta_fixed, z, ds, np.array([True]))
    P = sum(np.linalg.matrix_power(ds * L, p) / math.factorial(p) for p in range(5))
    np.testing.assert_allclose(z1[:, 0, 0], P @ z[:, 0, 0], atol=1e-13)
    # global error against the exact exponential is fourth order
    errs = []
    for nst in (10, 20):
        zz = z.copy()
        for _ in range(nst):
            zz = F.rk4_step(g, lambda h: eta_fixed, zz, 1.0 / nst, np.array([True]))
        errs.append(np.linalg.norm(zz[:, 1, 0] - expm(L) @ z[:, 1, 0]))
    assert 12 < errs[0] / errs[1] < 20


def test_epq_graph_flow_matches_dense_wegner_flow():
    n = 8
    g = A.epq_graph(n)
    inp = workloads.make_inputs(1)
    gen, _ = GEN.make_generator(g, "wegner_graph")
    ds, nst = 1e-3, 400
    z, _ = F.integrate(g, gen, inp.z0, ds, [nst])
    H0 = inp.z0[:, 0, 0].reshape(n, n)

    def f(H):
        Hd = np.diag(np.diag(H))
        eta = Hd @ H - H @ Hd
        return eta @ H - H @ eta

    Hd_end = brute.rk4_dense(f, H0, ds, nst)
    np.testing.assert_allclose(z[:, 0, 0].reshape(n, n), Hd_end, atol=1e-10)
    # invariants of a unitary flow, within RK4 error
    Hs = z[:, 0, 0].reshape(n, n)
    assert np.linalg.norm(Hs) == pytest.approx(np.linalg.norm(H0), rel=1e-9)
    np.testing.assert_allclose(np.linalg.eigvalsh(Hs), np.linalg.eigvalsh(H0), atol=1e-8)


def test_quadratic_majorana_flow_is_isospectral():
    """Quadratic strings close under the bracket; a quadratic h flows by an
    orthogonal conjugation of its 2n x 2n antisymmetric matrix A_ab = 2 h_ab,
    so the single-particle spectrum is conserved."""
    m = 12
    g = A.majorana_graph(m)
    gen, _ = GEN.make_generator(g, "g2", 0.5)
    z0 = workloads.small_majorana(m, 1, 1, seed=6)
    nq = math.comb(m, 2)
    z0[nq:] = 0.0
    def spectrum(h):
        Am = np.zeros((m, m))
        for t, (a, b) in enumerate(A.majorana_subsets(m)[:nq]):
            Am[a, b], Am[b, a] = 2 * h[t], -2 * h[t]
        return np.sort(np.abs(np.linalg.eigvals(Am).imag))

    errs = []
    for ds, nst in ((1e-2, 300), (5e-3, 600)):
        z, _ = F.integrate(g, gen, z0, ds, [nst])
        assert np.max(np.abs(z[nq:])) == 0.0
        errs.append(np.max(np.abs(spectrum(z[:nq, 0, 0]) - spectrum(z0[:nq, 0, 0]))))
    # conserved up to the integrator's error, which is fourth order in ds
    assert errs[1] < 1e-6
    assert 10 < errs[0] / errs[1] < 25
    # and the off-diagonal part decays (Wegner-type generator)
    off = ~g.diag[:nq]
    assert np.linalg.norm(z[:nq][off]) < 0.5 * np.linalg.norm(z0[:nq][off])


def test_majorana_flow_conserves_norm_and_gram():
    """For any real eta the action is antisymmetric (orthonormal basis, orthogonal
    projection), so |h|^2, |o|^2 and <h, o> are conserved up to RK4 error."""
    m = 10
    g = A.majorana_graph(m)
    gen, _ = GEN.make_generator(g, "g2", 0.5)
    z0 = workloads.small_majorana(m, 2, 3, seed=2, obs_quartic=True)
    drift = []
    for ds, nst in ((1e-2, 50), (5e-3, 100)):
        z, _ = F.integrate(g, gen, z0, ds, [nst, nst])
        gram0 = np.einsum("nas,nbs->sab", z0, z0)
        gram = np.einsum("nas,nbs->sab", z, z)
        drift.append(np.max(np.abs(gram - gram0)) / np.max(np.abs(gram0)))
    assert drift[1] < 1e-6
    assert drift[0] / drift[1] > 8     # vanishes at fourth order in ds


def test_ragged_sets_independent():
    m = 8
    g = A.majorana_graph(m)
    gen, _ = GEN.make_generator(g, "g2", 0.5)
    z0 = workloads.small_majorana(m, 3, 2, seed=12)
    ns = np.array([7, 0, 3])
    z, _ = F.integrate(g, gen, z0, 1e-2, ns)
    np.testing.assert_array_equal(z[:, :, 1], z0[:, :, 1])
    for s in (0, 2):
        zs, _ = F.integrate(g, gen, z0[:, :, s:s + 1], 1e-2, ns[s:s + 1])
        np.testing.assert_allclose(z[:, :, s], zs[:, :, 0], rtol=0, atol=1e-14)


# -------------------------------------------------------------- adjoint ------

@pytest.mark.parametrize("alg,size,kind,nops", [("majorana", 8, "g2", 2),
                                               ("epq", 4, "wegner_graph", 1)])
def test_discrete_adjoint_matches_central_differences(alg, size, kind, nops):
    g = A.graph_for(alg, size)
    gen, vjp = GEN.make_generator(g, kind, 0.5)
    if alg == "majorana":
        z0 = workloads.small_majorana(size, 2, nops, seed=5)
        ns = np.array([9, 6])
    else:
        h = workloads.random_dense((size, size), seed=1)
        h = h + h.T + np.diag(np.arange(size) * 1.0)
        z0 = h.reshape(-1, 1, 1)
        ns = np.array([9])
    ds = 2e-2
    wts = workloads.random_dense(z0.shape, seed=6)

    def loss(z):
        zend, _ = F.integrate(g, gen, z, ds, ns)
        return np.sum(wts * zend)

    lam = F.flow_adjoint(g, gen, vjp, z0, ds, ns, wts, ckpt_every=4)
    lam1 = F.flow_adjoint(g, gen, vjp, z0, ds, ns, wts, ckpt_every=1)
    np.testing.assert_array_equal(lam, lam1)
    rng = np.random.default_rng(4)
    for _ in range(3):
        v = rng.normal(size=z0.shape)
        eps = 1e-5
        fd = (loss(z0 + eps * v) - loss(z0 - eps * v)) / (2 * eps)
        assert np.sum(lam * v) == pytest.approx(fd, rel=2e-8)


# ---------------------------------------------------- sampled-row action ----

@pytest.mark.parametrize("m", [10, 12])
def test_apply_rows_equals_apply_at_those_rows(m):
    """apply_rows (the reference of every full-size sampled GPU test) on the
    records of just the sampled targets equals the pinned whole-graph apply at
    those rows, including the first and last quadratic and quartic targets.
    A selection by the wrong record field or the wrong operand row fails."""
    full = A.majorana_graph(m)
    nq = math.comb(m, 2)
    rng = np.random.default_rng(m)
    rows = np.array([0, 1, nq - 1, nq, nq + 1, full.N - 1] + list(rng.integers(0, full.N, 10)))
    sub = A.majorana_graph(m, targets=rows)
    eta = workloads.random_dense((full.N, 3), seed=30 + m)
    x = workloads.random_dense((full.N, 2, 3), seed=40 + m)
    ref = G.apply(full, eta, x)[rows]
    scale = np.abs(ref).max()
    np.testing.assert_allclose(G.apply_rows(sub, eta, x, rows), ref, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(G.apply_rows(full, eta, x, rows), ref, rtol=0, atol=1e-13 * scale)

    # the same sum with a mistake in the selection must not pass
    def planted(g, e, xx, rr, key):
        out = np.zeros((len(rr),) + xx.shape[1:])
        for t, r in enumerate(rr):
            sel = key(g) == r
            out[t] = np.sum(g.c[sel, None, None] * e[g.i[sel]][:, None, :] * xx[g.j[sel]], axis=0)
        return out

    for key in (lambda g: g.i, lambda g: g.j):
        assert np.abs(planted(full, eta, x, rows, key) - ref).max() > 1e-3 * scale


# ------------------------------------------------------------------- G1 ----

def test_g1_closed_form_on_hand_built_hamiltonian():
    """eta_S = h_S / (2 sum_{a in F(S)} |eps_a| + delta) on a hand-built
    H_0 + V at m = 8 (pairs (0,1), (2,3), (4,5), (6,7)), with the flipped pairs
    of each string written out by hand: {0,2} flips pairs 0 and 1, {1,6}
    pairs 0 and 3, {0,1,2,4} pairs 1 and 2, {0,2,4,6} all four, {2,3,4,7}
    pairs 2 and 3; the diagonal strings {0,1} and {0,1,2,3} get eta = 0."""
    m, delta = 8, 0.25
    reg = A.MajoranaRegistry(m)
    row = lambda modes: int(reg.index_of(np.array([sum(1 << q for q in modes)], dtype=np.uint64))[0])
    eps = [0.9, -0.4, 1.3, -2.0]
    h = np.zeros((reg.N, 1))
    for a, e in enumerate(eps):
        h[row((2 * a, 2 * a + 1)), 0] = e
    V = {(0, 2): 0.3, (1, 6): -0.7, (0, 1, 2, 4): 0.11, (0, 2, 4, 6): -0.05, (2, 3, 4, 7): 0.2}
    flips = {(0, 2): (0, 1), (1, 6): (0, 3), (0, 1, 2, 4): (1, 2), (0, 2, 4, 6): (0, 1, 2, 3), (2, 3, 4, 7): (2, 3)}
    for S, v in V.items():
        h[row(S), 0] = v
    h[row((0, 1, 2, 3)), 0] = 0.6          # a diagonal quartic
    eta = GEN.G1(m, delta)(h)
    for S, v in V.items():
        want = v / (2 * sum(abs(eps[a]) for a in flips[S]) + delta)
        assert abs(eta[row(S), 0] - want) < 1e-15
    for S in ((0, 1), (2, 3), (0, 1, 2, 3)):
        assert eta[row(S), 0] == 0.0
    assert np.count_nonzero(eta) == len(V)


@pytest.mark.parametrize("m", [8, 10])
def test_g1_jvp_and_vjp(m):
    """G1's JVP against central differences (exact up to rounding away from
    eps_a = 0: eta is a rational function there) and its VJP against the JVP
    through <gbar, J dh> = <J^T gbar, dh>."""
    g1 = GEN.G1(m, 0.5)
    h = workloads.small_majorana(m, 3, 1, seed=17)[:, 0, :]
    dh = workloads.random_dense(h.shape, seed=18)
    jv = g1.jvp(h, dh)
    for step in (1e-5, 1e-6):
        fd = (g1(h + step * dh) - g1(h - step * dh)) / (2 * step)
        assert np.abs(fd - jv).max() < 1e-7 * np.abs(jv).max()
    gbar = workloads.random_dense(h.shape, seed=19)
    lhs = np.sum(gbar * jv)
    rhs = np.sum(g1.vjp(h, gbar) * dh)
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1.0)


def test_g1_engine_flow_matches_numpy_flow():
    """The C engine's G1 flow equals the NumPy oracle's (same RK4, same records)."""
    from oracle import native
    m = 10
    g = A.majorana_graph(m)
    z0 = workloads.small_majorana(m, 2, 2, seed=23)
    gen, _ = GEN.make_generator(g, "g1", 0.5)
    zr, _ = F.integrate(g, gen, z0, 1e-2, [15, 9])
    ze, _ = native.Engine(g, "g1", 0.5).flow(z0, 1e-2, [15, 9])
    assert np.abs(ze - zr).max() < 1e-12 * np.abs(zr).max()
