"""GPU parity of the RK4 coflow and its discrete adjoint (C ABI) vs the oracle."""
import numpy as np
import pytest

import gpu_util as U
import workloads
from oracle import algebra as A
from oracle import flow as OF
from oracle import gen as OG
from oracle import native

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    return _lib


def _flow(L, g, z0, ns, gen, prec, ds, ckpt_every=0, flags=None):
    z = torch.tensor(z0, device=DEV).contiguous()
    N, nops, nsets = z0.shape
    T = int(max(ns))
    ck = None
    if ckpt_every:
        ck = torch.zeros(((T + ckpt_every - 1) // ckpt_every, N, nops, nsets), dtype=torch.float64, device=DEV)
    p = L.flow_params(gen, prec, ds, 0.5, ckpt_every) if flags is None else \
        L.flow_params(gen, prec, ds, 0.5, ckpt_every, flags=flags)
    L.cut_flow_integrate(g, p, nsets, nops, list(ns), z, ck)
    torch.cuda.synchronize()
    return z.cpu().numpy(), ck


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_epq_wegner_flow_full_config(L):
    """n=8 one-body flow, Wegner generator as a graph pass, ds=1e-3 to s=10
    (10^4 RK4 steps): FP64 GPU flow vs the oracle with the same RK4."""
    U.say("[flow] epq n=8 wegner 10000 steps")
    w = workloads.WORKLOADS[1]
    inp = workloads.make_inputs(1)
    g = U.graph(L, "epq", 8)
    z, _ = _flow(L, g, inp.z0, inp.n_steps, L.CUT_GEN_WEGNER_GRAPH, L.CUT_F64, w.ds)
    og = A.epq_graph(8)
    zr, _ = native.Engine(og, "wegner_graph").flow(inp.z0, w.ds, inp.n_steps)
    assert np.max(np.abs(z - zr)) < 1e-10
    H0 = inp.z0[:, 0, 0].reshape(8, 8)
    H = z[:, 0, 0].reshape(8, 8)
    assert abs(np.linalg.norm(H) - np.linalg.norm(H0)) < 1e-8 * np.linalg.norm(H0)
    np.testing.assert_allclose(np.linalg.eigvalsh(H), np.linalg.eigvalsh(H0), atol=1e-7)


# default chunked form; quadratic-target blocks; blocks + shared-triple tiles
# default; blocks with XCD remap; blocks with tiles; B-chunk 16 with XCD remap
FLOW_TILINGS = [(1024, 512, 0), (1024, 512, 17), (1024, 512, 19), (1024, 512, 64 | 1)]


@pytest.mark.parametrize("tiling", FLOW_TILINGS)
@pytest.mark.parametrize("prec", ["F64", "F32X", "F32C"])
def test_majorana_flow_ragged(L, prec, tiling):
    U.say(f"[flow] majorana m=12 ragged {prec} tiling {tiling}")
    m = 12
    g = U.graph(L, "majorana", m)
    L.cut_graph_set_tiling(g, *tiling)
    og = A.majorana_graph(m)
    z0 = workloads.small_majorana(m, 5, 3, seed=21)
    ns = np.array([40, 0, 17, 40, 3], dtype=np.int32)
    z, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, getattr(L, "CUT_" + prec), 1e-2)
    L.cut_graph_set_tiling(g, 1024, 512, 0)
    gen, _ = OG.make_generator(og, "g2", 0.5)
    zr, _ = OF.integrate(og, gen, z0, 1e-2, ns)
    np.testing.assert_array_equal(z[:, :, 1], z0[:, :, 1])   # zero steps: untouched
    for s in range(5):
        for op in range(3):
            r = _rel(z[:, op, s], zr[:, op, s])
            assert r < (1e-13 if prec == "F64" else 1e-7), (s, op, r)


@pytest.mark.parametrize("tiling", [(1024, 512, 0), (64, 64, 1), (1024, 64, 8)])
@pytest.mark.parametrize("prec", ["F64", "F32C"])
def test_majorana_one_column_flow(L, prec, tiling):
    """One coefficient set, H only (the plain FP64 flow's shape: one-column
    passes, one record per lane), chunked tilings (at m = 24 the quadratic
    targets, 3,124 records, are the chunked ones in the first tiling; the others
    also cut quartic targets), hipGraph, against the oracle."""
    U.say(f"[flow] majorana m=24 one column {prec} tiling {tiling}")
    m = 24
    g = U.graph(L, "majorana", m)
    L.cut_graph_set_tiling(g, *tiling)
    og = A.majorana_graph(m)
    z0 = workloads.small_majorana(m, 1, 1, seed=29)
    z, _ = _flow(L, g, z0, [25], L.CUT_GEN_G2, getattr(L, "CUT_" + prec), 1e-2, flags=L.CUT_FLOW_HIPGRAPH)
    L.cut_graph_set_tiling(g, 1024, 512, 0)
    gen, _ = OG.make_generator(og, "g2", 0.5)
    zr, _ = OF.integrate(og, gen, z0, 1e-2, [25])
    r = _rel(z[:, 0, 0], zr[:, 0, 0])
    assert r < (1e-13 if prec == "F64" else 1e-7), r


@pytest.mark.parametrize("prec", ["F64", "F32C"])
def test_majorana_flow_g1(L, prec):
    """The literal generator G1 in the flow (ragged, hipGraph) against the
    oracle over a short window (G1 rotates coefficients instead of damping
    them, so longer flows amplify every rounding; see the precision study)."""
    U.say(f"[flow] majorana m=12 G1 {prec}")
    m = 12
    g = U.graph(L, "majorana", m)
    og = A.majorana_graph(m)
    z0 = workloads.small_majorana(m, 4, 2, seed=27)
    ns = np.array([10, 3, 10, 0], dtype=np.int32)
    z, _ = _flow(L, g, z0, ns, L.CUT_GEN_G1, getattr(L, "CUT_" + prec), 1e-2)
    gen, _ = OG.make_generator(og, "g1", 0.5)
    zr, _ = OF.integrate(og, gen, z0, 1e-2, ns)
    np.testing.assert_array_equal(z[:, :, 3], z0[:, :, 3])
    for s in range(4):
        for op in range(2):
            r = _rel(z[:, op, s], zr[:, op, s])
            assert r < (1e-12 if prec == "F64" else 1e-6), (s, op, r)


@pytest.mark.parametrize("tiling", FLOW_TILINGS)
def test_majorana_flow_many_sets(L, tiling):
    """40 ragged sets x 2 operands (64-lane form, tiles usable), F32C, hipGraph."""
    U.say(f"[flow] majorana m=12 40 sets tiling {tiling}")
    m = 12
    g = U.graph(L, "majorana", m)
    L.cut_graph_set_tiling(g, *tiling)
    og = A.majorana_graph(m)
    z0 = workloads.small_majorana(m, 40, 2, seed=23)
    ns = np.array([(7 * b) % 23 + 1 for b in range(40)], dtype=np.int32)
    z, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, L.CUT_F32C, 1e-2)
    L.cut_graph_set_tiling(g, 1024, 512, 0)
    gen, _ = OG.make_generator(og, "g2", 0.5)
    zr, _ = OF.integrate(og, gen, z0, 1e-2, ns)
    for s in range(40):
        for op in range(2):
            r = _rel(z[:, op, s], zr[:, op, s])
            assert r < 1e-7, (s, op, r)


@pytest.mark.parametrize("tiling", FLOW_TILINGS)
def test_flow_graph_replay_matches_stream_path(L, tiling):
    m = 10
    g = U.graph(L, "majorana", m)
    L.cut_graph_set_tiling(g, *tiling)
    z0 = workloads.small_majorana(m, 4, 2, seed=8)
    ns = [25, 10, 25, 1]
    a, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, L.CUT_F32C, 1e-2, flags=L.CUT_FLOW_HIPGRAPH)
    b, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, L.CUT_F32C, 1e-2, flags=0)
    c, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, L.CUT_F32C, 1e-2, flags=L.CUT_FLOW_HIPGRAPH)
    L.cut_graph_set_tiling(g, 1024, 512, 0)
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("prec", ["F64", "F32C"])
def test_ragged_flow_compacted_phases(L, prec):
    """24 sets whose active prefix shrinks through 16, 8, 4, 2 and 1 sets, so the
    flow repacks its state to ever fewer sets (writing the finished ones out):
    against the oracle per set and operand; bitwise the flow that keeps every
    set in its layout (a checkpointed flow: full states in caller order);
    hipGraph replays bitwise the stream path; a flow resumed inside a repacked
    phase bitwise the uninterrupted one; a set with zero steps untouched."""
    m = 12
    g = U.graph(L, "majorana", m)
    L.cut_graph_set_tiling(g, 1024, 512, 17)
    og = A.majorana_graph(m)
    nsets, nops = 24, 2
    z0 = workloads.small_majorana(m, nsets, nops, seed=31)
    ns = np.array([(5 * b) % 24 + 6 for b in range(nsets)], dtype=np.int32)
    ns[7] = 0
    ns[11] = 30
    P = getattr(L, "CUT_" + prec)
    U.say(f"[flow] compacted phases {prec}: hipGraph")
    a, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, P, 1e-2, flags=L.CUT_FLOW_HIPGRAPH)
    U.say(f"[flow] compacted phases {prec}: stream order")
    b, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, P, 1e-2, flags=0)
    U.say(f"[flow] compacted phases {prec}: resumed at step 22")
    z = torch.tensor(z0, device=DEV).contiguous()
    L.cut_flow_integrate(g, L.flow_params(L.CUT_GEN_G2, P, 1e-2, 0.5, step_end=22), nsets, nops, list(ns), z)
    L.cut_flow_integrate(g, L.flow_params(L.CUT_GEN_G2, P, 1e-2, 0.5, step_begin=22), nsets, nops, list(ns), z)
    torch.cuda.synchronize()
    c = z.cpu().numpy()
    U.say(f"[flow] compacted phases {prec}: checkpointed (uncompacted)")
    d, _ = _flow(L, g, z0, ns, L.CUT_GEN_G2, P, 1e-2, ckpt_every=4, flags=L.CUT_FLOW_HIPGRAPH)
    L.cut_graph_set_tiling(g, 1024, 512, 0)
    assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)
    np.testing.assert_array_equal(a[:, :, 7], z0[:, :, 7])
    gen, _ = OG.make_generator(og, "g2", 0.5)
    zr, _ = OF.integrate(og, gen, z0, 1e-2, ns)
    for s in range(nsets):
        for op in range(nops):
            r = _rel(a[:, op, s], zr[:, op, s])
            assert r < (1e-13 if prec == "F64" else 1e-7), (s, op, r)


def test_config2_short_flow_precision(L):
    """Majorana m=24 (config-2 graph, 2.56M records), H + 2 quadratic observables,
    100 RK4 steps: FP64 vs the oracle's C engine, float passes vs FP64."""
    U.say("[flow] m=24 config-2 inputs, 100 steps")
    w = workloads.WORKLOADS[2]
    inp = workloads.make_inputs(2)
    ns = [100]
    g = U.graph(L, "majorana", 24)
    z64, _ = _flow(L, g, inp.z0, ns, L.CUT_GEN_G2, L.CUT_F64, w.ds)
    og = A.majorana_graph(24)
    zr, _ = native.Engine(og, "g2", w.delta).flow(inp.z0, w.ds, ns)
    for op in range(3):
        assert _rel(z64[:, op, 0], zr[:, op, 0]) < 1e-12
    for prec, bound in (("F32C", 1e-7), ("F32X", 1e-7)):
        z, _ = _flow(L, g, inp.z0, ns, L.CUT_GEN_G2, getattr(L, "CUT_" + prec), w.ds)
        for op in range(3):
            assert _rel(z[:, op, 0], zr[:, op, 0]) < bound, (prec, op)


@pytest.mark.parametrize("alg,size,kind,nops", [("majorana", 10, "g2", 2), ("epq", 5, "wegner_graph", 1)])
def test_flow_adjoint_vs_oracle(L, alg, size, kind, nops):
    U.say(f"[adjoint flow] {alg} {size} {kind}")
    g = U.graph(L, alg, size)
    og = A.graph_for(alg, size)
    if alg == "majorana":
        z0 = workloads.small_majorana(size, 3, nops, seed=13)
        ns = np.array([23, 9, 0], dtype=np.int32)
    else:
        h = workloads.random_dense((size, size), seed=3)
        z0 = (h + h.T + np.diag(np.arange(size) * 1.0)).reshape(-1, 1, 1)
        ns = np.array([23], dtype=np.int32)
    ds, C = 1e-2, 5
    K = L.CUT_GEN_G2 if kind == "g2" else L.CUT_GEN_WEGNER_GRAPH
    z, ck = _flow(L, g, z0, ns, K, L.CUT_F64, ds, ckpt_every=C)
    lam_end = workloads.random_dense(z0.shape, seed=14)
    lam = torch.tensor(lam_end, device=DEV).contiguous()
    L.cut_flow_adjoint(g, L.flow_params(K, L.CUT_F64, ds, 0.5, C), z0.shape[2], z0.shape[1], list(ns), ck, lam)
    torch.cuda.synchronize()
    gen, vjp = OG.make_generator(og, kind, 0.5)
    ref = OF.flow_adjoint(og, gen, vjp, z0, ds, ns, lam_end, ckpt_every=C)
    assert _rel(lam.cpu().numpy(), ref) < 1e-12


def test_flow_function_autograd_config5_reduced(L):
    """Config-5 shape (m=24, 8 sets, H only, checkpoints every 16 steps) over a
    shortened flow: torch autograd through FlowFn vs the oracle's C-engine
    discrete adjoint, and vs central differences of FP64 GPU flows."""
    from paper_2609_14831_amd.flow import flow
    U.say("[autograd] m=24 8 sets 40 steps")
    w = workloads.WORKLOADS[5]
    inp = workloads.make_inputs(5, with_fd=4)
    g = U.graph(L, "majorana", 24)
    og = A.majorana_graph(24)
    ns = [40] * 8
    z0 = torch.tensor(inp.z0, device=DEV, requires_grad=True)
    zend = flow(z0, g, ns, L.CUT_GEN_G2, w.ds, w.delta, 16)
    pairs = torch.tensor(og.pairs, device=DEV)
    loss = zend[pairs, 0, :].sum()
    loss.backward()
    grad = z0.grad.cpu().numpy()
    lam_end = np.zeros_like(inp.z0)
    lam_end[og.pairs, 0, :] = 1.0
    ref = native.Engine(og, "g2", w.delta).flow_adjoint(inp.z0, w.ds, ns, lam_end, ckpt_every=16)
    assert _rel(grad, ref) < 1e-11
    with torch.no_grad():
        for d in inp.fd_dirs:
            v = torch.tensor(d[:, None, :], device=DEV)
            eps = 1e-6
            lp = flow(z0 + eps * v, g, ns, L.CUT_GEN_G2, w.ds, w.delta, 16)[pairs, 0, :].sum()
            lm = flow(z0 - eps * v, g, ns, L.CUT_GEN_G2, w.ds, w.delta, 16)[pairs, 0, :].sum()
            fd = float((lp - lm) / (2 * eps))
            an = float(np.sum(grad[:, 0, :] * d))
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * np.linalg.norm(grad)), (fd, an)


def test_pairing_drift_100_steps(L):
    """Duality invariant of the discrete flow (Eq. duality-invariant): an
    operand X flowed 100 RK4 steps with H on the config-2 graph (m = 24, 8 sets,
    FP64), and a dual w pulled back through the same steps by cut_flow_adjoint
    with no Hamiltonian cotangent, keep <w(0), X(0)> = <w(T), X(T)> up to
    rounding: X(T) is linear in X(0) for a fixed H(0), and w(0) is the
    transpose of that linear map applied to w(T)."""
    U.say("[pairing drift] m=24 8 sets 100 steps")
    m, nsets, ds, T, C = 24, 8, 5e-3, 100, 16
    g = U.graph(L, "majorana", m)
    z0 = workloads.small_majorana(m, nsets, 2, seed=81)
    ns = [T] * nsets
    z, ck = _flow(L, g, z0, ns, L.CUT_GEN_G2, L.CUT_F64, ds, ckpt_every=C)
    w_end = np.zeros_like(z0)
    w_end[:, 1, :] = workloads.random_dense((z0.shape[0], nsets), seed=82)
    lam = torch.tensor(w_end, device=DEV).contiguous()
    L.cut_flow_adjoint(g, L.flow_params(L.CUT_GEN_G2, L.CUT_F64, ds, 0.5, C), nsets, 2, ns, ck, lam)
    torch.cuda.synchronize()
    w0 = lam.cpu().numpy()[:, 1, :]
    before = np.sum(w0 * z0[:, 1, :], axis=0)
    after = np.sum(w_end[:, 1, :] * z[:, 1, :], axis=0)
    scale = np.sum(np.abs(w0 * z0[:, 1, :]), axis=0) + np.sum(np.abs(w_end[:, 1, :] * z[:, 1, :]), axis=0)
    drift = np.abs(after - before)
    U.say(f"[pairing drift] max |<w(T),X(T)> - <w(0),X(0)>| = {drift.max():.3e}, "
          f"relative {np.max(drift / scale):.3e}, |<w,X>| ~ {np.abs(after).max():.3e}")
    assert np.all(drift < 1e-13 * scale)
