"""GPU parity at the workloads' full sizes.

* config 3 (m=40, 39.5M records, 64 sets x 5 operands), in the launch
  configuration bench.py times (G2 generator, compensated float passes, RK4 steps
  replayed from one hipGraph, default tiling): two whole RK4 steps of every
  coefficient against the oracle's C engine; sampled single actions per target;
* config 3 directional derivative (cut_graph_jvp) on sampled targets;
* config 3, the whole ragged flow of all 64 sets (421 ... 3,660 steps) in the
  benchmark's launch configuration: the shortest and the longest set against
  the oracle's C engine;
* config 4 (m=64, 457.7M records, 16 sets): sampled single actions per target;
  two RK4 steps of sets 0 and 15 against the oracle's C engine; the 200-step
  flow (float passes vs FP64 passes, norm conservation); norm drift at 4th
  order;
* config 2: the whole flow to s=10 against the oracle's stored flow;
* config 5: the whole-flow gradient against the oracle's stored discrete adjoint
  and central differences of FP64 flows (32 directions).

Tolerances: flowed coefficients within 1e-7 (norm-wise relative, per set and
operand) for the float passes, 1e-11 for FP64; gradients within 1e-6 of central
differences.
"""
import os

import numpy as np
import pytest

import gpu_util as U
import workloads
from oracle import algebra as A
from oracle import gen as OG
from oracle import graph as OGr
from oracle import native

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    return _lib


def _rel_cols(a, b):
    """max over (op, set) of |a - b|_2 / |b|_2 along the registry axis."""
    num = np.linalg.norm(a - b, axis=0)
    den = np.linalg.norm(b, axis=0)
    return float(np.max(num / den))


def _flow(L, g, z0, ns, prec, w, steps=None, flags=None):
    z = torch.tensor(z0, device=DEV).contiguous()
    N, nops, nsets = z0.shape
    p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0,
                      flags=L.CUT_FLOW_HIPGRAPH if flags is None else flags,
                      step_begin=0, step_end=-1 if steps is None else steps)
    L.cut_flow_integrate(g, p, nsets, nops, [int(v) for v in ns], z)
    torch.cuda.synchronize()
    return z.cpu().numpy()


@pytest.fixture(scope="module")
def cfg3(L):
    w = workloads.WORKLOADS[3]
    U.say("[cfg3] build + load m=40")
    g = U.graph(L, "majorana", 40, adjoint=False)
    # the tiling the benchmark runs: autotuned for 64 sets x 5 operands, F32C
    U.say(f"[cfg3] autotuned {L.cut_graph_autotune(g, w.nsets, w.nops, L.CUT_F32C, 0)}")
    return g, w, workloads.make_inputs(3)


@pytest.fixture(scope="module")
def cfg3_oracle():
    U.say("[cfg3] oracle graph (C engine)")
    return native.majorana_graph(40)


@pytest.mark.timeout(600)
def test_cfg3_two_rk4_steps_every_coefficient(L, cfg3, cfg3_oracle):
    g, w, inp = cfg3
    U.say("[cfg3] oracle 2 RK4 steps on 64 sets x 5 operands")
    zr, _ = native.Engine(cfg3_oracle, "g2", w.delta).flow(inp.z0, w.ds, [2] * w.nsets)
    # each precision in the tiling the benchmark's autotuner picks for it (F32C
    # first: the fixture tuned it), F32X also with quadratic-target blocks + tiles
    runs = (("F32C", 1e-7, None), ("F32X", 1e-7, "auto"), ("F32X", 1e-7, (1024, 512, 19)), ("F64", 1e-11, None))
    for name, tol, tiling in runs:
        if tiling == "auto":
            U.say(f"[cfg3] autotuned {L.cut_graph_autotune(g, w.nsets, w.nops, L.CUT_F32X, 0)}")
        elif tiling is not None:
            L.cut_graph_set_tiling(g, *tiling)
        U.say(f"[cfg3] GPU 2 steps {name} tiling {tiling}")
        z = _flow(L, g, inp.z0, inp.n_steps, getattr(L, "CUT_" + name), w, steps=2)
        r = _rel_cols(z - inp.z0, zr - inp.z0)
        U.say(f"[cfg3] {name}: max relative error of the 2-step increment {r:.3e}")
        assert _rel_cols(z, zr) < tol
        assert r < (1e-6 if name != "F64" else 1e-10)
    t = L.cut_graph_autotune(g, w.nsets, w.nops, L.CUT_F32C, 0)   # cached: restores the F32C tiling
    L.cut_graph_set_tiling(g, t["long_records"], t["chunk_records"], t["tiling_flags"])


def _flow_windows(L, g, z0, ns, prec, w, what, window=1000):
    """The whole ragged flow in the benchmark's launch configuration (hipGraph
    replays, the graph's current tiling), in windows of `window` steps resumed
    from the state (bitwise the uninterrupted flow), printing its progress."""
    z = torch.tensor(z0, device=DEV).contiguous()
    N, nops, nsets = z0.shape
    T = int(max(ns))
    for t0 in range(0, T, window):
        p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                          step_begin=t0, step_end=min(T, t0 + window))
        L.cut_flow_integrate(g, p, nsets, nops, [int(v) for v in ns], z)
        torch.cuda.synchronize()
        U.say(f"[{what}] steps {t0} .. {min(T, t0 + window)} of {T}")
    return z.cpu().numpy()


@pytest.mark.timeout(900)
def test_cfg3_full_ragged_flow_shortest_and_longest_set(L, cfg3):
    """All 64 sets over their whole uneven flows (421 ... 3,660 RK4 steps), in
    the benchmark's launch configuration; the shortest and the longest set
    against the oracle's C engine flowing that set alone (stored by
    tests/golden/make_oracle_goldens.py): F32C / F32X within 1e-7, F64 within
    1e-11 (norm-wise per operand)."""
    g, w, inp = cfg3
    sets = []
    for name in os.listdir(GOLD):
        if name.startswith("cfg3_full_flow_set"):
            sets.append(int(name[len("cfg3_full_flow_set"):-4]))
    if len(sets) < 2:
        pytest.skip("oracle goldens not generated")
    ns = inp.n_steps
    assert sorted(sets) == sorted([int(np.argmin(ns)), int(np.argmax(ns))])
    refs = {b: np.load(os.path.join(GOLD, f"cfg3_full_flow_set{b}.npy"))[:, :, 0] for b in sets}
    for name, tol in (("F32C", 1e-7), ("F32X", 1e-7), ("F64", 1e-11)):
        P = getattr(L, "CUT_" + name)
        U.say(f"[cfg3 full] autotuned {name}: {L.cut_graph_autotune(g, w.nsets, w.nops, P, 0)}")
        z = _flow_windows(L, g, inp.z0, ns, P, w, f"cfg3 full {name}")
        for b in sets:
            err = _rel_cols(z[:, :, b], refs[b])
            U.say(f"[cfg3 full] {name} set {b} ({int(ns[b])} steps): relative error {err:.3e}")
            assert err < tol
        # every set moved, and none past its own end: a frozen set's state is
        # the state its last step left (checked through the norm, which the flow
        # conserves to RK4 accuracy)
        n0 = np.linalg.norm(inp.z0, axis=0)
        drift = np.max(np.abs(np.linalg.norm(z, axis=0) - n0) / n0)
        U.say(f"[cfg3 full] {name} max norm drift {drift:.3e}")
        assert drift < 1e-4
    t = L.cut_graph_autotune(g, w.nsets, w.nops, L.CUT_F32C, 0)   # cached: restores the F32C tiling
    L.cut_graph_set_tiling(g, t["long_records"], t["chunk_records"], t["tiling_flags"])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("tiling", [None, (1024, 512, 0), (1024, 64, 9), (1024, 128, 8)])
def test_cfg3_sampled_single_actions(L, cfg3, tiling):
    g, w, inp = cfg3
    if tiling is not None:
        L.cut_graph_set_tiling(g, *tiling)
    reg = A.MajoranaRegistry(40)
    rows = np.array([0, 1, 779, 780, 781, 40000, reg.N - 1] +
                    list(np.random.default_rng(5).integers(0, reg.N, 25)))
    og = A.majorana_graph(40, targets=rows)
    eta = OG.G2(40, w.delta)(inp.z0[:, 0, :])
    x = inp.z0
    ref = OGr.apply_rows(og, eta, x, rows)
    ga = A.Graph("majorana", 40, og.N, og.k, og.i, og.j, np.abs(og.c), og.diag, og.pairs, 1.0)
    S = OGr.apply_rows(ga, np.abs(eta), np.abs(x), rows)
    for name in ("F64", "F32X", "F32C"):
        P = getattr(L, "CUT_" + name)
        dt = torch.float64 if P == L.CUT_F64 else torch.float32
        y = torch.zeros((reg.N, 320), dtype=torch.float64, device=DEV)
        L.cut_graph_apply(g, 0, P, 64, 5, torch.tensor(eta, device=DEV).to(dt),
                          torch.tensor(x.reshape(reg.N, 320), device=DEV).to(dt), y)
        torch.cuda.synchronize()
        got = y.cpu().numpy().reshape(reg.N, 5, 64)[rows]
        bound = {"F64": U.sum_bound(16948), "F32X": 2 * U.U32 + U.sum_bound(16948),
                 "F32C": 2 * U.U32 + U.dot2_bound(16948)}[name] * S + 1e-300
        U.assert_within(got, ref, bound, f"cfg3 sampled {name} tiling {tiling}")
    t = L.cut_graph_autotune(g, w.nsets, w.nops, L.CUT_F32C, 0)   # cached: restores the tuned tiling
    L.cut_graph_set_tiling(g, t["long_records"], t["chunk_records"], t["tiling_flags"])


@pytest.mark.timeout(300)
def test_cfg3_sampled_directional_derivative(L, cfg3):
    """cut_graph_jvp at full size (64 sets x 5 operands, the benchmark's tiling)
    on sampled targets: dy = apply(eta'(h) dh, x) + apply(eta(h), dx) and
    y = apply(eta(h), x) against the oracle's rows; bounds as the sampled
    single actions, with S the sums over |terms| of both products."""
    g, w, inp = cfg3
    reg = A.MajoranaRegistry(40)
    rows = np.array([0, 5, 779, 780, 90000, reg.N - 1] + list(np.random.default_rng(7).integers(0, reg.N, 20)))
    og = A.majorana_graph(40, targets=rows)
    ga = A.Graph("majorana", 40, og.N, og.k, og.i, og.j, np.abs(og.c), og.diag, og.pairs, 1.0)
    h = inp.z0[:, 0, :]
    x = inp.z0
    dh = workloads.random_dense(h.shape, seed=71)
    dx = workloads.random_dense(x.shape, seed=72)
    gen = OG.G2(40, w.delta)
    eta, deta = gen(h), gen.jvp(h, dh)
    ref = OGr.apply_rows(og, deta, x, rows) + OGr.apply_rows(og, eta, dx, rows)
    S = OGr.apply_rows(ga, np.abs(deta), np.abs(x), rows) + OGr.apply_rows(ga, np.abs(eta), np.abs(dx), rows)
    yref = OGr.apply_rows(og, eta, x, rows)
    Sy = OGr.apply_rows(ga, np.abs(eta), np.abs(x), rows)
    for name in ("F32C", "F64"):
        P = getattr(L, "CUT_" + name)
        U.say(f"[cfg3] jvp {name}")
        y = torch.zeros((reg.N, 320), dtype=torch.float64, device=DEV)
        dy = torch.zeros((reg.N, 320), dtype=torch.float64, device=DEV)
        L.cut_graph_jvp(g, L.CUT_GEN_G2, w.delta, P, 64, 5, torch.tensor(h, device=DEV).contiguous(),
                        torch.tensor(dh, device=DEV), torch.tensor(x.reshape(reg.N, 320), device=DEV),
                        torch.tensor(dx.reshape(reg.N, 320), device=DEV), y, dy)
        torch.cuda.synchronize()
        pb = {"F64": U.sum_bound(16948), "F32C": 2 * U.U32 + U.dot2_bound(16948)}[name]
        got = dy.cpu().numpy().reshape(reg.N, 5, 64)[rows]
        U.assert_within(got, ref, pb * S + 1e-12 * np.abs(ref).max(), f"cfg3 jvp dy {name}")
        goty = y.cpu().numpy().reshape(reg.N, 5, 64)[rows]
        U.assert_within(goty, yref, pb * Sy + 1e-12 * np.abs(yref).max(), f"cfg3 jvp y {name}")


@pytest.mark.timeout(900)
def test_cfg4_stress_graph(L):
    w = workloads.WORKLOADS[4]
    U.say("[cfg4] build m=64 (457.7M records)")
    path = U.bundle_path(L, "majorana", 64)
    desc = None
    g = L.cut_graph_load(path, 0, 0)
    try:
        desc = L.cut_graph_info(g)
        assert desc["n_records"] == 457_720_704 and desc["n_ops"] == 637_392
        inp = workloads.make_inputs(4)
        reg = A.MajoranaRegistry(64)
        rows = np.array([0, 2015, 2016, reg.N // 2, reg.N - 1] +
                        list(np.random.default_rng(6).integers(0, reg.N, 11)))
        U.say("[cfg4] oracle sampled targets")
        og = native.majorana_graph(64, targets=rows)
        eta = OG.G2(64, w.delta)(inp.z0[:, 0, :])
        ref = OGr.apply_rows(og, eta, inp.z0, rows)
        ga = A.Graph("majorana", 64, og.N, og.k, og.i, og.j, np.abs(og.c), og.diag, og.pairs, 1.0)
        S = OGr.apply_rows(ga, np.abs(eta), np.abs(inp.z0), rows)
        for name, tiling in (("F64", (1024, 512, 0)), ("F32C", (1024, 512, 0)), ("F32C", (1024, 128, 9))):
            U.say(f"[cfg4] apply {name} tiling {tiling}")
            L.cut_graph_set_tiling(g, *tiling)
            P = getattr(L, "CUT_" + name)
            dt = torch.float64 if P == L.CUT_F64 else torch.float32
            y = torch.zeros((reg.N, 16), dtype=torch.float64, device=DEV)
            L.cut_graph_apply(g, 0, P, 16, 1, torch.tensor(eta, device=DEV).to(dt),
                              torch.tensor(inp.z0.reshape(reg.N, 16), device=DEV).to(dt), y)
            torch.cuda.synchronize()
            got = y.cpu().numpy().reshape(reg.N, 1, 16)[rows]
            bound = {"F64": U.sum_bound(75764), "F32C": 2 * U.U32 + U.dot2_bound(75764)}[name] * S + 1e-300
            U.assert_within(got, ref, bound, f"cfg4 sampled {name} tiling {tiling}")
        gold = os.path.join(GOLD, "cfg4_two_steps.npy")
        if os.path.exists(gold):
            # two whole RK4 steps of all 16 sets in the benchmark's launch
            # configuration (autotuned, hipGraph); sets 0 and 15 against the
            # oracle's C engine (stored by tests/golden/make_oracle_goldens.py)
            zr = np.load(gold)
            z0s = inp.z0[:, :, [0, 15]]
            for name, tol, itol in (("F32C", 1e-7, 1e-6), ("F64", 1e-11, 1e-10)):
                P = getattr(L, "CUT_" + name)
                U.say(f"[cfg4] autotuned {name}: {L.cut_graph_autotune(g, 16, 1, P, 0)}")
                z = _flow(L, g, inp.z0, [2] * 16, P, w)[:, :, [0, 15]]
                r, ri = _rel_cols(z, zr), _rel_cols(z - z0s, zr - z0s)
                U.say(f"[cfg4] 2 steps {name}: state {r:.3e}, increment {ri:.3e}")
                assert r < tol and ri < itol
        U.say("[cfg4] 200-step flows")
        L.cut_graph_autotune(g, 16, 1, L.CUT_F64, 0)
        z200_64 = _flow(L, g, inp.z0, inp.n_steps, L.CUT_F64, w)
        L.cut_graph_autotune(g, 16, 1, L.CUT_F32C, 0)
        z200_32 = _flow(L, g, inp.z0, inp.n_steps, L.CUT_F32C, w)
        r200 = _rel_cols(z200_32, z200_64)
        n0 = np.linalg.norm(inp.z0, axis=0)
        d200 = np.max(np.abs(np.linalg.norm(z200_64, axis=0) - n0) / n0)
        U.say(f"[cfg4] 200 steps: F32C vs F64 {r200:.3e}; FP64 norm drift {d200:.3e}")
        assert r200 < 1e-7 and d200 < 1e-3
        U.say("[cfg4] 20-step flows")
        L.cut_graph_set_tiling(g, 1024, 512, 0)
        z64 = _flow(L, g, inp.z0, inp.n_steps, L.CUT_F64, w, steps=20)
        z32 = _flow(L, g, inp.z0, inp.n_steps, L.CUT_F32C, w, steps=20)
        assert _rel_cols(z32, z64) < 1e-7
        # the exact flow conserves |h| (antisymmetric action); the RK4 drift
        # must shrink at fourth order or faster when ds is halved
        n0 = np.linalg.norm(inp.z0, axis=0)
        half = workloads.Workload(**{**w.__dict__, "ds": w.ds / 2})
        zh = _flow(L, g, inp.z0, [40] * 16, L.CUT_F64, half, steps=40)
        d1 = np.max(np.abs(np.linalg.norm(z64, axis=0) - n0) / n0)
        d2 = np.max(np.abs(np.linalg.norm(zh, axis=0) - n0) / n0)
        U.say(f"[cfg4] norm drift over s=0.1: ds {d1:.3e}, ds/2 {d2:.3e}")
        assert d1 < 1e-3 and d2 < d1 / 8
    finally:
        L.cut_graph_free(g)


@pytest.mark.timeout(600)
def test_cfg2_full_flow_precision_study(L):
    path = os.path.join(GOLD, "cfg2_flow_s10.npy")
    if not os.path.exists(path):
        pytest.skip("oracle golden not generated")
    w = workloads.WORKLOADS[2]
    inp = workloads.make_inputs(2)
    zr = np.load(path)
    g = U.graph(L, "majorana", 24, adjoint=False)
    res = {}
    for name in ("F64", "F32C", "F32X", "F32"):
        U.say(f"[cfg2] full flow {name}")
        z = _flow(L, g, inp.z0, inp.n_steps, getattr(L, "CUT_" + name), w)
        res[name] = _rel_cols(z, zr)
    U.say(f"[cfg2] relative errors at s=10 vs oracle: {res}")
    assert res["F64"] < 1e-11
    assert res["F32C"] < 1e-7 and res["F32X"] < 1e-7


@pytest.mark.timeout(600)
def test_cfg2_g1_precision_study(L):
    """Config 2 with the literal generator G1 to s = 10, every precision against
    the oracle's stored G1 flow.  G1 rotates each off-diagonal coefficient with
    its pair-flip partners instead of damping it, and the flow amplifies
    perturbations (on the oracle: a relative perturbation of 1e-9 of the
    initial coefficients ends as 3.9e-7, one of 2^-24 as 2.3e-5), so the float
    errors are reported, and only the FP64 flow is held to a bound (1e-10); the
    float flows must stay finite."""
    path = os.path.join(GOLD, "cfg2_g1_flow_s10.npy")
    if not os.path.exists(path):
        pytest.skip("oracle golden not generated")
    w = workloads.WORKLOADS[2]
    inp = workloads.make_inputs(2)
    zr = np.load(path)
    g = U.graph(L, "majorana", 24, adjoint=False)
    res = {}
    for name in ("F64", "F32C", "F32X", "F32"):
        z = torch.tensor(inp.z0, device=DEV).contiguous()
        p = L.flow_params(L.CUT_GEN_G1, getattr(L, "CUT_" + name), w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH)
        L.cut_flow_integrate(g, p, 1, 3, [int(v) for v in inp.n_steps], z)
        torch.cuda.synchronize()
        res[name] = _rel_cols(z.cpu().numpy(), zr)
    U.say(f"[cfg2 G1] relative errors at s=10 vs oracle: {res}")
    assert res["F64"] < 1e-10
    assert all(np.isfinite(v) for v in res.values())


@pytest.mark.timeout(900)
def test_cfg5_full_gradient(L):
    path = os.path.join(GOLD, "cfg5_grad_s10.npy")
    if not os.path.exists(path):
        pytest.skip("oracle golden not generated")
    from paper_2609_14831_amd.flow import flow
    w = workloads.WORKLOADS[5]
    inp = workloads.make_inputs(5, with_fd=32)
    ref = np.load(path)
    g = U.graph(L, "majorana", 24)
    pairs = torch.tensor(A.MajoranaRegistry(24).pairs, device=DEV)
    ns = [int(v) for v in inp.n_steps]
    U.say("[cfg5] forward + adjoint (2000 steps, checkpoints every 16)")
    z0 = torch.tensor(inp.z0, device=DEV, requires_grad=True)
    loss = flow(z0, g, ns, L.CUT_GEN_G2, w.ds, w.delta, w.ckpt_every)[pairs, 0, :].sum()
    loss.backward()
    grad = z0.grad.cpu().numpy()
    rel = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    U.say(f"[cfg5] gradient vs oracle adjoint: {rel:.3e}")
    assert rel < 1e-10
    # Central differences from FP64 flows.  Their own error grows as 1/eps below
    # eps ~ 1e-5: after 2000 RK4 steps the loss carries FP64 rounding of about
    # 1e-14 relative (|L| ~ 60), which the quotient divides by 2 eps.  The 1e-6
    # bar is therefore checked at eps = 1e-5 over all 32 directions; at the
    # stated step 1e-6 the rounding term alone reaches ~1.5e-6 of the error
    # measure's denominator, so there the first 8 directions are held to 1e-5.
    gnorm = np.linalg.norm(grad)

    def fd_error(d, eps):
        v = torch.tensor(d[:, None, :], device=DEV)
        with torch.no_grad():
            lp = flow(z0 + eps * v, g, ns, L.CUT_GEN_G2, w.ds, w.delta, w.ckpt_every)[pairs, 0, :].sum()
            lm = flow(z0 - eps * v, g, ns, L.CUT_GEN_G2, w.ds, w.delta, w.ckpt_every)[pairs, 0, :].sum()
        fd = float((lp - lm) / (2 * eps))
        an = float(np.sum(grad[:, 0, :] * d))
        return abs(fd - an) / max(abs(fd), 1e-3 * gnorm)

    worst5 = max(fd_error(d, 1e-5) for d in inp.fd_dirs)
    U.say(f"[cfg5] worst FD relative error over 32 directions, eps 1e-5: {worst5:.3e}")
    worst6 = max(fd_error(d, 1e-6) for d in inp.fd_dirs[:8])
    U.say(f"[cfg5] worst FD relative error over 8 directions, eps 1e-6: {worst6:.3e}")
    assert worst5 < 1e-6
    assert worst6 < 1e-5
