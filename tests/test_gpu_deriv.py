"""GPU parity of the derivative entry points through the C ABI against the oracle.

* cut_generator_jvp: element-wise against the oracle's product / quotient-rule
  JVP (relative 1e-12 of the largest element: FP64 arithmetic, different order);
* cut_graph_jvp / cut_graph_vjp: element-wise against oracle.deriv.  With
  S = the same sums over |terms| (oracle), per element:
    FP64 passes        |got - ref| <= 2 gamma_n S + 1e-12 max|ref|
    float passes       |got - ref| <= (2^-23 + pass bound) S + 1e-12 max|ref|
  (n the longest segment; the pass bounds are those of the single-action
  tests: 2 gamma_n for F32X, gamma_n^2 + 2^-52 for F32C; 2^-23 covers the two
  float-rounded factors of each product; the max|ref| term covers the FP64
  generator and its derivative, evaluated in a different order);
* the pairing <w, dF> = <g_h, dh> + <g_x, dx> of the GPU JVP and VJP (the
  forward-adjoint pairing defect), relative to the sizes of its three terms;
* the finite-difference scan of the GPU action against the GPU JVP.
"""
import numpy as np
import pytest

import gpu_util as U
import workloads
from oracle import algebra as A
from oracle import deriv as OD
from oracle import gen as OG
from oracle import graph as OGr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    return _lib


_og = {}


def oracle_graph(alg, size):
    if (alg, size) not in _og:
        _og[(alg, size)] = A.graph_for(alg, size)
    return _og[(alg, size)]


def _abs_graph(og):
    return A.Graph(og.algebra, og.size, og.N, og.k, og.i, og.j, np.abs(og.c), og.diag, og.pairs, 1.0)


def _hamiltonian(alg, size, N, nsets, seed):
    if alg == "epq":
        h = workloads.random_dense((size, size, nsets), seed=seed)
        return (h + h.transpose(1, 0, 2)).reshape(N, nsets)
    return workloads.small_majorana(size, nsets, 1, seed=seed)[:, 0, :]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _kind(L, kind):
    return {"g2": L.CUT_GEN_G2, "g1": L.CUT_GEN_G1}.get(kind, L.CUT_GEN_WEGNER_GRAPH)


GENS = [("epq", 8, "wegner_graph"), ("majorana", 10, "wegner_graph"), ("majorana", 10, "g2"),
        ("majorana", 16, "g2"), ("majorana", 10, "g1"), ("majorana", 16, "g1")]


@pytest.mark.parametrize("alg,size,kind", GENS)
def test_generator_jvp_parity(L, alg, size, kind):
    U.say(f"[generator jvp] {alg} {size} {kind}")
    g = U.graph(L, alg, size)
    og = oracle_graph(alg, size)
    N, nsets = og.N, 5
    h = _hamiltonian(alg, size, N, nsets, seed=21)
    dh = workloads.random_dense((N, nsets), seed=22)
    out = torch.zeros((N, nsets), dtype=torch.float64, device=DEV)
    L.cut_generator_jvp(g, _kind(L, kind), 0.5, nsets, _t(h), _t(dh), out)
    torch.cuda.synchronize()
    ref = OG.make_generator_jvp(og, kind, 0.5)(h, dh)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _pass_bound(L, prec, seg):
    if prec == L.CUT_F64:
        return U.sum_bound(seg)
    return 2 * U.U32 + (U.sum_bound(seg) if prec == L.CUT_F32X else U.dot2_bound(seg))


def _run_jvp(L, g, kind, prec, h, x, dh, dx, want_y=True):
    N, nops, nsets = x.shape
    cols = nops * nsets
    y = torch.full((N, cols), np.nan, dtype=torch.float64, device=DEV) if want_y else None
    dy = torch.full((N, cols), np.nan, dtype=torch.float64, device=DEV)
    L.cut_graph_jvp(g, _kind(L, kind), 0.5, prec, nsets, nops, _t(h),
                    None if dh is None else _t(dh), _t(x.reshape(N, cols)),
                    None if dx is None else _t(dx.reshape(N, cols)), y, dy)
    torch.cuda.synchronize()
    yy = None if y is None else y.cpu().numpy().reshape(N, nops, nsets)
    return yy, dy.cpu().numpy().reshape(N, nops, nsets)


JVP_CASES = [("majorana", 16, "g2", 8, 3), ("majorana", 12, "wegner_graph", 4, 2), ("epq", 8, "wegner_graph", 3, 2),
             ("majorana", 16, "g2", 40, 2)]


@pytest.mark.parametrize("alg,size,kind,nsets,nops", JVP_CASES)
@pytest.mark.parametrize("prec", ["F64", "F32C", "F32X"])
def test_graph_jvp_parity(L, alg, size, kind, nsets, nops, prec):
    U.say(f"[jvp] {alg} {size} {kind} sets {nsets} ops {nops} {prec}")
    P = getattr(L, "CUT_" + prec)
    g = U.graph(L, alg, size)
    og = oracle_graph(alg, size)
    ga = _abs_graph(og)
    N = og.N
    gen, _ = OG.make_generator(og, kind, 0.5)
    jvp = OG.make_generator_jvp(og, kind, 0.5)
    h = _hamiltonian(alg, size, N, nsets, seed=31)
    x = workloads.random_dense((N, nops, nsets), seed=32)
    x[:, 0, :] = h                       # operand 0 is the Hamiltonian, as in the flow
    dh = workloads.random_dense((N, nsets), seed=33)
    dx = workloads.random_dense((N, nops, nsets), seed=34)
    seg = int(np.diff(og.offsets()).max())
    eta, deta = gen(h), jvp(h, dh)
    zh, zx = np.zeros_like(h), np.zeros_like(x)
    tilings = [None] if alg == "epq" else [(1024, 512, 0), (16, 16, 1), (1024, 16, 25), (1024, 512, 19)]
    for tiling in tilings:
        if tiling is not None:
            L.cut_graph_set_tiling(g, *tiling)
        for a, b, tag in ((dh, dx, "both"), (dh, None, "dh"), (None, dx, "dx")):
            y, dy = _run_jvp(L, g, kind, P, h, x, a, b)
            ref = OD.action_jvp(og, gen, jvp, h, x, zh if a is None else a, zx if b is None else b)
            S = np.zeros_like(x)
            if a is not None:
                S += OGr.apply(ga, np.abs(deta), np.abs(x))
            if b is not None:
                S += OGr.apply(ga, np.abs(eta), np.abs(b))
            bound = _pass_bound(L, P, seg) * S + 1e-12 * np.abs(ref).max()
            U.assert_within(dy, ref, bound, f"dy {tag} tiling {tiling}")
            yref = OD.action(og, gen, h, x)
            Sy = OGr.apply(ga, np.abs(eta), np.abs(x))
            U.assert_within(y, yref, _pass_bound(L, P, seg) * Sy + 1e-12 * np.abs(yref).max(),
                            f"y {tag} tiling {tiling}")
    L.cut_graph_set_tiling(g, 1024, 512, 0)


VJP_CASES = [("majorana", 16, "g2", 8, 3), ("majorana", 12, "wegner_graph", 4, 2), ("epq", 8, "wegner_graph", 3, 2),
             ("majorana", 12, "g1", 4, 2)]


@pytest.mark.parametrize("alg,size,kind,nsets,nops", VJP_CASES)
@pytest.mark.parametrize("prec", ["F64", "F32C"])
def test_graph_vjp_parity(L, alg, size, kind, nsets, nops, prec):
    U.say(f"[vjp] {alg} {size} {kind} sets {nsets} ops {nops} {prec}")
    P = getattr(L, "CUT_" + prec)
    g = U.graph(L, alg, size)
    og = oracle_graph(alg, size)
    N = og.N
    cols = nops * nsets
    gen, vjp = OG.make_generator(og, kind, 0.5)
    h = _hamiltonian(alg, size, N, nsets, seed=41)
    x = workloads.random_dense((N, nops, nsets), seed=42)
    w = workloads.random_dense((N, nops, nsets), seed=43)
    gh_ref, gx_ref = OD.action_vjp(og, gen, vjp, h, x, w)
    # per-element scales of the two outputs: the same sums over |terms|
    ga = _abs_graph(og)
    Sx = OGr.adjoint_x(ga, np.abs(gen(h)), np.abs(w))
    seg = int(max(np.bincount(og.j, minlength=N).max(), np.bincount(og.i, minlength=N).max()))
    tol_x = _pass_bound(L, P, seg)
    # g_h = eta'(h)^T geta, a fixed linear map (FP64) of geta, whose elements
    # carry the pass bound relative to their sums over |terms| (the adjoint pass
    # into the generator sums F32C_GROUP records x nops operands per float
    # partial).  Per element: |dg_h| <= |eta'(h)|^T (bound_geta), with the
    # entries of |eta'(h)| taken column by column from the oracle's generator
    # JVP, plus the FP64 rounding of the map itself on |eta'(h)|^T |geta|.
    seg_i = int(np.bincount(og.i, minlength=N).max())
    tol_g = U.sum_bound(seg_i) if P == L.CUT_F64 else 2 * U.U32 + U.dot2_bound(seg_i, U.F32C_GROUP * nops)
    v_geta = tol_g * OGr.adjoint_eta(ga, np.abs(w), np.abs(x))
    a_geta = np.abs(OGr.adjoint_eta(og, w, x))
    jvp = OG.make_generator_jvp(og, kind, 0.5)
    tol_h = np.zeros((N, nsets))
    for q in range(N):
        e = np.zeros((N, nsets))
        e[q] = 1.0
        col = np.abs(jvp(h, e))
        tol_h[q] = np.sum(col * v_geta, axis=0) + 64 * U.U64 * np.sum(col * a_geta, axis=0)
    tol_h += 1e-300
    th, tx, tw = _t(h), _t(x.reshape(N, cols)), _t(w.reshape(N, cols))
    gh = torch.full((N, nsets), np.nan, dtype=torch.float64, device=DEV)
    gx = torch.full((N, cols), np.nan, dtype=torch.float64, device=DEV)
    L.cut_graph_vjp(g, _kind(L, kind), 0.5, P, nsets, nops, th, tx, tw, gh, gx)
    torch.cuda.synchronize()
    U.assert_within(gx.cpu().numpy().reshape(N, nops, nsets), gx_ref, tol_x * Sx + 1e-12 * np.abs(gx_ref).max(), "g_x")
    U.assert_within(gh.cpu().numpy(), gh_ref, tol_h, "g_h")
    # accumulate, and each output alone
    gh0 = workloads.random_dense((N, nsets), seed=44)
    gx0 = workloads.random_dense((N, cols), seed=45)
    gh.copy_(_t(gh0))
    gx.copy_(_t(gx0))
    L.cut_graph_vjp(g, _kind(L, kind), 0.5, P, nsets, nops, th, tx, tw, gh, None, flags=L.CUT_ACCUMULATE)
    L.cut_graph_vjp(g, _kind(L, kind), 0.5, P, nsets, nops, th, None, tw, None, gx, flags=L.CUT_ACCUMULATE)
    torch.cuda.synchronize()
    U.assert_within(gh.cpu().numpy(), gh0 + gh_ref, tol_h + 1e-15 * np.abs(gh0 + gh_ref), "g_h accumulate")
    U.assert_within(gx.cpu().numpy().reshape(N, nops, nsets), gx0.reshape(N, nops, nsets) + gx_ref,
                    tol_x * Sx + 1e-12 * np.abs(gx_ref).max() + 1e-15 * np.abs(gx0.reshape(N, nops, nsets)),
                    "g_x accumulate")


@pytest.mark.parametrize("alg,size,kind", [("majorana", 24, "g2"), ("majorana", 12, "wegner_graph"),
                                           ("epq", 8, "wegner_graph")])
def test_pairing_defect(L, alg, size, kind):
    """<w, J (dh, dx)> against <J^T w, (dh, dx)> on the GPU, FP64 passes; the
    m = 24 case is the config-2 graph with 8 sets and H + 2 operands."""
    nsets, nops = 8, 3
    g = U.graph(L, alg, size)
    N = L.cut_graph_info(g)["n_ops"]
    h = _hamiltonian(alg, size, N, nsets, seed=51)
    x = workloads.random_dense((N, nops, nsets), seed=52)
    x[:, 0, :] = h
    dh = workloads.random_dense((N, nsets), seed=53)
    dx = workloads.random_dense((N, nops, nsets), seed=54)
    w = workloads.random_dense((N, nops, nsets), seed=55)
    _, dy = _run_jvp(L, g, kind, L.CUT_F64, h, x, dh, dx, want_y=False)
    gh = torch.zeros((N, nsets), dtype=torch.float64, device=DEV)
    gx = torch.zeros((N, nops * nsets), dtype=torch.float64, device=DEV)
    L.cut_graph_vjp(g, _kind(L, kind), 0.5, L.CUT_F64, nsets, nops, _t(h), _t(x.reshape(N, -1)),
                    _t(w.reshape(N, -1)), gh, gx)
    torch.cuda.synchronize()
    lhs = float(np.sum(w * dy))
    a = float(np.sum(gh.cpu().numpy() * dh))
    b = float(np.sum(gx.cpu().numpy().reshape(N, nops, nsets) * dx))
    defect = lhs - (a + b)
    scale = abs(lhs) + abs(a) + abs(b)
    U.say(f"[pairing] {alg} {size} {kind}: <w,Jv> = {lhs:.17e}, defect {defect:.3e}, "
          f"relative {abs(defect) / scale:.3e}")
    assert abs(defect) < 1e-13 * scale


@pytest.mark.parametrize("kind", ["wegner_graph", "g2"])
def test_fd_scan_config2(L, kind):
    """Centred differences of the GPU action (FP64; cut_generator then
    cut_graph_apply) against the GPU JVP on the config-2 graph (m = 24), 8 sets,
    H + 2 operands, along directions with N(0,1) entries.  The operand direction
    is linear, so only rounding remains (~ u S / eps).  With the Wegner block
    generator the action is quadratic in h and centred differences are exact up
    to rounding too; with G2 (a quotient) an eps^2 truncation term adds."""
    m, nsets, nops = 24, 8, 3
    K = _kind(L, kind)
    g = U.graph(L, "majorana", m)
    N = L.cut_graph_info(g)["n_ops"]
    h = workloads.small_majorana(m, nsets, 1, seed=61)[:, 0, :]
    x = workloads.random_dense((N, nops, nsets), seed=62)
    x[:, 0, :] = h
    dh = workloads.random_dense((N, nsets), seed=63)
    dx = workloads.random_dense((N, nops, nsets), seed=64)
    steps = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7]
    cols = nops * nsets

    def action(hh, xx):
        eta = torch.zeros((N, nsets), dtype=torch.float64, device=DEV)
        y = torch.zeros((N, cols), dtype=torch.float64, device=DEV)
        L.cut_generator(g, K, 0.5, nsets, _t(hh), eta)
        L.cut_graph_apply(g, 0, L.CUT_F64, nsets, nops, eta, _t(xx.reshape(N, cols)), y)
        torch.cuda.synchronize()
        return y.cpu().numpy().reshape(N, nops, nsets)

    res = {}
    for name, a, b in (("h", dh, None), ("x", None, dx)):
        _, exact = _run_jvp(L, g, kind, L.CUT_F64, h, x, a, b, want_y=False)
        errs = {}
        for eps in steps:
            hp, hm = (h + eps * a, h - eps * a) if a is not None else (h, h)
            xp, xm = (x + eps * b, x - eps * b) if b is not None else (x, x)
            fd = (action(hp, xp) - action(hm, xm)) / (2 * eps)
            errs[eps] = float(np.max(np.abs(fd - exact)) / np.max(np.abs(exact)))
        res[name] = errs
        U.say(f"[fd scan] {kind} {name}: " + ", ".join(f"{e:.0e}: {v:.3e}" for e, v in errs.items()))
    window = (1e-3, 1e-4, 1e-5)
    assert max(res["x"][e] for e in window) < 1e-9
    if kind == "wegner_graph":
        assert max(res["h"][e] for e in window) < 1e-9
    else:
        # second order while truncation dominates, and a small floor
        assert 30 < res["h"][1e-3] / res["h"][1e-4] < 300
        assert min(res["h"].values()) < 1e-8


def test_jvp_argument_errors(L):
    g = U.graph(L, "majorana", 10)
    N = L.cut_graph_info(g)["n_ops"]
    h = torch.zeros((N, 2), dtype=torch.float64, device=DEV)
    x = torch.zeros((N, 2), dtype=torch.float64, device=DEV)
    dy = torch.zeros((N, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(L.CutError, match="both tangents"):
        L.cut_graph_jvp(g, L.CUT_GEN_G2, 0.5, L.CUT_F64, 2, 1, h, None, x, None, None, dy)
    with pytest.raises(L.CutError, match="CUT_E_INVAL"):
        L.cut_graph_jvp(g, L.CUT_GEN_G2, 0.5, L.CUT_F64, 2, 1, h, h, None, None, None, dy)
    with pytest.raises(L.CutError, match="both outputs"):
        L.cut_graph_vjp(g, L.CUT_GEN_G2, 0.5, L.CUT_F64, 2, 1, h, x, x, None, None)
    ge = U.graph(L, "epq", 4)
    with pytest.raises(L.CutError, match="CUT_E_UNSUPPORTED"):
        L.cut_generator_jvp(ge, L.CUT_GEN_G2, 0.5, 1, h[:16, :1], h[:16, :1], dy[:16, :1])


def test_action_autograd_reverse_and_forward_mode(L):
    """paper_2609_14831_amd.flow.action: torch reverse mode (cut_graph_vjp) and
    forward mode (cut_graph_jvp) against the oracle's transpose and directional
    derivative, m = 12, G2, FP64."""
    from paper_2609_14831_amd.flow import action
    alg, size, kind, nsets, nops = "majorana", 12, "g2", 3, 2
    g = U.graph(L, alg, size)
    og = oracle_graph(alg, size)
    N = og.N
    gen, vjp = OG.make_generator(og, kind, 0.5)
    jvp = OG.make_generator_jvp(og, kind, 0.5)
    h = _hamiltonian(alg, size, N, nsets, seed=91)
    x = workloads.random_dense((N, nops, nsets), seed=92)
    w = workloads.random_dense((N, nops, nsets), seed=93)
    dh = workloads.random_dense((N, nsets), seed=94)
    dx = workloads.random_dense((N, nops, nsets), seed=95)
    th = _t(h).requires_grad_(True)
    tx = _t(x).requires_grad_(True)
    y = action(th, tx, g, L.CUT_GEN_G2, 0.5, L.CUT_F64)
    (y * _t(w)).sum().backward()
    gh_ref, gx_ref = OD.action_vjp(og, gen, vjp, h, x, w)
    np.testing.assert_allclose(th.grad.cpu().numpy(), gh_ref, rtol=1e-11, atol=1e-12 * np.abs(gh_ref).max())
    np.testing.assert_allclose(tx.grad.cpu().numpy(), gx_ref, rtol=1e-11, atol=1e-12 * np.abs(gx_ref).max())
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        y2 = action(fwAD.make_dual(_t(h), _t(dh)), fwAD.make_dual(_t(x), _t(dx)), g, L.CUT_GEN_G2, 0.5, L.CUT_F64)
        dy = fwAD.unpack_dual(y2).tangent
    ref = OD.action_jvp(og, gen, jvp, h, x, dh, dx)
    np.testing.assert_allclose(dy.cpu().numpy(), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(y.detach().cpu().numpy(), OD.action(og, gen, h, x), rtol=1e-11,
                               atol=1e-12 * np.abs(y.detach().cpu().numpy()).max())
