"""GPU parity of the outside-space action C_q (Eq. graph-actions, third line;
Eq. projected-flow) through cut_graph_apply(which = CUT_GRAPH_OUTSIDE) against
the oracle's brute-force records.

Bounds per element, S = sum_e |c_e eta_i x_j| over the target's 20 (m - 6)
records (oracle): FP64 and CUT_F32X 2 gamma_n S against the oracle on the same
operands; CUT_F32C (gamma_n^2 + 2^-52) S; float modes against the FP64-operand
oracle add 2 * 2^-24 S.
"""
import numpy as np
import pytest

import gpu_util as U
import workloads
from oracle import algebra as A
from oracle import graph as OGr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    return _lib


def _bound(L, P, seg):
    if P == L.CUT_F64:
        return U.sum_bound(seg)
    return 2 * U.U32 + (U.sum_bound(seg) if P == L.CUT_F32X else U.dot2_bound(seg))


def _apply_outside(L, g, P, eta, x, n_out):
    N, nops, nsets = x.shape
    dt = torch.float64 if P == L.CUT_F64 else torch.float32
    y = torch.full((n_out, nops * nsets), np.nan, dtype=torch.float64, device=DEV)
    L.cut_graph_apply(g, L.CUT_GRAPH_OUTSIDE, P, nsets, nops, torch.tensor(eta, device=DEV).to(dt),
                      torch.tensor(x.reshape(N, nops * nsets), device=DEV).to(dt), y)
    torch.cuda.synchronize()
    return y.cpu().numpy().reshape(n_out, nops, nsets)


@pytest.mark.parametrize("m,nsets,nops", [(8, 1, 1), (10, 3, 2), (12, 8, 3), (16, 64, 1), (16, 5, 4),
                                          (12, 40, 2)])
@pytest.mark.parametrize("prec", ["F64", "F32C", "F32X"])
def test_outside_action_parity(L, m, nsets, nops, prec):
    U.say(f"[outside] m={m} sets {nsets} ops {nops} {prec}")
    P = getattr(L, "CUT_" + prec)
    g = U.outside_graph(L, m)
    info = L.cut_graph_info(g)
    og = A.majorana_outside_graph(m)
    assert info["n_out_ops"] == og.n_out and info["n_out_records"] == og.E
    eta = workloads.random_dense((og.N, nsets), seed=m + 1, scale=0.5)
    x = workloads.random_dense((og.N, nops, nsets), seed=m + 2)
    got = _apply_outside(L, g, P, eta, x, og.n_out)
    ga = A.OutsideGraph(m, og.N, og.n_out, og.k, og.i, og.j, np.abs(og.c), og.masks)
    S = OGr.apply_outside(ga, np.abs(eta), np.abs(x))
    seg = 20 * (m - 6)
    U.assert_within(got, OGr.apply_outside(og, eta, x), _bound(L, P, seg) * S + 1e-300, f"C {prec}")
    if P != L.CUT_F64:
        ref32 = OGr.apply_outside(og, U.f32(eta), U.f32(x))
        tight = (U.sum_bound(seg) if P == L.CUT_F32X else U.dot2_bound(seg)) * S + 1e-300
        U.assert_within(got, ref32, tight, f"C {prec} on float operands")


@pytest.mark.parametrize("tiling", [(1024, 512, 0), (64, 64, 1), (16, 16, 5)])
def test_outside_action_config2_sampled(L, tiling):
    """The config-2 graph (m = 24) with its 48.45M outside-space records, 8 sets
    x 3 operands, on sampled outside targets, under several tilings (targets
    longer than the long-record threshold are split over a workgroup)."""
    m, nsets, nops = 24, 8, 3
    U.say(f"[outside] m=24 sampled tiling {tiling}")
    g = U.outside_graph(L, m)
    L.cut_graph_set_tiling(g, *tiling)
    n_out = L.cut_graph_info(g)["n_out_ops"]
    z = workloads.small_majorana(m, nsets, nops, seed=91)
    eta = workloads.random_dense((z.shape[0], nsets), seed=92, scale=0.5)
    rows = np.concatenate([[0, 1, n_out - 1], np.random.default_rng(93).integers(0, n_out, 29)])
    og = A.majorana_outside_graph(m, targets=rows)
    ga = A.OutsideGraph(m, og.N, og.n_out, og.k, og.i, og.j, np.abs(og.c), og.masks)
    ref = OGr.apply_outside(og, eta, z)[rows]
    S = OGr.apply_outside(ga, np.abs(eta), np.abs(z))[rows]
    for name in ("F64", "F32C", "F32X"):
        P = getattr(L, "CUT_" + name)
        got = _apply_outside(L, g, P, eta, z, n_out)[rows]
        U.assert_within(got, ref, _bound(L, P, 360) * S + 1e-300, f"m=24 C {name} tiling {tiling}")
    L.cut_graph_set_tiling(g, 1024, 512, 0)


def test_outside_errors(L):
    g = U.graph(L, "majorana", 10)
    N = L.cut_graph_info(g)["n_ops"]
    assert L.cut_graph_info(g)["n_out_ops"] == 0
    a = torch.zeros((N, 1), dtype=torch.float64, device=DEV)
    with pytest.raises(L.CutError, match="outside-space"):
        L.cut_graph_apply(g, L.CUT_GRAPH_OUTSIDE, L.CUT_F64, 1, 1, a, a, a)
    go = U.outside_graph(L, 10)
    with pytest.raises(L.CutError, match="adjoint"):
        L.cut_graph_apply_adjoint(go, L.CUT_GRAPH_OUTSIDE, L.CUT_F64, 1, 1, a, a, a, a, None)


def _flow_outside(L, g, z0, ns, prec, ds, outside, flags):
    N, nops, nsets = z0.shape
    z = torch.tensor(z0, device=DEV).contiguous()
    leak = torch.zeros(nops * nsets, dtype=torch.float64, device=DEV) if outside else None
    p = L.flow_params(L.CUT_GEN_G2, prec, ds, 0.5, 0, flags=flags, outside_norm2=leak)
    L.cut_flow_integrate(g, p, nsets, nops, [int(v) for v in ns], z)
    torch.cuda.synchronize()
    return z.cpu().numpy(), None if leak is None else leak.cpu().numpy().reshape(nops, nsets)


@pytest.mark.parametrize("prec,tol", [("F64", 1e-11), ("F32C", 1e-5), ("F32X", 1e-5)])
def test_flow_outside_diagnostic_vs_oracle(L, prec, tol):
    """The flow's outside-space diagnostic (RK4 quadrature of the integral of
    |C_X|^2) on m = 16 with ragged sets, against the oracle; the flowed state is
    bitwise the same with and without it, with and without the hipGraph."""
    from oracle import flow as OF
    from oracle import gen as OG
    m, ds = 16, 0.01
    U.say(f"[outside flow] m=16 {prec}")
    P = getattr(L, "CUT_" + prec)
    g = U.outside_graph(L, m)
    z0 = workloads.small_majorana(m, 3, 2, seed=95)
    ns = np.array([12, 5, 0], dtype=np.int32)
    og_l = A.majorana_graph(m)
    og = A.majorana_outside_graph(m)
    gen, _ = OG.make_generator(og_l, "g2", 0.5)
    zr, leak_r = OF.integrate_outside(og_l, gen, og, z0, ds, ns)
    for flags in (L.CUT_FLOW_HIPGRAPH, 0):
        z_off, _ = _flow_outside(L, g, z0, ns, P, ds, False, flags)
        z_on, leak = _flow_outside(L, g, z0, ns, P, ds, True, flags)
        np.testing.assert_array_equal(z_on, z_off)
        assert np.all(leak[:, 2] == 0.0)
        rel = np.abs(leak - leak_r) / np.maximum(np.abs(leak_r), 1e-300)
        U.say(f"[outside flow] {prec} flags {flags}: leak {leak[:, :2].ravel()}, max rel err {rel[:, :2].max():.3e}")
        assert np.all(rel[:, :2] < tol)
        if prec == "F64":
            assert np.abs(z_on - zr).max() < 1e-11 * np.abs(zr).max()


@pytest.mark.parametrize("prec,tol", [("F64", 1e-11), ("F32C", 1e-5)])
def test_flow_outside_diagnostic_scrambled_sets(L, prec, tol):
    """12 ragged sets in no particular order (the flow runs them sorted by step
    count and permutes the diagnostic's columns with them): the diagnostic per
    column against the oracle, and added to what the array held, column by
    column; the flowed state bitwise the same with and without it (the passes
    are cut into the same pieces), with and without the hipGraph; a set with
    zero steps untouched."""
    from oracle import flow as OF
    from oracle import gen as OG
    m, ds = 16, 0.01
    U.say(f"[outside flow] m=16 12 scrambled sets {prec}")
    P = getattr(L, "CUT_" + prec)
    g = U.outside_graph(L, m)
    nsets, nops = 12, 2
    z0 = workloads.small_majorana(m, nsets, nops, seed=97)
    ns = np.array([3, 9, 0, 6, 9, 4, 7, 1, 9, 2, 8, 5], dtype=np.int32)
    og_l = A.majorana_graph(m)
    og = A.majorana_outside_graph(m)
    gen, _ = OG.make_generator(og_l, "g2", 0.5)
    zr, leak_r = OF.integrate_outside(og_l, gen, og, z0, ds, ns)
    base = np.arange(1, nops * nsets + 1, dtype=np.float64).reshape(nops, nsets)
    for flags in (L.CUT_FLOW_HIPGRAPH, 0):
        z_off, _ = _flow_outside(L, g, z0, ns, P, ds, False, flags)
        z_on, leak = _flow_outside(L, g, z0, ns, P, ds, True, flags)
        np.testing.assert_array_equal(z_on, z_off)
        np.testing.assert_array_equal(z_on[:, :, 2], z0[:, :, 2])
        assert np.all(leak[:, 2] == 0.0)
        live = ns > 0
        rel = np.abs(leak - leak_r)[:, live] / np.maximum(np.abs(leak_r[:, live]), 1e-300)
        U.say(f"[outside flow] scrambled {prec} flags {flags}: max rel err {rel.max():.3e}")
        assert np.all(rel < tol)
        z = torch.tensor(z0, device=DEV).contiguous()
        acc = torch.tensor(base.ravel(), device=DEV)
        L.cut_flow_integrate(g, L.flow_params(L.CUT_GEN_G2, P, ds, 0.5, 0, flags=flags, outside_norm2=acc),
                             nsets, nops, [int(v) for v in ns], z)
        torch.cuda.synchronize()
        added = acc.cpu().numpy().reshape(nops, nsets) - base
        assert np.all(np.abs(added - leak) <= 1e-12 * base)
        if prec == "F64":
            assert np.abs(z_on - zr).max() < 1e-11 * np.abs(zr).max()


def test_flow_outside_config2_unchanged_trajectory(L):
    """Config-2 graph (m = 24, 48.45M outside-space records), 8 sets x 3
    operands, 20 steps, F32C: the trajectory is bitwise the same with the
    diagnostic on, and the hipGraph replay gives the same diagnostic as the
    stream-ordered path."""
    m, ds = 24, 5e-3
    U.say("[outside flow] m=24 20 steps")
    g = U.outside_graph(L, m)
    z0 = workloads.small_majorana(m, 8, 3, seed=96)
    ns = np.full(8, 20, dtype=np.int32)
    z_off, _ = _flow_outside(L, g, z0, ns, L.CUT_F32C, ds, False, L.CUT_FLOW_HIPGRAPH)
    z_on, leak = _flow_outside(L, g, z0, ns, L.CUT_F32C, ds, True, L.CUT_FLOW_HIPGRAPH)
    _, leak_s = _flow_outside(L, g, z0, ns, L.CUT_F32C, ds, True, 0)
    np.testing.assert_array_equal(z_on, z_off)
    np.testing.assert_array_equal(leak, leak_s)
    assert np.all(np.isfinite(leak)) and np.all(leak > 0)
