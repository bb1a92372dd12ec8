"""GPU parity of single graph actions through the C ABI against the oracle.

Bounds (written per element, with S = sum_e |c_e eta_i x_j| from the oracle):
* FP64 passes: |y - y_oracle| <= 2 gamma_n S, gamma_n = n 2^-53 / (1 - n 2^-53), n the
  longest segment (two recursive summations in different orders);
* float-operand passes against the oracle evaluated on the same float-rounded
  operands: CUT_F32X (exact products, FP64 sums) <= 2 gamma_n S; CUT_F32C
  (error-free products, two-sum: the compensated dot product of Ogita, Rump and
  Oishi) <= (gamma_n^2 + 2^-52) * S with gamma_n = n u / (1 - n u), u = 2^-24 and
  n the longest segment; CUT_F32 (plain float sums) <= n * 2^-24 * S;
* float-operand passes against the FP64-operand oracle: <= 2 * 2^-24 * S + the
  above (each product has two rounded float operands).
"""
import numpy as np
import pytest

import gpu_util as U
import workloads
from oracle import algebra as A
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


def _inputs(N, nsets, nops, seed):
    eta = workloads.random_dense((N, nsets), seed=seed, scale=0.5)
    x = workloads.random_dense((N, nops, nsets), seed=seed + 1)
    return eta, x


def _abs_sum(og, eta, x):
    ga = A.Graph(og.algebra, og.size, og.N, og.k, og.i, og.j, np.abs(og.c), og.diag, og.pairs,
                 og.gen_sign)
    return OGr.apply(ga, np.abs(eta), np.abs(x))


def _run_apply(L, g, prec, eta, x, nsets, nops, which=0, y0=None, flags=0):
    N = eta.shape[0]
    dt = torch.float64 if prec == L.CUT_F64 else torch.float32
    te = torch.tensor(eta, device=DEV).to(dt)
    tx = torch.tensor(x.reshape(N, nops * nsets), device=DEV).to(dt)
    y = torch.zeros((N, nops * nsets), dtype=torch.float64, device=DEV) if y0 is None else \
        torch.tensor(y0.reshape(N, nops * nsets), device=DEV)
    L.cut_graph_apply(g, which, prec, nsets, nops, te, tx, y, flags)
    torch.cuda.synchronize()
    return y.cpu().numpy().reshape(N, nops, nsets)


CASES = [("epq", 8, 1, 1), ("epq", 8, 4, 2), ("majorana", 8, 1, 1), ("majorana", 8, 3, 2),
         ("majorana", 12, 1, 3), ("majorana", 12, 8, 1), ("majorana", 12, 64, 5),
         ("majorana", 12, 100, 2), ("majorana", 16, 16, 1), ("majorana", 24, 1, 3), ("majorana", 24, 1, 1)]
PRECS = ["F64", "F32X", "F32C", "F32"]


# (long-target threshold, chunk length, CUT_TILE_* flags): default chunked form;
# 16-record chunks with XCD remap; shared-triple tiles; four-wavefront split (no
# chunks); shared-triple chunks of quartic targets (one or two triples a chunk,
# with and without XCD remap); quadratic-target blocks (alone, with remap, with
# triple chunks, with shared-triple tiles); B-chunks of 32, 16 and 8 sets
# (alone, with short chunks and XCD remap, with blocks)
TILINGS = [(1024, 512, 0), (16, 16, 1), (64, 64, 3), (64, 64, 4), (1024, 8, 9), (16, 32, 9), (1024, 128, 8),
           (1024, 512, 16), (1024, 512, 17), (1024, 16, 25), (1024, 512, 18), (64, 64, 19),
           (1024, 512, 32), (16, 16, 65), (64, 64, 96 | 16)]


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("alg,size,nsets,nops", CASES)
def test_apply_parity(L, alg, size, nsets, nops, prec, tiling):
    U.say(f"[apply] {alg} {size} nsets={nsets} nops={nops} {prec} tiling={tiling}")
    g = U.graph(L, alg, size)
    L.cut_graph_set_tiling(g, *tiling)
    og = oracle_graph(alg, size)
    eta, x = _inputs(og.N, nsets, nops, seed=size * 7 + nsets)
    P = getattr(L, "CUT_" + prec)
    y = _run_apply(L, g, P, eta, x, nsets, nops)
    S = _abs_sum(og, eta, x)
    seg = np.diff(og.offsets()).max()
    if prec == "F64":
        U.assert_within(y, OGr.apply(og, eta, x), U.sum_bound(seg) * S + 1e-300, "F64 vs oracle")
    else:
        ref32 = OGr.apply(og, U.f32(eta), U.f32(x))
        acc = {"F32X": U.sum_bound(seg), "F32C": U.dot2_bound(seg), "F32": seg * U.U32}[prec]
        U.assert_within(y, ref32, acc * S + 1e-300, f"{prec} vs oracle on float operands")
        U.assert_within(y, OGr.apply(og, eta, x), (2 * U.U32 + acc) * S + 1e-300, f"{prec} vs FP64 oracle")
    L.cut_graph_set_tiling(g, 1024, 512, 0)


def test_apply_accumulate_and_gen_records(L):
    g = U.graph(L, "majorana", 12)
    og = oracle_graph("majorana", 12)
    eta, x = _inputs(og.N, 4, 2, seed=3)
    y0 = workloads.random_dense((og.N, 2, 4), seed=4)
    y = _run_apply(L, g, L.CUT_F64, eta, x, 4, 2, y0=y0, flags=L.CUT_ACCUMULATE)
    S = _abs_sum(og, eta, x) + np.abs(y0)
    U.assert_within(y, y0 + OGr.apply(og, eta, x), U.sum_bound(np.diff(og.offsets()).max() + 1) * S, "accumulate")
    ge = og.eta_records()
    y = _run_apply(L, g, L.CUT_F64, eta, x, 4, 2, which=1)
    U.assert_within(y, OGr.apply(ge, eta, x), U.sum_bound(og.N) * _abs_sum(ge, eta, x) + 1e-300, "E_eta records")


def test_apply_bitwise_deterministic(L):
    g = U.graph(L, "majorana", 16)
    og = oracle_graph("majorana", 16)
    eta, x = _inputs(og.N, 16, 3, seed=9)
    for tiling in ((32, 32, 1), (1024, 16, 9), (1024, 512, 17), (1024, 512, 19)):
        L.cut_graph_set_tiling(g, *tiling)
        for P in (L.CUT_F64, L.CUT_F32C):
            a = _run_apply(L, g, P, eta, x, 16, 3)
            b = _run_apply(L, g, P, eta, x, 16, 3)
            assert np.array_equal(a, b)
    L.cut_graph_set_tiling(g, 1024, 512, 0)


@pytest.mark.parametrize("prec", ["F64", "F32X", "F32C"])
@pytest.mark.parametrize("alg,size,nsets,nops", [("epq", 6, 2, 2), ("majorana", 10, 1, 1),
                                                 ("majorana", 12, 5, 3), ("majorana", 12, 64, 2)])
def test_adjoint_parity(L, alg, size, nsets, nops, prec):
    U.say(f"[adjoint] {alg} {size} nsets={nsets} nops={nops} {prec}")
    g = U.graph(L, alg, size)
    og = oracle_graph(alg, size)
    N = og.N
    eta, x = _inputs(N, nsets, nops, seed=31)
    w = workloads.random_dense((N, nops, nsets), seed=33)
    P = getattr(L, "CUT_" + prec)
    dt = torch.float64 if P == L.CUT_F64 else torch.float32
    te = torch.tensor(eta, device=DEV).to(dt)
    tx = torch.tensor(x.reshape(N, -1), device=DEV).to(dt)
    tw = torch.tensor(w.reshape(N, -1), device=DEV).to(dt)
    gx = torch.zeros((N, nops * nsets), dtype=torch.float64, device=DEV)
    geta = torch.zeros((N, nsets), dtype=torch.float64, device=DEV)
    L.cut_graph_apply_adjoint(g, 0, P, nsets, nops, te, tx, tw, gx, geta)
    torch.cuda.synchronize()
    if P != L.CUT_F64:
        eta, x, w = U.f32(eta), U.f32(x), U.f32(w)
    nmax = max(np.bincount(og.j).max(), np.bincount(og.i).max()) * nops
    tol = U.sum_bound(nmax) if prec in ("F64", "F32X") else U.dot2_bound(nmax, U.F32C_GROUP * nops)
    ga = A.Graph(og.algebra, og.size, N, og.k, og.i, og.j, np.abs(og.c), og.diag, og.pairs, 1.0)
    U.assert_within(gx.cpu().numpy().reshape(N, nops, nsets), OGr.adjoint_x(og, eta, w),
                    tol * OGr.adjoint_x(ga, np.abs(eta), np.abs(w)) + 1e-300, "g_x")
    U.assert_within(geta.cpu().numpy(), OGr.adjoint_eta(og, w, x),
                    tol * OGr.adjoint_eta(ga, np.abs(w), np.abs(x)) + 1e-300, "g_eta")


@pytest.mark.parametrize("alg,size,kind", [("epq", 8, "wegner_graph"), ("majorana", 10, "wegner_graph"),
                                           ("majorana", 10, "g2"), ("majorana", 16, "g2"),
                                           ("majorana", 10, "g1"), ("majorana", 16, "g1")])
def test_generator_and_vjp_parity(L, alg, size, kind):
    U.say(f"[generator] {alg} {size} {kind}")
    g = U.graph(L, alg, size)
    og = oracle_graph(alg, size)
    N = og.N
    nsets = 5
    if alg == "epq":
        h = workloads.random_dense((size, size, nsets), seed=5)
        h = (h + h.transpose(1, 0, 2)).reshape(N, nsets)
    else:
        h = workloads.small_majorana(size, nsets, 1, seed=5)[:, 0, :]
    gen, vjp = OG.make_generator(og, kind, 0.5)
    K = {"g2": L.CUT_GEN_G2, "g1": L.CUT_GEN_G1}.get(kind, L.CUT_GEN_WEGNER_GRAPH)
    th = torch.tensor(h, device=DEV)
    te = torch.zeros((N, nsets), dtype=torch.float64, device=DEV)
    L.cut_generator(g, K, 0.5, nsets, th, te)
    gb = workloads.random_dense((N, nsets), seed=6)
    tg = torch.zeros((N, nsets), dtype=torch.float64, device=DEV)
    L.cut_generator_vjp(g, K, 0.5, nsets, th, torch.tensor(gb, device=DEV), tg)
    torch.cuda.synchronize()
    ref = gen(h)
    np.testing.assert_allclose(te.cpu().numpy(), ref, rtol=1e-13, atol=1e-14 * np.abs(ref).max())
    rv = vjp(h, gb)
    np.testing.assert_allclose(tg.cpu().numpy(), rv, rtol=1e-12, atol=1e-13 * np.abs(rv).max())
