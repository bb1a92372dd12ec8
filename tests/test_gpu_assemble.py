"""GPU parity of cut_assemble (multi-operator assembly, FP64 on the matrix
cores) against the oracle.

Bound per element: |Y - Y_ref| <= 2 gamma_S sum_s |X[n][s] W[s][k]| (two FP64
sums of the same S products in different orders; gamma_S = S u / (1 - S u),
u = 2^-53).  Selections (one weight +-1 per output) are exact.
"""
import numpy as np
import pytest

import gpu_util as U
import workloads
from oracle import assemble as AS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    return _lib


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


@pytest.mark.parametrize("N,S,K", [(1, 1, 1), (7, 5, 9), (64, 16, 64), (65, 17, 63), (300, 120, 1024),
                                   (10902, 120, 1024), (92170, 120, 130)])
def test_assemble_parity(L, N, S, K):
    U.say(f"[assemble] N={N} S={S} K={K}")
    X = workloads.random_dense((N, S), seed=N + S)
    W = workloads.random_dense((S, K), seed=K + 1)
    Y = torch.full((N, K), np.nan, dtype=torch.float64, device=DEV)
    L.cut_assemble(_t(X), _t(W), Y)
    torch.cuda.synchronize()
    ref = AS.assemble(X, W)
    bound = U.sum_bound(S) * (np.abs(X) @ np.abs(W)) + 1e-300
    U.assert_within(Y.cpu().numpy(), ref, bound, "assemble")


def test_assemble_strided_accumulate_and_selection(L):
    N, S, K = 200, 40, 70
    Xb = workloads.random_dense((N, S + 9), seed=1)
    Wb = workloads.random_dense((S, K + 3), seed=2)
    Yb = workloads.random_dense((N, K + 5), seed=3)
    tX, tW, tY = _t(Xb), _t(Wb), _t(Yb)
    L.cut_assemble(tX[:, :S], tW[:, :K], tY[:, :K], flags=L.CUT_ACCUMULATE)
    torch.cuda.synchronize()
    got = tY.cpu().numpy()
    ref = Yb[:, :K] + AS.assemble(Xb[:, :S], Wb[:, :K])
    bound = U.sum_bound(S + 1) * (np.abs(Xb[:, :S]) @ np.abs(Wb[:, :K]) + np.abs(Yb[:, :K]))
    U.assert_within(got[:, :K], ref, bound, "accumulate")
    np.testing.assert_array_equal(got[:, K:], Yb[:, K:])      # padding untouched
    # selections are exact
    Wsel = np.zeros((S, K))
    rng = np.random.default_rng(4)
    Wsel[rng.integers(0, S, K), np.arange(K)] = rng.choice([-1.0, 1.0], K)
    Y = torch.zeros((N, K), dtype=torch.float64, device=DEV)
    L.cut_assemble(_t(Xb[:, :S]), _t(Wsel), Y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Y.cpu().numpy(), Xb[:, :S] @ Wsel)


def test_assembly_commutes_with_the_gpu_flow(L):
    """m = 16, 24 source operators flowed with one Hamiltonian (every set holds
    the same H and one source), 10 FP64 RK4 steps; assembling the flowed sources
    with 40 weight vectors equals flowing the 40 assembled sources."""
    m, S, K, steps = 16, 24, 40, 10
    g = U.graph(L, "majorana", m)
    N = L.cut_graph_info(g)["n_ops"]
    h = workloads.small_majorana(m, 1, 1, seed=7)[:, 0, 0]
    X0 = workloads.random_dense((N, S), seed=8)
    W = workloads.random_dense((S, K), seed=9)

    def transform(ops):
        n = ops.shape[1]
        z = np.zeros((N, 2, n))
        z[:, 0, :] = h[:, None]
        z[:, 1, :] = ops
        tz = _t(z)
        p = L.flow_params(L.CUT_GEN_G2, L.CUT_F64, 0.01, 0.5, 0)
        L.cut_flow_integrate(g, p, n, 2, [steps] * n, tz)
        return tz[:, 1, :]

    XT = transform(X0)                          # [N, S] view, row stride 2 S
    Y = torch.zeros((N, K), dtype=torch.float64, device=DEV)
    L.cut_assemble(XT, _t(W), Y)
    direct = transform(X0 @ W)
    torch.cuda.synchronize()
    a, b = Y.cpu().numpy(), direct.cpu().numpy()
    assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(b))


def test_assemble_argument_errors(L):
    x = torch.zeros((4, 3), dtype=torch.float64, device=DEV)
    w = torch.zeros((3, 5), dtype=torch.float64, device=DEV)
    y = torch.zeros((4, 5), dtype=torch.float64, device=DEV)
    with pytest.raises(L.CutError, match="CUT_E_INVAL"):
        L.cut_assemble(x, w, y, flags=4)
    st = L.lib().cut_assemble(x.data_ptr(), 2, 4, 3, w.data_ptr(), 5, 5, y.data_ptr(), 5, 0, None)
    assert st == L.CUT_E_INVAL and "leading dimension" in L.cut_last_error()
