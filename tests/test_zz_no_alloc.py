"""The allocation-free forward action (cut_graph_apply_noalloc) against
cut_graph_apply, through the C ABI: two calls in a row, the second with a
smaller input, in the default chunked tiling and with quadratic-target blocks
(both keep partial rows in the fixed device scratch), bitwise equal; and a
shape whose partial rows exceed the scratch is refused before any launch."""
import ctypes as C

import numpy as np
import pytest

import gpu_util as U
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    f = _lib.lib().cut_graph_apply_noalloc
    f.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                  C.c_int64, C.c_void_p, C.c_int64, C.c_uint32, C.c_void_p]
    f.restype = C.c_int
    return _lib


def _noalloc(L, g, prec, nsets, nops, eta, x, y):
    st = L.lib().cut_graph_apply_noalloc(g, 0, prec, nsets, nops, eta.data_ptr(), eta.stride(0), x.data_ptr(),
                                         x.stride(0), y.data_ptr(), y.stride(0), 0,
                                         torch.cuda.current_stream().cuda_stream)
    return st


@pytest.mark.parametrize("tiling", [(1024, 512, 0), (1024, 256, 17)])
@pytest.mark.parametrize("prec", ["F64", "F32C"])
def test_noalloc_apply_matches_apply(L, tiling, prec):
    path = U.bundle_path(L, "majorana", 24)
    g = L.cut_graph_load(path, 0, 0)
    try:
        L.cut_graph_set_tiling(g, *tiling)
        P = getattr(L, "CUT_" + prec)
        dt = torch.float64 if P == L.CUT_F64 else torch.float32
        for nsets, nops, seed in ((8, 3, 1), (2, 2, 2)):
            U.say(f"[noalloc] {prec} tiling {tiling} nsets {nsets} nops {nops}")
            z0 = workloads.small_majorana(24, nsets, nops, seed=seed)
            N = z0.shape[0]
            eta = torch.tensor(workloads.random_dense((N, nsets), seed=seed + 5, scale=0.3), device=DEV).to(dt)
            x = torch.tensor(z0.reshape(N, nops * nsets), device=DEV).to(dt)
            y0 = torch.full((N, nops * nsets), np.nan, dtype=torch.float64, device=DEV)
            y1 = torch.full((N, nops * nsets), np.nan, dtype=torch.float64, device=DEV)
            st = _noalloc(L, g, P, nsets, nops, eta, x, y1)
            assert st == L.CUT_OK, L.cut_last_error()
            L.cut_graph_apply(g, 0, P, nsets, nops, eta, x, y0)
            torch.cuda.synchronize()
            a, b = y0.cpu().numpy(), y1.cpu().numpy()
            assert np.all(np.isfinite(a))
            np.testing.assert_array_equal(b, a)
    finally:
        L.cut_graph_free(g)


def test_noalloc_refuses_shape_beyond_scratch(L):
    path = U.bundle_path(L, "majorana", 24)
    g = L.cut_graph_load(path, 0, 0)
    try:
        L.cut_graph_set_tiling(g, 1024, 64, 0)     # many partial rows
        nsets, nops = 4096, 8                      # 32768 columns x 8 bytes per partial row
        eta = torch.zeros((1, 1), dtype=torch.float32, device=DEV)
        st = L.lib().cut_graph_apply_noalloc(g, 0, L.CUT_F32C, nsets, nops, eta.data_ptr(), nsets,
                                             eta.data_ptr(), nops * nsets, eta.data_ptr(), nops * nsets, 0, None)
        assert st == L.CUT_E_INVAL and "scratch" in L.cut_last_error()
    finally:
        L.cut_graph_free(g)
