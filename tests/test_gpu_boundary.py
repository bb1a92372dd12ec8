"""Conventions of the C boundary on the GPU (calls through the C ABI).

* work areas: after cut_graph_reserve (and tuning) the computing entry points
  neither allocate nor move the work area, and give bitwise the same results
  call after call; a shape that was not reserved is refused before any launch;
* failure handling forced from the host: a non-finite coefficient in h0 makes
  the flow report CUT_E_NUMERIC (or set the caller's device flag without
  synchronising);
* resume: a flow stopped at step T/2 and resumed from its state with
  step_begin = T/2 is bitwise the uninterrupted flow (hipGraph and stream
  order);
* validated reload in a fresh process (Sec. 2.3 / Sec. 3.3: exact reload): a
  newly launched process that loads the same bundle gives bitwise the same
  action.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import gpu_util as U
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2609_14831_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def g24(L):
    """A private handle (no other test reserves on it)."""
    path = U.bundle_path(L, "majorana", 24)
    g = L.cut_graph_load(path, 0, L.CUT_LOAD_ADJOINT)
    yield g
    L.cut_graph_free(g)


def _inputs(m, nsets, nops, seed):
    z0 = workloads.small_majorana(m, nsets, nops, seed=seed)
    N = z0.shape[0]
    eta = workloads.random_dense((N, nsets), seed=seed + 1, scale=0.3)
    return z0, eta


def test_unreserved_shape_is_refused(L, g24):
    U.say("[boundary] unreserved shapes")
    nsets, nops = 8, 3
    z0, eta = _inputs(24, nsets, nops, 3)
    N = z0.shape[0]
    x = torch.tensor(z0.reshape(N, nops * nsets), device=DEV)
    y = torch.zeros_like(x)
    # the default tiling chunks the long quadratic targets: partial rows needed
    with pytest.raises(L.CutError) as e:
        L.cut_graph_apply(g24, 0, L.CUT_F64, nsets, nops, torch.tensor(eta, device=DEV), x, y, reserve=False)
    assert e.value.status == L.CUT_E_INVAL and "cut_graph_reserve" in str(e.value)
    z = torch.tensor(z0, device=DEV).contiguous()
    with pytest.raises(L.CutError) as e:
        L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3), nsets, nops, [3] * nsets, z,
                             reserve=False)
    assert e.value.status == L.CUT_E_INVAL
    torch.cuda.synchronize()
    np.testing.assert_array_equal(z.cpu().numpy(), z0)   # nothing ran
    with pytest.raises(L.CutError):
        L.cut_graph_reserve(g24, nsets, nops, 0, 0)
    with pytest.raises(L.CutError):
        L.cut_graph_reserve(g24, nsets, nops, 0, L.CUT_RESERVE_ADJOINT)


def test_tiling_flags_round_trip(L, g24):
    """Tiling flags: unknown bits are refused, every B-chunk field is
    accepted, and the tuner (which also tries B-chunks) returns known bits
    only."""
    U.say("[boundary] tiling flags")
    with pytest.raises(L.CutError) as e:
        L.cut_graph_set_tiling(g24, 1024, 512, 128)
    assert e.value.status == L.CUT_E_INVAL
    for b in (32, 16, 8):
        L.cut_graph_set_tiling(g24, 1024, 512, L.CUT_TILE_BCHUNK(b) | L.CUT_TILE_XCD_REMAP)
    t = L.cut_graph_autotune(g24, 16, 2, L.CUT_F32C, 0)
    assert t["tiling_flags"] & ~127 == 0
    L.cut_graph_set_tiling(g24, 1024, 512, 0)


def test_leading_dimension_beyond_32_bits_refused(L, g24):
    """The kernels multiply row indices by 32-bit strides: a leading dimension
    of 2^31 elements or more is refused on the host (before any launch, so the
    small buffers below are never read), through the raw C entry point."""
    U.say("[boundary] leading dimension limit")
    import ctypes as C
    nsets, nops = 1, 1
    L.cut_graph_reserve(g24, nsets, nops, 0, L.CUT_RESERVE_APPLY)
    eta = torch.zeros(16, dtype=torch.float64, device=DEV)
    x = torch.zeros(16, dtype=torch.float64, device=DEV)
    y = torch.zeros(16, dtype=torch.float64, device=DEV)
    st = L.lib().cut_graph_apply(g24, 0, L.CUT_F64, nsets, nops, C.c_void_p(eta.data_ptr()), 1 << 31,
                                 C.c_void_p(x.data_ptr()), 1, C.c_void_p(y.data_ptr()), 1, 0, None)
    torch.cuda.synchronize()
    assert st == L.CUT_E_INVAL and "2^31" in L.cut_last_error()


def test_work_area_fixed_after_reserve_and_tuning(L, g24):
    nsets, nops = 8, 3
    z0, eta = _inputs(24, nsets, nops, 5)
    N = z0.shape[0]
    L.cut_graph_reserve(g24, nsets, nops, 16, L.CUT_RESERVE_APPLY | L.CUT_RESERVE_FLOW | L.CUT_RESERVE_DERIV |
                        L.CUT_RESERVE_ADJOINT)
    U.say(f"[boundary] tuned {L.cut_graph_autotune(g24, nsets, nops, L.CUT_F32C, 1)}")
    before = L.cut_graph_reserved_bytes(g24)
    assert before > 0
    et = torch.tensor(eta, device=DEV)
    x = torch.tensor(z0.reshape(N, nops * nsets), device=DEV)
    ys = []
    for _ in range(3):
        for prec in (L.CUT_F64, L.CUT_F32C):
            dt = torch.float64 if prec == L.CUT_F64 else torch.float32
            y = torch.zeros_like(x)
            L.cut_graph_apply(g24, 0, prec, nsets, nops, et.to(dt), x.to(dt), y, reserve=False)
            ys.append(y.cpu().numpy())
    for k in range(2, len(ys)):
        np.testing.assert_array_equal(ys[k], ys[k % 2])
    zs = []
    for _ in range(2):
        z = torch.tensor(z0, device=DEV).contiguous()
        L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3), nsets, nops, [6] * nsets, z,
                             reserve=False)
        zs.append(z.cpu().numpy())
    np.testing.assert_array_equal(zs[0], zs[1])
    h = torch.tensor(z0[:, 0, :], device=DEV).contiguous()
    dy = torch.zeros_like(x)
    L.cut_graph_jvp(g24, L.CUT_GEN_G2, 0.5, L.CUT_F32C, nsets, nops, h, h, x, x, None, dy, reserve=False)
    gh = torch.zeros_like(h)
    L.cut_graph_vjp(g24, L.CUT_GEN_G2, 0.5, L.CUT_F64, nsets, nops, h, x, x, gh, None, reserve=False)
    torch.cuda.synchronize()
    assert L.cut_graph_reserved_bytes(g24) == before


def test_nonfinite_h0_reported(L, g24):
    nsets, nops = 4, 2
    z0, _ = _inputs(24, nsets, nops, 7)
    z0[100, 0, 2] = np.nan
    L.cut_graph_reserve(g24, nsets, nops, 0, L.CUT_RESERVE_FLOW)
    U.say("[boundary] NaN in h0, synchronous report")
    z = torch.tensor(z0, device=DEV).contiguous()
    with pytest.raises(L.CutError) as e:
        L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3), nsets, nops, [4] * nsets, z)
    assert e.value.status == L.CUT_E_NUMERIC
    U.say("[boundary] NaN in h0, device flag")
    flag = torch.full((1,), 7, dtype=torch.int32, device=DEV)
    z = torch.tensor(z0, device=DEV).contiguous()
    L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3, nonfinite=flag), nsets, nops,
                         [4] * nsets, z)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
    zf = z.cpu().numpy()
    # sets without the NaN flow on unharmed (sets are independent)
    assert np.all(np.isfinite(zf[:, :, [0, 1, 3]]))
    z0[100, 0, 2] = 0.5
    z = torch.tensor(z0, device=DEV).contiguous()
    L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3, nonfinite=flag), nsets, nops,
                         [4] * nsets, z)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0


@pytest.mark.parametrize("flags", [0, 1])
def test_resume_from_midpoint_is_bitwise(L, g24, flags):
    nsets, nops = 8, 3
    z0, _ = _inputs(24, nsets, nops, 9)
    ns = [40, 17, 33, 40, 8, 25, 40, 21]
    L.cut_graph_reserve(g24, nsets, nops, 0, L.CUT_RESERVE_FLOW)
    U.say(f"[boundary] resume, flags {flags}")
    full = torch.tensor(z0, device=DEV).contiguous()
    L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3, flags=flags), nsets, nops, ns, full)
    part = torch.tensor(z0, device=DEV).contiguous()
    L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3, flags=flags, step_end=20), nsets,
                         nops, ns, part)
    L.cut_flow_integrate(g24, L.flow_params(L.CUT_GEN_G2, L.CUT_F32C, 5e-3, flags=flags, step_begin=20),
                         nsets, nops, ns, part)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(part.cpu().numpy(), full.cpu().numpy())


_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2609_14831_amd import _lib as L
path, inp, out = sys.argv[2], sys.argv[3], sys.argv[4]
d = np.load(inp)
eta, x = d["eta"], d["x"]
g = L.cut_graph_load(path, 0, 0)
y = torch.zeros(x.shape, dtype=torch.float64, device="cuda:0")
L.cut_graph_apply(g, 0, L.CUT_F32C, eta.shape[1], x.shape[1] // eta.shape[1],
                  torch.tensor(eta, device="cuda:0"), torch.tensor(x, device="cuda:0"), y)
torch.cuda.synchronize()
np.save(out, y.cpu().numpy())
print(L.cut_graph_info(g)["checksum"])
L.cut_graph_free(g)
"""


def test_fresh_process_reload_is_bitwise(L, tmp_path):
    path = U.bundle_path(L, "majorana", 16)
    nsets, nops = 4, 2
    z0, eta = _inputs(16, nsets, nops, 11)
    N = z0.shape[0]
    eta32, x32 = eta.astype(np.float32), z0.reshape(N, nops * nsets).astype(np.float32)
    np.savez(tmp_path / "in.npz", eta=eta32, x=x32)
    g = L.cut_graph_load(path, 0, 0)
    try:
        y = torch.zeros((N, nops * nsets), dtype=torch.float64, device=DEV)
        L.cut_graph_apply(g, 0, L.CUT_F32C, nsets, nops, torch.tensor(eta32, device=DEV),
                          torch.tensor(x32, device=DEV), y)
        torch.cuda.synchronize()
        mine = y.cpu().numpy()
        chk = L.cut_graph_info(g)["checksum"]
    finally:
        L.cut_graph_free(g)
    U.say("[boundary] fresh-process reload")
    r = subprocess.run([sys.executable, "-c", _CHILD, ROOT, path, str(tmp_path / "in.npz"),
                        str(tmp_path / "out.npy")], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert int(r.stdout.strip().splitlines()[-1]) == chk
    np.testing.assert_array_equal(np.load(tmp_path / "out.npy"), mine)
