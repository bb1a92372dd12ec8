"""ctypes binding of libcutgraph.so: argument marshalling only.

Every function has the name of the C entry point it calls (include/cutgraph.h)
and takes torch device tensors where the C function takes device pointers.
No arithmetic of the method happens here, and there is no fallback: if the
HIP library is missing, importing this module raises.

Work areas: the C computing entry points never allocate; a shape must be
reserved first (cut_graph_reserve).  For convenience the wrappers of those
entry points call cut_graph_reserve for their shape before the call (a no-op
once the shape is reserved) unless ``reserve=False`` is passed, which gives the
C behaviour unchanged (CUT_E_INVAL for a shape that was not reserved).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcutgraph.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libcutgraph.so not built at {LIB_PATH}; run `python -c 'import __graft_entry__ as g; g.build()'`")

# torch ships its own HIP and HSA runtimes; loading it first makes the library
# bind to those (same sonames) instead of bringing a second runtime into the
# process, which leaves one of the two without a device
import torch  # noqa: E402,F401

_L = C.CDLL(LIB_PATH)

# status codes / enums (mirror include/cutgraph.h)
CUT_OK, CUT_E_INVAL, CUT_E_IO, CUT_E_FORMAT, CUT_E_CHECKSUM = 0, 1, 2, 3, 4
CUT_E_NOMEM, CUT_E_DEVICE, CUT_E_NUMERIC, CUT_E_UNSUPPORTED = 5, 6, 7, 8
CUT_ALG_EPQ, CUT_ALG_MAJORANA, CUT_ALG_PAULI_BOSON = 1, 2, 3
CUT_GRAPH_FLOW, CUT_GRAPH_GEN, CUT_GRAPH_OUTSIDE = 0, 1, 2
CUT_BUILD_OUTSIDE = 1
CUT_F64, CUT_F32C, CUT_F32X, CUT_F32 = 0, 1, 2, 3
CUT_GEN_WEGNER_GRAPH, CUT_GEN_G2, CUT_GEN_G1 = 1, 2, 3
CUT_ACCUMULATE = 1
CUT_LOAD_ADJOINT, CUT_LOAD_NO_CHECKSUM = 1, 2
CUT_FLOW_HIPGRAPH = 1
CUT_FLOW_TIME_PASSES = 2
CUT_TILE_XCD_REMAP, CUT_TILE_TRIPLES, CUT_TILE_NO_CHUNKS, CUT_TILE_TRIPLE_CHUNKS = 1, 2, 4, 8
CUT_TILE_QUAD_BLOCKS = 16
CUT_TILE_BCHUNK_SHIFT = 5


def CUT_TILE_BCHUNK(b: int) -> int:
    """Tiling flag of the B-chunk b (32, 16 or 8 sets per lane group; 64: none)."""
    return {64: 0, 32: 1, 16: 2, 8: 3}[b] << CUT_TILE_BCHUNK_SHIFT


CUT_RESERVE_APPLY, CUT_RESERVE_FLOW, CUT_RESERVE_DERIV, CUT_RESERVE_ADJOINT = 1, 2, 4, 8

STATUS_NAMES = {0: "CUT_OK", 1: "CUT_E_INVAL", 2: "CUT_E_IO", 3: "CUT_E_FORMAT",
                4: "CUT_E_CHECKSUM", 5: "CUT_E_NOMEM", 6: "CUT_E_DEVICE", 7: "CUT_E_NUMERIC",
                8: "CUT_E_UNSUPPORTED"}

# symbols declared in include/cutgraph.h
EXPORTS = ["cut_graph_build", "cut_graph_load", "cut_graph_info", "cut_graph_free",
           "cut_graph_apply", "cut_graph_apply_noalloc", "cut_graph_apply_adjoint", "cut_generator", "cut_generator_vjp",
           "cut_generator_jvp", "cut_graph_jvp", "cut_graph_vjp", "cut_assemble", "cut_graph_labels",
           "cut_flow_integrate", "cut_flow_adjoint", "cut_graph_set_tiling", "cut_graph_autotune",
           "cut_flow_last_timing", "cut_graph_reserve", "cut_graph_reserved_bytes", "cut_last_error",
           "cut_version"]


class CutError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class cut_graph_desc(C.Structure):
    _fields_ = [("algebra", C.c_int32), ("size", C.c_int32), ("n_ops", C.c_int64),
                ("n_records", C.c_int64), ("n_gen_records", C.c_int64), ("n_pairs", C.c_int64),
                ("n_out_ops", C.c_int64), ("n_out_records", C.c_int64), ("n_gen_ops", C.c_int64), ("checksum", C.c_uint64), ("file_bytes", C.c_int64), ("build_seconds", C.c_double),
                ("identifier", C.c_char * 96)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["identifier"] = self.identifier.decode()
        return d


class cut_flow_params(C.Structure):
    _fields_ = [("generator", C.c_int32), ("precision", C.c_int32), ("ds", C.c_double),
                ("delta", C.c_double), ("ckpt_every", C.c_int32), ("flags", C.c_uint32),
                ("step_begin", C.c_int64), ("step_end", C.c_int64), ("outside_norm2", C.c_void_p),
                ("nonfinite", C.c_void_p)]


_vp, _i32, _i64, _u32, _dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
_L.cut_graph_build.argtypes = [_i32, _i32, C.c_char_p, _i32, _u32, C.POINTER(cut_graph_desc)]
_L.cut_graph_load.argtypes = [C.c_char_p, _i32, _u32, C.POINTER(_vp)]
_L.cut_graph_info.argtypes = [_vp, C.POINTER(cut_graph_desc)]
_L.cut_graph_free.argtypes = [_vp]
_L.cut_graph_free.restype = None
_L.cut_graph_apply.argtypes = [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _u32, _vp]
_L.cut_graph_apply_noalloc.argtypes = [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _u32, _vp]
_L.cut_graph_apply_adjoint.argtypes = [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                       _vp, _i64, _vp, _i64, _u32, _vp]
_L.cut_generator.argtypes = [_vp, _i32, _dbl, _i64, _vp, _i64, _vp, _i64, _vp]
_L.cut_generator_vjp.argtypes = [_vp, _i32, _dbl, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]
_L.cut_graph_labels.argtypes = [_vp, _i32, C.POINTER(C.c_uint64), _i64]
_L.cut_assemble.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _u32, _vp]
_L.cut_generator_jvp.argtypes = [_vp, _i32, _dbl, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]
_L.cut_graph_jvp.argtypes = [_vp, _i32, _dbl, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                             _vp, _i64, _vp, _i64, _vp]
_L.cut_graph_vjp.argtypes = [_vp, _i32, _dbl, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                             _vp, _i64, _u32, _vp]
_L.cut_flow_integrate.argtypes = [_vp, C.POINTER(cut_flow_params), _i64, _i64, C.POINTER(_i32), _vp, _vp,
                                  _vp]
_L.cut_flow_adjoint.argtypes = [_vp, C.POINTER(cut_flow_params), _i64, _i64, C.POINTER(_i32), _vp, _vp, _vp]
_L.cut_graph_set_tiling.argtypes = [_vp, _i64, _i64, _u32]
_L.cut_graph_reserve.argtypes = [_vp, _i64, _i64, _i64, _u32]
_L.cut_graph_reserved_bytes.argtypes = [_vp, C.POINTER(_i64)]


class cut_flow_timing(C.Structure):
    _fields_ = [("pass_ms", C.c_double), ("pass_launches", C.c_int64), ("gen_ms", C.c_double),
                ("gen_launches", C.c_int64)]


_L.cut_flow_last_timing.argtypes = [_vp, C.POINTER(cut_flow_timing)]


class cut_tuning(C.Structure):
    _fields_ = [("long_records", C.c_int64), ("chunk_records", C.c_int64), ("tiling_flags", C.c_uint32),
                ("precision", C.c_int32),
                ("pass_ms", C.c_double), ("default_ms", C.c_double)]


_L.cut_graph_autotune.argtypes = [_vp, _i64, _i64, _i32, _i32, C.POINTER(cut_tuning)]
_L.cut_last_error.restype = C.c_char_p
_L.cut_version.restype = C.c_char_p
for _name in EXPORTS:
    if _name not in ("cut_graph_free", "cut_last_error", "cut_version"):
        getattr(_L, _name).restype = C.c_int


def lib():
    return _L


def _check(st: int):
    if st != CUT_OK:
        raise CutError(st, _L.cut_last_error().decode(errors="replace"))


def cut_last_error() -> str:
    return _L.cut_last_error().decode(errors="replace")


def cut_version() -> str:
    return _L.cut_version().decode()


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _ld(t, default: int) -> int:
    if t is None:
        return default
    if t.dim() == 1:
        return default
    return t.stride(0)


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------- compile --
def cut_graph_build(algebra: int, size: int, path: str, threads: int = 0, flags: int = 0) -> dict:
    """flags: CUT_BUILD_OUTSIDE to include the outside-space records."""
    d = cut_graph_desc()
    _check(_L.cut_graph_build(algebra, size, path.encode(), threads, flags, C.byref(d)))
    return d.as_dict()


# ------------------------------------------------------------------- load --
def cut_graph_load(path: str, device: int = 0, flags: int = 0) -> int:
    h = _vp()
    _check(_L.cut_graph_load(path.encode(), device, flags, C.byref(h)))
    return h.value


def cut_graph_info(g: int) -> dict:
    d = cut_graph_desc()
    _check(_L.cut_graph_info(g, C.byref(d)))
    return d.as_dict()


def cut_graph_labels(g: int, which: int = 0):
    """Registry labels as a numpy uint64 array (which: CUT_GRAPH_FLOW / _GEN / _OUTSIDE)."""
    import numpy as np
    d = cut_graph_info(g)
    n = {0: d["n_ops"], 1: d["n_gen_ops"] or d["n_ops"], 2: d["n_out_ops"]}[which]
    out = np.zeros(n, dtype=np.uint64)
    _check(_L.cut_graph_labels(g, which, out.ctypes.data_as(C.POINTER(C.c_uint64)), n))
    return out


def cut_graph_free(g: int) -> None:
    _L.cut_graph_free(g)


def cut_graph_set_tiling(g: int, long_records: int, chunk_records: int, flags: int) -> None:
    """flags: CUT_TILE_XCD_REMAP | CUT_TILE_TRIPLES | CUT_TILE_NO_CHUNKS | CUT_TILE_TRIPLE_CHUNKS
    | CUT_TILE_QUAD_BLOCKS | CUT_TILE_BCHUNK(b)."""
    _check(_L.cut_graph_set_tiling(g, long_records, chunk_records, flags))


# ------------------------------------------------------------- work areas --
def cut_graph_reserve(g: int, nsets: int, nops: int, ckpt_every: int = 0, what: int = CUT_RESERVE_APPLY) -> None:
    """Sizes the handle's work areas for calls of this shape (CUT_RESERVE_* flags)."""
    _check(_L.cut_graph_reserve(g, nsets, nops, ckpt_every, what))


def cut_graph_reserved_bytes(g: int) -> int:
    b = _i64()
    _check(_L.cut_graph_reserved_bytes(g, C.byref(b)))
    return b.value


# ------------------------------------------------------------------ apply --
def cut_graph_apply(g: int, which: int, precision: int, nsets: int, nops: int, eta, x, y,
                    flags: int = 0, stream=None, reserve: bool = True) -> None:
    """y[k, op*nsets+s] (=|+=) sum_e c eta[i, s] x[j, op*nsets+s]; 2-D row-major tensors."""
    if reserve:
        cut_graph_reserve(g, nsets, nops, 0, CUT_RESERVE_APPLY)
    _check(_L.cut_graph_apply(g, which, precision, nsets, nops, _ptr(eta), _ld(eta, nsets), _ptr(x),
                              _ld(x, nops * nsets), _ptr(y), _ld(y, nops * nsets), flags,
                              _stream(stream)))


def cut_graph_apply_noalloc(g: int, which: int, precision: int, nsets: int, nops: int, eta, x, y,
                            flags: int = 0, stream=None) -> None:
    """cut_graph_apply with its partial rows in the library's fixed device array
    (no reservation, nothing allocated)."""
    _check(_L.cut_graph_apply_noalloc(g, which, precision, nsets, nops, _ptr(eta), _ld(eta, nsets), _ptr(x),
                                      _ld(x, nops * nsets), _ptr(y), _ld(y, nops * nsets), flags,
                                      _stream(stream)))


def cut_graph_apply_adjoint(g: int, which: int, precision: int, nsets: int, nops: int, eta, x, w,
                            g_x, g_eta, flags: int = 0, stream=None) -> None:
    _check(_L.cut_graph_apply_adjoint(
        g, which, precision, nsets, nops, _ptr(eta), _ld(eta, nsets), _ptr(x), _ld(x, nops * nsets),
        _ptr(w), _ld(w, nops * nsets), _ptr(g_x), _ld(g_x, nops * nsets), _ptr(g_eta),
        _ld(g_eta, nsets), flags, _stream(stream)))


def cut_generator(g: int, kind: int, delta: float, nsets: int, h, eta, stream=None) -> None:
    _check(_L.cut_generator(g, kind, delta, nsets, _ptr(h), _ld(h, nsets), _ptr(eta), _ld(eta, nsets),
                            _stream(stream)))


def cut_generator_vjp(g: int, kind: int, delta: float, nsets: int, h, gbar, g_h, stream=None,
                      reserve: bool = True) -> None:
    if reserve:
        cut_graph_reserve(g, nsets, 1, 0, CUT_RESERVE_APPLY)
    _check(_L.cut_generator_vjp(g, kind, delta, nsets, _ptr(h), _ld(h, nsets), _ptr(gbar),
                                _ld(gbar, nsets), _ptr(g_h), _ld(g_h, nsets), _stream(stream)))


# ------------------------------------------------------------ derivatives --
def cut_generator_jvp(g: int, kind: int, delta: float, nsets: int, h, dh, deta, stream=None) -> None:
    _check(_L.cut_generator_jvp(g, kind, delta, nsets, _ptr(h), _ld(h, nsets), _ptr(dh), _ld(dh, nsets),
                                _ptr(deta), _ld(deta, nsets), _stream(stream)))


def cut_graph_jvp(g: int, kind: int, delta: float, precision: int, nsets: int, nops: int, h, dh, x, dx,
                  y, dy, stream=None, reserve: bool = True) -> None:
    """dy = apply(eta'(h) dh, x) + apply(eta(h), dx); y = apply(eta(h), x) when given.
    dh, dx, x and y may be None as the C function allows."""
    if reserve:
        cut_graph_reserve(g, nsets, nops, 0, CUT_RESERVE_DERIV)
    cols = nops * nsets
    _check(_L.cut_graph_jvp(g, kind, delta, precision, nsets, nops, _ptr(h), _ld(h, nsets), _ptr(dh),
                            _ld(dh, nsets), _ptr(x), _ld(x, cols), _ptr(dx), _ld(dx, cols), _ptr(y),
                            _ld(y, cols), _ptr(dy), _ld(dy, cols), _stream(stream)))


def cut_graph_vjp(g: int, kind: int, delta: float, precision: int, nsets: int, nops: int, h, x, w,
                  g_h, g_x, flags: int = 0, stream=None, reserve: bool = True) -> None:
    """g_x (=|+=) L(eta(h))^T w; g_h (=|+=) eta'(h)^T geta(w, x); either output may be None."""
    if reserve:
        cut_graph_reserve(g, nsets, nops, 0, CUT_RESERVE_DERIV)
    cols = nops * nsets
    _check(_L.cut_graph_vjp(g, kind, delta, precision, nsets, nops, _ptr(h), _ld(h, nsets), _ptr(x),
                            _ld(x, cols), _ptr(w), _ld(w, cols), _ptr(g_h), _ld(g_h, nsets), _ptr(g_x),
                            _ld(g_x, cols), flags, _stream(stream)))


# --------------------------------------------------------------- assembly --
def cut_assemble(X, W, Y, flags: int = 0, stream=None) -> None:
    """Y (=|+=) X @ W for 2-D float64 device tensors X [N, S], W [S, K], Y [N, K]."""
    N, S = X.shape
    K = W.shape[1]
    _check(_L.cut_assemble(_ptr(X), _ld(X, S), N, S, _ptr(W), _ld(W, K), K, _ptr(Y), _ld(Y, K), flags,
                           _stream(stream)))


# ------------------------------------------------------------------- flow --
def flow_params(generator: int, precision: int, ds: float, delta: float = 0.5, ckpt_every: int = 0,
                flags: int = CUT_FLOW_HIPGRAPH, step_begin: int = 0, step_end: int = -1, outside_norm2=None,
                nonfinite=None):
    """outside_norm2: None, or a device float64 tensor of nops*nsets elements that
    the flow accumulates the outside-space diagnostic into.  nonfinite: None (the
    call synchronises and raises CUT_E_NUMERIC on a non-finite result) or a
    device int32 tensor the call sets to 1 on a non-finite result, without
    synchronising."""
    return cut_flow_params(generator, precision, ds, delta, ckpt_every, flags, step_begin, step_end,
                           _ptr(outside_norm2), _ptr(nonfinite))


def _steps_arg(n_steps):
    arr = (C.c_int32 * len(n_steps))(*[int(v) for v in n_steps])
    return arr


def cut_flow_integrate(g: int, params: cut_flow_params, nsets: int, nops: int, n_steps, z, ckpt=None,
                       stream=None, reserve: bool = True) -> None:
    """z: device float64 [N, nops, nsets] contiguous, advanced in place."""
    if reserve:
        cut_graph_reserve(g, nsets, nops, 0, CUT_RESERVE_FLOW)
    _check(_L.cut_flow_integrate(g, C.byref(params), nsets, nops, _steps_arg(n_steps), _ptr(z),
                                 _ptr(ckpt), _stream(stream)))


def cut_graph_autotune(g: int, nsets: int, nops: int, precision: int, allow_other_float: int = 1) -> dict:
    t = cut_tuning()
    _check(_L.cut_graph_autotune(g, nsets, nops, precision, allow_other_float, C.byref(t)))
    return {k: getattr(t, k) for k, _ in t._fields_}


def cut_flow_last_timing(g: int) -> dict:
    t = cut_flow_timing()
    _check(_L.cut_flow_last_timing(g, C.byref(t)))
    return {k: getattr(t, k) for k, _ in t._fields_}


def cut_flow_adjoint(g: int, params: cut_flow_params, nsets: int, nops: int, n_steps, ckpt, lam,
                     stream=None, reserve: bool = True) -> None:
    if reserve:
        cut_graph_reserve(g, nsets, nops, params.ckpt_every, CUT_RESERVE_ADJOINT)
    _check(_L.cut_flow_adjoint(g, C.byref(params), nsets, nops, _steps_arg(n_steps), _ptr(ckpt),
                               _ptr(lam), _stream(stream)))
