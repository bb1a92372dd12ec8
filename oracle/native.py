"""ctypes wrapper of the oracle's plain-C FP64 engine (``ref_engine.c``).

Test infrastructure (see the package docstring).  The engine receives the
oracle's own records and generator stencil, so it is a second, faster
evaluation of exactly the NumPy oracle's arithmetic; tests cross-check the two.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .algebra import Graph
from .gen import G2

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ref_engine.c")
LIB = os.path.join(_HERE, "libref_engine.so")

_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class _OrcGraph(C.Structure):
    _fields_ = [("N", C.c_int64), ("nops", C.c_int64), ("nsets", C.c_int64),
                ("off", _i64p), ("ri", _i32p), ("rj", _i32p), ("rc", _f64p),
                ("kind", C.c_int),
                ("st_off", _i64p), ("st_a", _i32p), ("st_p", _i32p), ("st_c", _f64p),
                ("pairs", _i32p), ("delta", C.c_double),
                ("eoff", _i64p), ("ei", _i32p), ("ej", _i32p), ("ec", _f64p),
                ("gsign", C.c_double)]


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB, SRC])
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB)
        for name in ("orc_apply", "orc_adj_x", "orc_adj_eta"):
            getattr(_lib, name).argtypes = [C.c_void_p, _f64p, _f64p, _f64p]
        _lib.orc_flow.argtypes = [C.c_void_p, _f64p, C.c_double, _i32p, C.c_int, _f64p]
        _lib.orc_flow_adjoint.argtypes = [C.c_void_p, _f64p, C.c_double, _i32p, C.c_int, _f64p]
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


class Engine:
    """Holds contiguous copies of one oracle graph (+ generator) for the C engine."""

    def __init__(self, g: Graph, generator: str, delta: float = 0.5, g2: G2 = None):
        self.g = g
        self.keep = []
        self.off = np.ascontiguousarray(g.offsets(), dtype=np.int64)
        self.ri = np.ascontiguousarray(g.i, dtype=np.int32)
        self.rj = np.ascontiguousarray(g.j, dtype=np.int32)
        self.rc = np.ascontiguousarray(g.c, dtype=np.float64)
        st = dict(off=np.zeros(g.N + 1, np.int64), a=np.zeros(1, np.int32),
                  p=np.zeros(1, np.int32), c=np.zeros(1), pairs=np.zeros(1, np.int32))
        eo = dict(off=np.zeros(g.N + 1, np.int64), i=np.zeros(1, np.int32),
                  j=np.zeros(1, np.int32), c=np.zeros(1))
        if generator == "g2":
            kind = 0
            gen = g2 if g2 is not None else G2(g.size, delta)
            S = np.concatenate([s[0] for s in gen.stencil])
            a = np.concatenate([np.full(s[0].size, q, np.int32) for q, s in enumerate(gen.stencil)])
            P = np.concatenate([s[1] for s in gen.stencil])
            cc = np.concatenate([s[2] for s in gen.stencil])
            order = np.lexsort((a, S))
            cnt = np.bincount(S, minlength=g.N)
            st = dict(off=np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64),
                      a=a[order].astype(np.int32), p=P[order].astype(np.int32),
                      c=cc[order].astype(np.float64),
                      pairs=gen.reg.pairs.astype(np.int32))
        elif generator == "wegner_graph":
            kind = 1
            ge = g.eta_records()
            eo = dict(off=ge.offsets().astype(np.int64), i=ge.i.astype(np.int32),
                      j=ge.j.astype(np.int32), c=ge.c.astype(np.float64))
        else:
            raise ValueError(generator)
        self.st, self.eo = st, eo
        self.kind, self.delta = kind, float(delta)

    def _struct(self, nops, nsets):
        s = _OrcGraph()
        s.N, s.nops, s.nsets = self.g.N, nops, nsets
        s.off, s.ri, s.rj, s.rc = (_p(self.off, _i64p), _p(self.ri, _i32p), _p(self.rj, _i32p),
                                   _p(self.rc, _f64p))
        s.kind = self.kind
        s.st_off, s.st_a, s.st_p, s.st_c = (_p(self.st["off"], _i64p), _p(self.st["a"], _i32p),
                                            _p(self.st["p"], _i32p), _p(self.st["c"], _f64p))
        s.pairs, s.delta = _p(self.st["pairs"], _i32p), self.delta
        s.eoff, s.ei, s.ej, s.ec = (_p(self.eo["off"], _i64p), _p(self.eo["i"], _i32p),
                                    _p(self.eo["j"], _i32p), _p(self.eo["c"], _f64p))
        s.gsign = self.g.gen_sign
        return s

    def apply(self, eta, x):
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        s = self._struct(x.shape[1], x.shape[2])
        lib().orc_apply(C.byref(s), _p(eta, _f64p), _p(x, _f64p), _p(y, _f64p))
        return y

    def adjoint_x(self, eta, w):
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = np.zeros_like(w)
        s = self._struct(w.shape[1], w.shape[2])
        lib().orc_adj_x(C.byref(s), _p(eta, _f64p), _p(w, _f64p), _p(out, _f64p))
        return out

    def adjoint_eta(self, w, x):
        w = np.ascontiguousarray(w, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros((w.shape[0], w.shape[2]))
        s = self._struct(w.shape[1], w.shape[2])
        lib().orc_adj_eta(C.byref(s), _p(w, _f64p), _p(x, _f64p), _p(out, _f64p))
        return out

    def flow(self, z0, ds, n_steps, ckpt_every=0):
        z = np.ascontiguousarray(z0, dtype=np.float64).copy()
        ns = np.ascontiguousarray(n_steps, dtype=np.int32)
        s = self._struct(z.shape[1], z.shape[2])
        T = int(ns.max()) if ns.size else 0
        ck = None
        if ckpt_every:
            ck = np.zeros(((T + ckpt_every - 1) // ckpt_every,) + z.shape)
        lib().orc_flow(C.byref(s), _p(z, _f64p), ds, _p(ns, _i32p), int(ckpt_every),
                       _p(ck, _f64p) if ck is not None else None)
        return z, ck

    def flow_adjoint(self, z0, ds, n_steps, lam_end, ckpt_every=16):
        z0 = np.ascontiguousarray(z0, dtype=np.float64)
        lam = np.ascontiguousarray(lam_end, dtype=np.float64).copy()
        ns = np.ascontiguousarray(n_steps, dtype=np.int32)
        s = self._struct(z0.shape[1], z0.shape[2])
        lib().orc_flow_adjoint(C.byref(s), _p(z0, _f64p), ds, _p(ns, _i32p), int(ckpt_every),
                               _p(lam, _f64p))
        return lam
