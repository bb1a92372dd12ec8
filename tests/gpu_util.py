"""Helpers for the GPU tests: graph build/load cache and error bounds."""
from __future__ import annotations

import os
import sys
import tempfile

import numpy as np

U32 = 2.0 ** -24   # unit roundoff of float32
U64 = 2.0 ** -53

_cache = {}
_tmp = tempfile.mkdtemp(prefix="cutgraph_tests_")


def sum_bound(n: int) -> float:
    """Bound (relative to sum |terms|) on the difference of two FP64 summations
    of the same n terms in different orders: 2 * gamma_n, gamma_n = n u/(1-n u)."""
    g = n * U64 / (1 - n * U64)
    return 2 * g


def gamma32(n: int) -> float:
    return n * U32 / (1 - n * U32)


# records whose terms the compensated float pass sums in one float partial
# (16 with 32-lane groups, 8 otherwise: the larger bounds both)
F32C_GROUP = 16


def dot2_bound(n: int, group: int = F32C_GROUP) -> float:
    """Relative (to sum |terms|) error bound of the compensated float pass over
    n terms: each group of at most `group` terms is summed in one float by FMAs
    (error gamma_group of the group's sum of |terms|; the adjoint pass into the
    generator sums F32C_GROUP records x nops operands per group), the group
    partials go through two-sum into (hi, lo) (the compensated sum of Ogita,
    Rump and Oishi: gamma_n^2), hi + lo is rounded to FP64 (2^-52)."""
    g = gamma32(n)
    return gamma32(group) + g * g + 2.0 ** -52


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def graph(L, alg: str, size: int, adjoint: bool = True):
    key = (alg, size, adjoint)
    if key not in _cache:
        path = os.path.join(_tmp, f"{alg}_{size}.cgb")
        if not os.path.exists(path):
            L.cut_graph_build(L.CUT_ALG_EPQ if alg == "epq" else L.CUT_ALG_MAJORANA, size, path)
        _cache[key] = L.cut_graph_load(path, 0, L.CUT_LOAD_ADJOINT if adjoint else 0)
    return _cache[key]


def outside_graph(L, m: int):
    """Majorana graph built with the outside-space records E_C."""
    key = ("majorana-outside", m)
    if key not in _cache:
        path = os.path.join(_tmp, f"majorana_out_{m}.cgb")
        if not os.path.exists(path):
            L.cut_graph_build(L.CUT_ALG_MAJORANA, m, path, 0, L.CUT_BUILD_OUTSIDE)
        _cache[key] = L.cut_graph_load(path, 0, 0)
    return _cache[key]


def bundle_path(L, alg: str, size: int) -> str:
    path = os.path.join(_tmp, f"{alg}_{size}.cgb")
    if not os.path.exists(path):
        L.cut_graph_build(L.CUT_ALG_EPQ if alg == "epq" else L.CUT_ALG_MAJORANA, size, path)
    return path


def f32(a: np.ndarray) -> np.ndarray:
    """FP32 rounding (round to nearest even) of an FP64 array, back in FP64."""
    return a.astype(np.float32).astype(np.float64)


def assert_within(got: np.ndarray, ref: np.ndarray, bound: np.ndarray, what: str) -> float:
    err = np.abs(got - ref)
    bad = err > bound
    if np.any(bad):
        idx = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {int(bad.sum())} elements beyond bound; first {tuple(idx)} "
                             f"got {got[tuple(idx)]!r} ref {ref[tuple(idx)]!r} bound {bound[tuple(idx)]!r}")
    scale = np.maximum(bound, 1e-300)
    return float(np.max(err / scale))
