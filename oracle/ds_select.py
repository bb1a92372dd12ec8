"""Spectral radius of the initial coflow map, used to fix the RK4 step.

Test infrastructure (see the package docstring).  For a workload's initial
coefficients h0 (per set) the coflow is locally x -> L(eta(h0)) x.  For Majorana
strings L is antisymmetric (orthonormal basis, real generator), so its spectral
radius equals its 2-norm, estimated by power iteration on -L^2 = L^T L.  The
step rule: ds = 5e-3 unless ds * rho > 0.5; then 0.5/rho rounded down to 1, 2 or
5 x 10^k.

Usage: python -m oracle.ds_select CFG [NSETS_SAMPLE]
"""
from __future__ import annotations

import math
import sys
import time

import numpy as np

import workloads
from . import algebra as A
from . import gen as GEN
from . import native


def spectral_radius(g, eta: np.ndarray, iters: int = 60, seed: int = 0) -> np.ndarray:
    """Per-set 2-norm of x -> apply(eta, x) (power iteration on L^T L = -L^2)."""
    eng = native.Engine(g, "g2", 0.5)
    rng = np.random.default_rng(seed)
    ns = eta.shape[1]
    v = rng.normal(size=(g.N, 1, ns))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    lam = np.zeros(ns)
    for _ in range(iters):
        w = -eng.apply(eta, eng.apply(eta, v))
        lam = np.sqrt(np.sum(w * v, axis=0)[0])
        v = w / np.linalg.norm(w, axis=0, keepdims=True)
    return lam


def rule(rho: float, base: float = 5e-3) -> float:
    if base * rho <= 0.5:
        return base
    x = 0.5 / rho
    e = math.floor(math.log10(x))
    for mant in (5, 2, 1):
        if mant * 10 ** e <= x:
            return mant * 10 ** e
    return 10 ** (e - 1) * 5


def main(cfg: int, nsample: int = 0):
    w = workloads.WORKLOADS[cfg]
    t = time.time()
    g = native.majorana_graph(w.size)
    print(f"graph m={w.size}: E={g.E} ({time.time() - t:.1f} s)", flush=True)
    inp = workloads.make_inputs(cfg)
    h0 = inp.z0[:, 0, :]
    if nsample and nsample < h0.shape[1]:
        idx = np.linspace(0, h0.shape[1] - 1, nsample).astype(int)
        h0 = h0[:, idx]
    eta = GEN.G2(w.size, w.delta)(h0)
    rho = spectral_radius(g, eta)
    print("rho per set:", np.array2string(rho, precision=3))
    print(f"max rho = {rho.max():.4f}; ds = {rule(rho.max())} (configured {w.ds})")


if __name__ == "__main__":
    main(int(sys.argv[1]), int(sys.argv[2]) if len(sys.argv) > 2 else 0)
