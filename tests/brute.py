"""Dense brute-force references used to pin the oracle (tests only).

Nothing here is shared with the oracle or the GPU path: operators are built as
explicit matrices (Jordan-Wigner for Majorana modes, unit matrices for E_pq)
and commutators are taken by matrix multiplication.
"""
from __future__ import annotations

import itertools
from functools import reduce

import numpy as np

_I = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)


def jw_majoranas(m: int):
    """gamma_0..gamma_{m-1} on n = m/2 qubits (Jordan-Wigner)."""
    n = m // 2
    out = []
    for a in range(n):
        for P in (_X, _Y):
            facs = [_Z] * a + [P] + [_I] * (n - a - 1)
            out.append(reduce(np.kron, facs))
    return out


def dense_strings(m: int):
    """(subsets, Gamma_S matrices) for the registry 2-subsets then 4-subsets."""
    g = jw_majoranas(m)
    subs = list(itertools.combinations(range(m), 2)) + list(itertools.combinations(range(m), 4))
    mats = []
    for S in subs:
        d = len(S)
        M = reduce(np.matmul, [g[a] for a in S])
        mats.append((1j ** (d * (d - 1) // 2)) * M)
    return subs, np.array(mats)


def dense_strings_of_degree(m: int, d: int):
    """(subsets, Gamma_S matrices) for every d-subset, lexicographic."""
    g = jw_majoranas(m)
    subs = list(itertools.combinations(range(m), d))
    mats = [(1j ** (d * (d - 1) // 2)) * reduce(np.matmul, [g[a] for a in S]) for S in subs]
    return subs, np.array(mats)


def project(mats: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Coefficients Tr(Gamma_K M) / dim over the registry (orthonormal basis)."""
    dim = M.shape[-1]
    return np.einsum("kxy,...yx->...k", mats, M) / dim


def epq_matrix(n: int, p: int, q: int) -> np.ndarray:
    E = np.zeros((n, n))
    E[p, q] = 1.0
    return E


def rk4_dense(f, z0, ds, nsteps):
    z = z0.copy()
    for _ in range(nsteps):
        a = f(z)
        b = f(z + 0.5 * ds * a)
        c = f(z + 0.5 * ds * b)
        d = f(z + ds * c)
        z = z + ds * (a + 2 * b + 2 * c + d) / 6.0
    return z
