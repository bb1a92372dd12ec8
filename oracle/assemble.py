"""Multi-operator assembly from a transformed operator library (FP64).

Test infrastructure (see the package docstring).

Sec. 2.4 (last paragraph) and Sec. 3.4: once a library of source operators has
been transformed, new operator combinations are formed from their transformed
coefficient vectors without another expansion or compilation.  The reading
taken here: an output is a linear combination of the sources with given
weights,
    Y[:, k] = sum_s W[s, k] X[:, s],
X the transformed library [N, S] (one coefficient vector per source), W the
weights [S, K].  Because the coflow is linear in the operand for a given
Hamiltonian trajectory (Eq. forward-coeff), Y equals the transform of the
combined source operators.
"""
from __future__ import annotations

import numpy as np


def assemble(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Y = X W (a library matrix product)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(W, dtype=np.float64)


def assemble_loops(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    """The definition written out (small cases only)."""
    N, S = X.shape
    K = W.shape[1]
    Y = np.zeros((N, K))
    for n in range(N):
        for k in range(K):
            acc = 0.0
            for s in range(S):
                acc += W[s, k] * X[n, s]
            Y[n, k] = acc
    return Y
