"""Seeded synthetic workloads for the compiled-CUT-graph hot path.

This module only draws random numbers and lays them out.  It holds none of the
method's arithmetic (no algebra, no records, no generator, no integrator), so
both the GPU library's tests/bench and the CPU oracle can take their inputs from
it without sharing any of the computation they are compared on.

Registry sizes are plain binomial counts: a Majorana registry over m modes holds
C(m,2) quadratic strings followed by C(m,4) quartic strings (canonical order: all
2-subsets, then all 4-subsets, each in lexicographic order); the one-body fermion
registry over n orbitals holds n*n operators E_pq at index p*n+q.

Coefficient state layout shared by every consumer: ``z[N, nops, nsets]`` float64,
row = registry index, op 0 = the Hamiltonian, ops 1.. = coflowed observables,
innermost = coefficient set.

Seed recipe (one stream per configuration): ``numpy.random.default_rng([260914831,
cfg])`` with the fixed draw order quadratic h, quartic h, observables, mass ratios
r_b, flow lengths s_max_b, finite-difference directions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 260914831


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic configuration (sizes, seeds, integration constants)."""

    cfg: int
    name: str
    algebra: str            # "epq" or "majorana"
    size: int               # n orbitals (epq) or m Majorana modes
    nsets: int
    nops: int               # 1 Hamiltonian + (nops-1) observables
    ds: float
    s_max: Optional[float]  # common flow length (None when drawn per set)
    generator: str          # "wegner_graph" or "g2"
    delta: float = 0.5
    fixed_steps: Optional[int] = None  # flows quoted in steps rather than s
    ckpt_every: int = 0

    @property
    def n_ops(self) -> int:
        if self.algebra == "epq":
            return self.size * self.size
        m = self.size
        return math.comb(m, 2) + math.comb(m, 4)

    @property
    def n_quad(self) -> int:
        return math.comb(self.size, 2) if self.algebra == "majorana" else 0

    @property
    def ncols(self) -> int:
        return self.nops * self.nsets


# ds for the Majorana configurations: 5e-3 unless ds*rho > 0.5 for the spectral
# radius rho of the linear map x -> [eta(h0), x] at the initial coefficients, in
# which case 0.5/rho rounded down to 1, 2 or 5 x 10^k.  The values below were
# fixed with the oracle's power iteration (oracle/ds_select.py prints rho).
WORKLOADS = {
    1: Workload(1, "epq_n8_wegner", "epq", 8, 1, 1, 1e-3, 10.0, "wegner_graph"),
    2: Workload(2, "majorana_m24_g2", "majorana", 24, 1, 3, 5e-3, 10.0, "g2"),
    3: Workload(3, "majorana_m40_batched", "majorana", 40, 64, 5, 5e-3, None, "g2"),
    4: Workload(4, "majorana_m64_stress", "majorana", 64, 16, 1, 5e-3, None, "g2",
                fixed_steps=200),
    5: Workload(5, "majorana_m24_adjoint", "majorana", 24, 8, 1, 5e-3, 10.0, "g2",
                ckpt_every=16),
}


def rng_for(cfg: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, cfg])


@dataclasses.dataclass
class Inputs:
    z0: np.ndarray                   # [N, nops, nsets] float64
    n_steps: np.ndarray              # [nsets] int32, whole RK4 steps per set
    r: Optional[np.ndarray] = None   # mass ratios (config 3)
    s_max: Optional[np.ndarray] = None
    fd_dirs: Optional[np.ndarray] = None  # [ndir, N, nsets] unit directions


def _steps(s: float, ds: float) -> int:
    return int(round(s / ds))


def make_epq(w: Workload, rng: np.random.Generator) -> Inputs:
    n = w.size
    iu = np.triu_indices(n, 1)
    off = rng.normal(0.0, 1.0, size=len(iu[0]))   # upper triangle, row-major
    dnoise = rng.normal(0.0, 0.1, size=n)
    h = np.zeros((n, n))
    h[iu] = off
    h = h + h.T
    h[np.arange(n), np.arange(n)] = np.arange(n) + dnoise
    z0 = h.reshape(n * n, 1, 1).copy()
    ns = np.array([_steps(w.s_max, w.ds)], dtype=np.int32)
    return Inputs(z0=z0, n_steps=ns)


def make_majorana(w: Workload, rng: np.random.Generator, with_fd: int = 0) -> Inputs:
    N, nq = w.n_ops, w.n_quad
    nquart = N - nq
    z0 = np.zeros((N, w.nops, w.nsets))
    quart_sd = 0.05 if w.cfg == 4 else 0.1
    r = smax = None
    if w.cfg == 3:
        # one base Hamiltonian shared by every set, rescaled per set below
        hq = rng.normal(0.0, 1.0, size=nq)
        h4 = rng.normal(0.0, quart_sd, size=nquart)
        z0[:nq, 0, :] = hq[:, None]
        z0[nq:, 0, :] = h4[:, None]
    else:
        hq = rng.normal(0.0, 1.0, size=(w.nsets, nq))
        h4 = rng.normal(0.0, quart_sd, size=(w.nsets, nquart))
        z0[:nq, 0, :] = hq.T
        z0[nq:, 0, :] = h4.T
    if w.nops > 1:
        # random quadratic observables, independent per set and per observable
        ob = rng.normal(0.0, 1.0, size=(w.nsets, w.nops - 1, nq))
        z0[:nq, 1:, :] = ob.transpose(2, 1, 0)
    if w.cfg == 3:
        # mass-scaling sweep: r_b = m/m0 ~ U[1,2]; quadratic coefficients scale
        # with (m0/m)^(1/2)
        r = rng.uniform(1.0, 2.0, size=w.nsets)
        z0[:nq, 0, :] *= r[None, :] ** -0.5
        smax = rng.uniform(2.0, 20.0, size=w.nsets)
        ns = np.array([_steps(s, w.ds) for s in smax], dtype=np.int32)
    elif w.fixed_steps is not None:
        ns = np.full(w.nsets, w.fixed_steps, dtype=np.int32)
    else:
        ns = np.full(w.nsets, _steps(w.s_max, w.ds), dtype=np.int32)
    fd = None
    if with_fd:
        v = rng.normal(0.0, 1.0, size=(with_fd, N, w.nsets))
        v /= np.linalg.norm(v.reshape(with_fd, -1), axis=1)[:, None, None]
        fd = v
    return Inputs(z0=z0, n_steps=ns, r=r, s_max=smax, fd_dirs=fd)


def make_inputs(cfg: int, with_fd: int = 0) -> Inputs:
    w = WORKLOADS[cfg]
    rng = rng_for(cfg)
    if w.algebra == "epq":
        return make_epq(w, rng)
    return make_majorana(w, rng, with_fd=with_fd)


def small_majorana(m: int, nsets: int, nops: int, seed: int, quart_sd: float = 0.1,
                   obs_quartic: bool = False) -> np.ndarray:
    """Seeded [N, nops, nsets] coefficients for tests at reduced mode counts."""
    nq = math.comb(m, 2)
    N = nq + math.comb(m, 4)
    rng = np.random.default_rng([SEED_BASE, 1000 + m, seed])
    z = np.zeros((N, nops, nsets))
    z[:nq, 0, :] = rng.normal(0.0, 1.0, size=(nq, nsets))
    z[nq:, 0, :] = rng.normal(0.0, quart_sd, size=(N - nq, nsets))
    if nops > 1:
        z[:nq, 1:, :] = rng.normal(0.0, 1.0, size=(nq, nops - 1, nsets))
        if obs_quartic:
            z[nq:, 1:, :] = rng.normal(0.0, quart_sd, size=(N - nq, nops - 1, nsets))
    return z


def random_dense(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain seeded N(0, scale) array for operand / adjoint-seed tests."""
    rng = np.random.default_rng([SEED_BASE, 7, seed])
    return rng.normal(0.0, scale, size=shape)


def pb_label(key: int, M: int, W: int):
    """(tau, c, a) of a Pauli-boson label key: W-bit fields, from the top:
    degree, tau (2 bits), then c_1, a_1, ..., c_M, a_M (the layout
    cut_graph_labels documents)."""
    mask = (1 << W) - 1
    c, a = [0] * M, [0] * M
    for m in range(M - 1, -1, -1):
        a[m] = key & mask
        key >>= W
        c[m] = key & mask
        key >>= W
    return (key & 3, tuple(c), tuple(a))


def pb_hermitian(labels, rng, diag_scale: float = 1.0, off_scale: float = 0.1) -> np.ndarray:
    """Seeded complex coefficients of a Hermitian operator over Pauli-boson
    labels (tau, c, a): h_{L^+} = conj(h_L) with B_{tau,c,a}^+ = B_{tau,a,c};
    block-diagonal labels (tau in {I, z}, c = a) ~ N(0, diag_scale), the others
    off_scale * (N(0,1) + i N(0,1)), real where a label is its own adjoint."""
    index = {L: n for n, L in enumerate(labels)}
    h = np.zeros(len(labels), dtype=complex)
    for n, L in enumerate(labels):
        m = index[(L[0], L[2], L[1])]
        if m < n:
            continue
        diag = L[0] in (0, 3) and L[1] == L[2]
        if m == n:
            h[n] = rng.normal() * (diag_scale if diag else off_scale)
        else:
            h[n] = off_scale * (rng.normal() + 1j * rng.normal())
            h[m] = np.conj(h[n])
    return h


def pb_fock_scale(labels) -> np.ndarray:
    """1 / sqrt(prod_m c_m! a_m!) per Pauli-boson label (tau, c, a): the size of
    (b^+)^c b^a between low Fock states grows like sqrt(c! a!), so coefficients
    drawn on this scale keep high-degree registries (degree 24) in range."""
    import math
    return np.array([1.0 / math.sqrt(math.prod(math.factorial(v) for v in L[1] + L[2])) for L in labels])


def real_split(v: np.ndarray) -> np.ndarray:
    """Interleaved real-split rows (axis 0): row 2r = Re v_r, row 2r + 1 = Im v_r."""
    out = np.empty((2 * v.shape[0],) + v.shape[1:])
    out[0::2] = v.real
    out[1::2] = v.imag
    return out


def from_real_split(a: np.ndarray) -> np.ndarray:
    """Inverse of real_split."""
    return a[0::2] + 1j * a[1::2]
