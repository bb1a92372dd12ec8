"""Writes the oracle's long-run results used as expected values by GPU tests.

Calls only the oracle (and the seeded workload generator):
  cfg2_flow_s10.npy  config 2 (m=24, H + 2 quadratic observables, G2, delta=0.5,
                     classic RK4 ds=5e-3 to s=10): z at s=10, shape [N, 3, 1]
  cfg5_grad_s10.npy  config 5 (m=24, 8 sets, H only, s=10, checkpoints every
                     16 steps): dL/dh0 for L = sum_b sum_a h_{P_a}(10), shape [N, 1, 8]
  cfg3_full_flow_set{b}.npy
                     config 3 (m=40, G2, delta=0.5, ds=5e-3): the whole ragged
                     flow of set b alone (H + 4 observables, n_b RK4 steps) for
                     the shortest and the longest set, shape [N, 5, 1]
  cfg4_two_steps.npy config 4 (m=64, G2, ds=5e-3): z after 2 RK4 steps of sets
                     0 and 15, shape [N, 1, 2]
  cfg2_g1_flow_s10.npy
                     config 2 with the literal generator G1 (delta=0.5): z at
                     s=10, shape [N, 3, 1] (precision study)

Sets are independent in the flow (each set's generator is built from its own
Hamiltonian column), so a set flowed alone is the set flowed in the batch.

Usage: python tests/golden/make_oracle_goldens.py [cfg2|cfg2_g1|cfg5|cfg3|cfg4 ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import native  # noqa: E402


def cfg2():
    w = workloads.WORKLOADS[2]
    inp = workloads.make_inputs(2)
    g = native.majorana_graph(w.size)
    t = time.time()
    z, _ = native.Engine(g, "g2", w.delta).flow(inp.z0, w.ds, inp.n_steps)
    np.save(os.path.join(HERE, "cfg2_flow_s10.npy"), z)
    print(f"cfg2: {inp.n_steps} steps in {time.time() - t:.1f} s", flush=True)


def cfg2_g1():
    """Config 2 with the literal generator G1 (precision study): z at s=10."""
    w = workloads.WORKLOADS[2]
    inp = workloads.make_inputs(2)
    g = native.majorana_graph(w.size)
    t = time.time()
    z, _ = native.Engine(g, "g1", w.delta).flow(inp.z0, w.ds, inp.n_steps)
    np.save(os.path.join(HERE, "cfg2_g1_flow_s10.npy"), z)
    print(f"cfg2 G1: {inp.n_steps} steps in {time.time() - t:.1f} s", flush=True)


def cfg5():
    w = workloads.WORKLOADS[5]
    inp = workloads.make_inputs(5)
    g = native.majorana_graph(w.size)
    lam_end = np.zeros_like(inp.z0)
    lam_end[g.pairs, 0, :] = 1.0
    t = time.time()
    lam = native.Engine(g, "g2", w.delta).flow_adjoint(inp.z0, w.ds, inp.n_steps, lam_end,
                                                        ckpt_every=w.ckpt_every)
    np.save(os.path.join(HERE, "cfg5_grad_s10.npy"), lam)
    print(f"cfg5: gradient in {time.time() - t:.1f} s", flush=True)


def cfg3_sets():
    """Indices of the shortest and the longest flow of config 3."""
    ns = workloads.make_inputs(3).n_steps
    return int(np.argmin(ns)), int(np.argmax(ns))


def cfg3():
    w = workloads.WORKLOADS[3]
    inp = workloads.make_inputs(3)
    t = time.time()
    g = native.majorana_graph(w.size)
    eng = native.Engine(g, "g2", w.delta)
    print(f"cfg3: oracle records in {time.time() - t:.1f} s", flush=True)
    for b in cfg3_sets():
        t = time.time()
        z, _ = eng.flow(inp.z0[:, :, b:b + 1], w.ds, inp.n_steps[b:b + 1])
        np.save(os.path.join(HERE, f"cfg3_full_flow_set{b}.npy"), z)
        print(f"cfg3: set {b}, {int(inp.n_steps[b])} steps in {time.time() - t:.1f} s", flush=True)


CFG4_SETS = (0, 15)


def cfg4():
    w = workloads.WORKLOADS[4]
    inp = workloads.make_inputs(4)
    t = time.time()
    g = native.majorana_graph(w.size)
    eng = native.Engine(g, "g2", w.delta)
    print(f"cfg4: oracle records in {time.time() - t:.1f} s", flush=True)
    sel = list(CFG4_SETS)
    t = time.time()
    z, _ = eng.flow(np.ascontiguousarray(inp.z0[:, :, sel]), w.ds, np.full(len(sel), 2, np.int32))
    np.save(os.path.join(HERE, "cfg4_two_steps.npy"), z)
    print(f"cfg4: 2 steps of sets {sel} in {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["cfg2", "cfg5"]
    for name in which:
        {"cfg2": cfg2, "cfg2_g1": cfg2_g1, "cfg5": cfg5, "cfg3": cfg3, "cfg4": cfg4}[name]()
