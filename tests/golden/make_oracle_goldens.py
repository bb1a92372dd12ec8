"""Writes the oracle's long-run results used as expected values by GPU tests.

Calls only the oracle (and the seeded workload generator):
  cfg2_flow_s10.npy  config 2 (m=24, H + 2 quadratic observables, G2, delta=0.5,
                     classic RK4 ds=5e-3 to s=10): z at s=10, shape [N, 3, 1]
  cfg5_grad_s10.npy  config 5 (m=24, 8 sets, H only, s=10, checkpoints every
                     16 steps): dL/dh0 for L = sum_b sum_a h_{P_a}(10), shape [N, 1, 8]

Usage: python tests/golden/make_oracle_goldens.py [cfg2|cfg5 ...]
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["cfg2", "cfg5"]
    for name in which:
        {"cfg2": cfg2, "cfg5": cfg5}[name]()
