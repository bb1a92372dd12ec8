"""Host-side checks of the benchmark's contract (no GPU): it runs on one GPU
only and says so for any other count; its algorithmic byte count per fused
pass matches the layout it describes; the roofline constants follow from the
chip's unit counts and published peaks."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_pass_bytes_and_ceilings():
    import bench
    N, E, nsets, nops = 92170, 39539760, 64, 5
    cols = nsets * nops
    # records, offsets, float generator and stage operand, FP64 state traffic
    # (z read, accumulator 14 B average), next float operand, FP64 H column
    want = 8 * E + 8 * (N + 1) + 4 * N * nsets + 4 * N * cols + 22 * N * cols + 4 * N * cols + 8 * N * nsets
    assert bench.pass_bytes(N, E, nsets, nops, 4) == want
    assert abs(bench.pass_bytes(N, E, nsets, nops, 4) - 1.2727e9) < 1e6
    # one 64-lane instruction per SIMD every 4 clocks: 64 lanes x 2 flops (FMA)
    # at that rate is the published non-packed FP32 / FP64 vector peak (78.6)
    assert abs(bench.VALU_INSTS_PER_S * 64 * 2 / 1e12 - 78.6) < 0.1
    assert bench.HBM_PEAK_GBS == 8000.0
