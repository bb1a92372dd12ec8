"""Test-side reader of the graph bundle file (layout of include/cutgraph.h,
cut_graph_build): header, section table, then 64-byte aligned sections."""
from __future__ import annotations

import struct

import numpy as np

HEADER = 256
SECTION = 32
NAMES = {1: "labels", 2: "diag", 3: "pairs", 4: "flow_off", 5: "flow_i", 6: "flow_j", 7: "flow_c",
         8: "gen_off", 9: "gen_i", 10: "gen_j", 11: "gen_c", 12: "out_labels", 13: "out_off",
         14: "out_i", 15: "out_j", 16: "out_c", 17: "gen_labels"}
DT = {1: np.uint64, 2: np.uint8, 3: np.int32, 4: np.int64, 5: np.int32, 6: np.int32, 7: np.int8,
      8: np.int64, 9: np.int32, 10: np.int32, 11: np.int8, 12: np.uint64, 13: np.int64, 14: np.int32,
      15: np.int32, 16: np.int8, 17: np.uint64}
FACTOR_SECTIONS = (7, 11, 16)


def read(path: str) -> dict:
    """Header fields and every section as a read-only array over a memory map of
    the file (nothing is copied, so multi-GB bundles read in place)."""
    b = np.memmap(path, dtype=np.uint8, mode="r")
    assert b[:8].tobytes() == b"CUTGRPH1"
    n_sections = struct.unpack_from("<I", b, 64)[0]
    table = struct.unpack_from("<Q", b, 72)[0]
    out = {"n_ops": struct.unpack_from("<q", b, 24)[0],
           "n_records": struct.unpack_from("<q", b, 32)[0],
           "gen_sign": struct.unpack_from("<i", b, 60)[0],
           "identifier": b[96:192].tobytes().split(b"\0")[0].decode(),
           "n_out_ops": struct.unpack_from("<q", b, 200)[0],
           "n_out_records": struct.unpack_from("<q", b, 208)[0],
           "n_gen_ops": struct.unpack_from("<q", b, 216)[0]}
    out["sections"] = {}
    for s in range(n_sections):
        sid, eb, off, cnt, ck = struct.unpack_from("<IIQQQ", b, table + s * SECTION)
        out["sections"][sid] = (off, cnt, eb)
        if sid in FACTOR_SECTIONS and eb in (4, 16):  # complex factors: int16 or FP64 (re, im)
            dt = np.int16 if eb == 4 else np.float64
            out[NAMES[sid]] = np.frombuffer(b, dtype=dt, count=2 * cnt, offset=off).reshape(cnt, 2)
        else:
            out[NAMES[sid]] = np.frombuffer(b, dtype=DT[sid], count=cnt, offset=off)
    return out


def records(d: dict, which: str = "flow"):
    off = d[f"{which}_off"]
    k = np.repeat(np.arange(off.size - 1), np.diff(off))
    c = d[f"{which}_c"]
    c = c.astype(np.float64) if c.ndim == 1 else c[:, 0].astype(np.float64) + 1j * c[:, 1].astype(np.float64)
    return (k.astype(np.int64), d[f"{which}_i"].astype(np.int64), d[f"{which}_j"].astype(np.int64), c)


def pb_label(key: int, M: int, W: int):
    import workloads
    return workloads.pb_label(key, M, W)
