"""Measured random-access ceilings of one GPU (hm_random_access).

For each access kind and buffer footprint, run n_ops random accesses and time
them with HIP events on the launch stream.  Rates are reported in accesses/s
and in GB/s of 64-byte lines (the unit the k-mer passes are priced in).

    python -m paper_1705_11147_amd.roofline [footprint_GB ...]
"""
from __future__ import annotations

import json
import sys

import torch

from . import abi

KINDS = {"load": abi.HM_RA_LOAD, "load_coherent": abi.HM_RA_LOAD_COHERENT, "atomic_add": abi.HM_RA_ATOMIC_ADD,
         "atomic_or_ret": abi.HM_RA_ATOMIC_OR_RET, "line_rmw": abi.HM_RA_LINE_RMW,
         "probe_cas": abi.HM_RA_PROBE_CAS,
         # one access in flight per thread (the others keep four)
         "load_serial": abi.HM_RA_LOAD | abi.HM_RA_SERIAL, "atomic_add_serial": abi.HM_RA_ATOMIC_ADD | abi.HM_RA_SERIAL,
         "probe_cas_serial": abi.HM_RA_PROBE_CAS | abi.HM_RA_SERIAL}


def measure(footprint_bytes: int, kinds=tuple(KINDS), n_ops: int = 1 << 28, reps: int = 3, device="cuda") -> dict:
    words = 1 << max(4, (int(footprint_bytes) // 8).bit_length() - 1)
    buf = torch.zeros(words, dtype=torch.int64, device=device)
    sink = torch.zeros(1, dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream()
    out = {"footprint_bytes": words * 8}
    for name in kinds:
        kind = KINDS[name]
        abi.call("hm_random_access", buf.data_ptr(), words, kind, n_ops // 8, 7, sink.data_ptr(), stream.cuda_stream)
        best = None
        for r in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            abi.call("hm_random_access", buf.data_ptr(), words, kind, n_ops, 11 + r, sink.data_ptr(),
                     stream.cuda_stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        rate = n_ops / (best / 1000)
        lines = 1  # every kind touches one 64-byte line per access
        out[name] = {"ops_per_s": rate, "line_GBps": rate * 64 * lines / 1e9, "ms": best}
    # streaming copy of half the buffer onto the other half
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    abi.call("hm_random_access", buf.data_ptr(), words, abi.HM_RA_COPY, 0, 0, sink.data_ptr(), stream.cuda_stream)
    e0.record(stream)
    abi.call("hm_random_access", buf.data_ptr(), words, abi.HM_RA_COPY, 0, 0, sink.data_ptr(), stream.cuda_stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    out["copy"] = {"GBps": words * 8 / (ms / 1000) / 1e9, "ms": ms}  # bytes read + written
    del buf
    return out


def copy_only(gib: float, device="cuda") -> dict:
    """One streaming copy of gib/2 GiB onto the other half of a gib-GiB buffer
    (reads and writes gib/2 GiB each): the reference dispatch for scaling
    byte counters such as FETCH_SIZE / WRITE_SIZE."""
    words = int(gib * 2 ** 30) // 8
    buf = torch.zeros(words, dtype=torch.int64, device=device)
    sink = torch.zeros(1, dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream()
    abi.call("hm_random_access", buf.data_ptr(), words, abi.HM_RA_COPY, 0, 0, sink.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return {"copy_bytes_read": words * 4, "copy_bytes_written": words * 4}


def main(argv):
    abi.lib()
    if argv and argv[0] == "--copy":
        print(json.dumps(copy_only(float(argv[1]) if len(argv) > 1 else 1.0)), flush=True)
        return
    sizes = [float(x) for x in argv] or [0.0625, 1.0, 16.0]
    for gb in sizes:
        print(json.dumps(measure(int(gb * 2 ** 30))), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
