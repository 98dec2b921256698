"""Host throughput of the CPU oracle (FP64): S steps of an N^3 grid on the headline box,
once on one thread, and as P concurrent single-threaded processes, each stepping the
same input (the oracle has no threads of its own; P defaults to the smaller of the
host's CPU count and 16).  The aggregate rate is P x S x N^3 / wall time.  It is a
reported baseline for the GPU figures, not a target.

Run: python tests/oracle_timing.py [--procs P] [--n N] [--steps S]
It lives with the tests because it runs the oracle.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_FIELDS = None  # inherited by forked workers
_STEPS = 1


def _one_step(_):
    from oracle import oracle as orc
    from paper_2210_06232_amd.workload import HEADLINE
    H, E = _FIELDS
    t0 = time.perf_counter()
    orc.step(H, E, tuple(HEADLINE["domain"]), HEADLINE["mu"], HEADLINE["eps"], HEADLINE["tau"], _STEPS)
    return time.perf_counter() - t0


def host():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def run(procs: int, n: int, steps: int = 1):
    global _FIELDS, _STEPS
    _STEPS = steps
    from paper_2210_06232_amd import inputs
    from paper_2210_06232_amd.workload import HEADLINE
    _FIELDS = inputs.random_fields((n, n, n), tuple(HEADLINE["domain"]), workload=2, p=2.0)
    pts = n ** 3 * steps
    single = _one_step(0)
    print(f"[oracle timing] one thread: {single:.2f} s", flush=True)
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        t0 = time.perf_counter()
        each = pool.map(_one_step, range(procs), chunksize=1)
        wall = time.perf_counter() - t0
    out = {"workload": HEADLINE["workload"] if n == HEADLINE["grid"][0] else f"{n}^3 sample of the headline box",
           "steps": steps,
           "unit": "field-point-steps/s",
           "single": {"threads": 1, "seconds": round(single, 2), "value": pts / single},
           "parallel": {"processes": procs, "wall_s": round(wall, 2), "max_process_s": round(max(each), 2),
                        "value": procs * pts / wall},
           "host": host()}
    print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--procs", type=int, default=min(os.cpu_count() or 1, 16))
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=1)
    a = ap.parse_args()
    run(a.procs, a.n, a.steps)


if __name__ == "__main__":
    main()
