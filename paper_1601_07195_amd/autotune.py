"""Autotuner for the batched persistent launch (qs_batch_run).

The launch shape of a batch -- threads per workgroup, the LDS chunk size
2^C (which also decides which states stay in LDS for the whole circuit),
the number K of higher qubits a gate segment may put into a chunk, the
persistent workgroups per compute unit and the queue order -- changes its
speed, never its results beyond rounding.  The best shape depends on the
amplitude type and on the mix of circuit widths and depths, so it is
measured: a coordinate-descent sweep times the candidate shapes on the
batch itself (or on a sample of it), one parameter at a time, keeping the
best, and caches the winner in a JSON file keyed by the dtype and the
batch's width/depth histogram.

Every timed call goes through the C ABI; nothing here computes physics.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import qs as Q

# Candidate values per parameter, swept in this order.
SPACE = {
    "lds_bits": (10, 11, 12),
    "khigh": (3, 4, 5, 6),
    "threads": (256, 512),
    "wg_per_cu": (1, 2, 3, 4),
    "order": (0, 1),
}
DEFAULT = {"threads": 256, "lds_bits": 11, "khigh": 5, "wg_per_cu": 2, "order": 0}


def valid(t: dict, dtype: int) -> bool:
    amp = 16 if dtype == Q.QS_C128 else 8
    if 2 * (1 << t["lds_bits"]) * amp > 128 * 1024:
        return False
    return 2 <= t["khigh"] <= min(8, t["lds_bits"] - 6)


def signature(batch: "Q.Batch") -> str:
    """Cache key: dtype, circuit count and the histogram of widths, with the
    mean gate count per width."""
    n = np.asarray(batch.n)
    gates = np.diff(batch.op_off)
    parts = []
    for w in np.unique(n):
        sel = n == w
        parts.append(f"{int(w)}:{int(sel.sum())}:{int(round(gates[sel].mean()))}")
    return f"dtype{batch.dtype}/c{batch.ncircuits}/" + ",".join(parts)


def time_run(batch: "Q.Batch", tuning: dict, repeats: int = 1) -> float:
    """Best wall time (s) of `repeats` synchronous qs_batch_run calls."""
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        batch.run_flat(tuning)
        best = min(best, time.perf_counter() - t0)
    return best


def tune(batch: "Q.Batch", repeats: int = 2, cache: str | None = None, log=None) -> dict:
    """Coordinate-descent search over SPACE; returns the fastest tuning as a
    dict of qs_batch_tuning fields (with the measured time under "_s")."""
    key = signature(batch)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return dict(table[key])
    batch.run_flat(DEFAULT)  # first call builds the schedule and workspace
    best = dict(DEFAULT)
    best_t = time_run(batch, best, repeats)
    tried = {tuple(sorted(best.items())): best_t}
    for name, values in SPACE.items():
        for v in values:
            cand = dict(best)
            cand[name] = v
            if name == "lds_bits":  # keep the chunk qubits valid for the new size
                cand["khigh"] = min(cand["khigh"], v - 6)
            k = tuple(sorted(cand.items()))
            if k in tried or not valid(cand, batch.dtype):
                continue
            batch.run_flat(cand)  # schedule for this (C, K) built outside the timing
            t = time_run(batch, cand, repeats)
            tried[k] = t
            if log:
                log(f"autotune {cand} {t * 1e3:.2f} ms")
            if t < best_t:
                best, best_t = cand, t
    out = dict(best)
    out["_s"] = best_t
    if cache:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = out
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return out


def fields(t: dict) -> dict:
    """The qs_batch_tuning fields of a tuning dict (drops "_s")."""
    return {k: v for k, v in t.items() if not k.startswith("_")}
