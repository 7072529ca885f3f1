"""Measured choice of the schedule knobs for one workload.

The planner's cost model picks the materialised depth of each half's copy
tree and packs gates into tiles of a fixed width.  This module times a small
grid of candidates on the GPU (tile width, light-cone limit, a forced
materialised depth around the model's choice) through the C ABI and keeps the
fastest.  Results are cached in a JSON file keyed by the circuit text, the cut
and the bitstring set.
"""

from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import Plan


def _key(text: str, mask: int, bits: np.ndarray, k0: int, k1: int) -> str:
    h = hashlib.sha256()
    h.update(text.encode())
    h.update(str((mask, k0, k1)).encode())
    h.update(np.ascontiguousarray(bits, dtype=np.uint64).tobytes())
    return h.hexdigest()[:24]


def _time_opts(text, mask, bits, k0, k1, opts, reps, stream, sync) -> float:
    p = Plan(text, mask, **opts)
    try:
        p.run_halves(k0, k1, bits, stream)
        p.amplitudes_device(0, _scratch(bits.size), None, stream)
        sync()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            p.reset(keep_bitstrings=True)
            p.run_halves(k0, k1, None, stream)
            p.amplitudes_device(0, _scratch(bits.size), None, stream)
            sync()
            best = min(best, time.perf_counter() - t0)
        return best
    finally:
        p.close()


_SCRATCH = {}


def _scratch(m: int) -> int:
    import torch
    t = _SCRATCH.get(m)
    if t is None:
        t = torch.empty(2 * m, dtype=torch.float32, device="cuda")
        _SCRATCH[m] = t
    return t.data_ptr()


def candidates(base_levels=(-1,)):
    out = []
    for ml in base_levels:
        for tb in (10, 11):
            for tq in (8, 10):
                out.append(dict(tile_bits=tb, tail_max_qubits=tq, materialize_level=ml))
    return out


def autotune(text: str, mask: int, bits, k0: int, k1: int, cache_path: str | None = None,
             reps: int = 2, extra_levels=(), stream=None, budget_s: float = 60.0) -> dict:
    """Fastest knob set for the workload: {'opts': {...}, 'ms': t, 'tried': [...]}"""
    import torch
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    key = _key(text, mask, bits, k0, k1)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    sync = torch.cuda.synchronize
    tried = []
    t_start = time.perf_counter()
    for opts in candidates((-1,) + tuple(extra_levels)):
        if time.perf_counter() - t_start > budget_s:
            break
        try:
            t = _time_opts(text, mask, bits, k0, k1, opts, reps, stream, sync)
        except Exception as e:  # a knob set the planner rejects
            tried.append({"opts": opts, "error": str(e)})
            continue
        tried.append({"opts": opts, "ms": t * 1e3})
    ok = [x for x in tried if "ms" in x]
    if not ok:
        raise RuntimeError("no candidate ran")
    best = min(ok, key=lambda x: x["ms"])
    res = {"opts": best["opts"], "ms": best["ms"], "tried": tried}
    if cache_path:
        cache[key] = res
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return res
