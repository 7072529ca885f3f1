"""Measured choice of the schedule knobs for a workload.

The planner's cost model picks the materialised depth of each half's copy
tree, packs gates into tiles of a fixed width, and lets a pass descend up to
two tree levels.  This module times candidate knob sets on the GPU through the
C ABI and keeps the fastest.  The knobs searched:

* ``tile_bits``: the fusion width, the state bits one wavefront tile holds
  (gates on them fuse into one pass over HBM): 9, 10 or 11;
* ``max_stages``: the fusion depth, the tree levels one pass may descend: 1 or 2;
* ``copies_per_launch``: the copy block one launch of the passes and the leaf
  evaluation covers (all copies, or a quarter of them per block);
* ``materialize_level``: the last materialised tree level (the cost model's
  choice, or forced one level either side of it);
* ``tail_max_qubits``: the largest light cone of the leaf evaluation: 8 or 10;
* ``no_exchange``: whether runs of passes may share a launch and exchange their
  workgroup tiles through LDS (0) or run one launch per pass (1).

The search is coordinate descent from the cost model's defaults: each knob in
turn takes every value with the others fixed, and the best is kept; the tile
width and the grouping are searched together (a wider tile changes whether
grouping pays).  A result
is stored in a JSON file under the workload's name, with the SHA-256 of the
circuit text, cut, copy range and bitstrings it was measured on; a reader
uses the stored knobs only if that key still matches.

    python -m paper_1802_06952_amd.autotune grid6x7_d20 grid6x6_d16 ... [--out FILE]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

from . import Plan, QSError

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")


def workload_key(text: str, mask: int, bits: np.ndarray, k0: int, k1: int) -> str:
    h = hashlib.sha256()
    h.update(text.encode())
    h.update(str((mask, k0, k1)).encode())
    h.update(np.ascontiguousarray(bits, dtype=np.uint64).tobytes())
    return h.hexdigest()[:24]


_SCRATCH = {}


def _scratch(m: int) -> int:
    import torch
    t = _SCRATCH.get(m)
    if t is None:
        t = torch.empty(2 * m, dtype=torch.float32, device="cuda")
        _SCRATCH[m] = t
    return t.data_ptr()


def time_opts(text, mask, bits, k0, k1, opts, reps=3, stream=None) -> float:
    """Best step time in seconds (run_halves over [k0, k1) plus the FP32
    assembly) of a plan with the given knobs, after one untimed step."""
    import torch
    p = Plan(text, mask, **opts)
    try:
        p.run_halves(k0, k1, bits, stream)
        p.amplitudes_device(0, _scratch(bits.size), None, stream)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            p.reset(keep_bitstrings=True)
            p.run_halves(k0, k1, None, stream)
            p.amplitudes_device(0, _scratch(bits.size), None, stream)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best
    finally:
        p.close()


def knob_values(n_cuts: int, k0: int, k1: int, model_levels: list[int]) -> dict:
    """The values tried per knob; the first of each list is the default."""
    span = k1 - k0
    cpl = [0]
    if span >= 4 and (span & (span - 1)) == 0:
        cpl.append(span // 4)
    lv = [-1]
    for base in sorted(set(model_levels)):
        for d in (-1, 1):
            if base + d >= 0 and base + d not in lv:
                lv.append(base + d)
    return {"tile_bits": [10, 9, 11], "max_stages": [2, 1], "copies_per_launch": cpl,
            "materialize_level": lv, "tail_max_qubits": [10, 8], "no_exchange": [0, 1]}


def autotune(text: str, mask: int, bits, k0: int, k1: int, reps: int = 3, stream=None,
             budget_s: float = 120.0, log=None) -> dict:
    """Fastest knob set by coordinate descent: {'opts', 'ms', 'default_ms', 'tried'}."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    probe = Plan(text, mask)
    try:
        d = probe.dump(k0, k1)
        n_cuts = probe.n_cuts
    finally:
        probe.close()
    model_levels = [s.get("lstar", 0) for s in d["sides"]]
    values = knob_values(n_cuts, k0, k1, model_levels)
    cur = {k: v[0] for k, v in values.items()}
    tried = {}
    # axes of the descent: tile width and grouping jointly, then one knob each
    axes = [[{"tile_bits": t, "no_exchange": e} for t in values["tile_bits"]
             for e in values["no_exchange"]]]
    axes += [[{k: v} for v in vals] for k, vals in values.items()
             if k not in ("tile_bits", "no_exchange")]

    def measure(opts):
        key = json.dumps(opts, sort_keys=True)
        if key not in tried:
            try:
                tried[key] = time_opts(text, mask, bits, k0, k1, opts, reps, stream) * 1e3
            except QSError as e:   # a knob set the planner rejects
                tried[key] = float("inf")
                if log:
                    log(f"  {opts}: {e}")
            if log and np.isfinite(tried[key]):
                log(f"  {opts}: {tried[key]:.3f} ms")
        return tried[key]

    t_start = time.perf_counter()
    default_ms = best_ms = measure(cur)
    for axis in axes:
        base = cur
        for part in axis:
            if time.perf_counter() - t_start > budget_s:
                break
            cand = dict(base, **part)
            if cand == base:
                continue
            ms = measure(cand)
            if ms < best_ms:
                best_ms, cur = ms, cand
    if not np.isfinite(best_ms):
        raise RuntimeError("no knob set ran")
    return {"opts": cur, "ms": best_ms, "default_ms": default_ms,
            "tried": [{"opts": json.loads(k), "ms": v if np.isfinite(v) else None}
                      for k, v in tried.items()]}


def load_tuned(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f).get("workloads", {})


def tuned_opts(name: str, key: str, path: str = DEFAULT_CACHE) -> dict | None:
    """Stored knobs of a workload if they were measured on the same inputs."""
    e = load_tuned(path).get(name)
    if e and e.get("key") == key:
        return e["opts"]
    return None


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--budget-s", type=float, default=120.0)
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from workloads import product_bitstrings, workload
    torch.cuda.set_device(0)
    store = {"workloads": load_tuned(a.out)}
    for name in a.workloads:
        w = workload(name)
        text = w.circuit_text()
        bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
        p = Plan(text, w.upper_mask)
        k1 = w.copy_end if w.copy_end is not None else (1 << p.n_cuts)
        p.close()
        print(f"autotune {name}: copies [{w.copy_begin}, {k1}), {bits.size} bitstrings", flush=True)
        r = autotune(text, w.upper_mask, bits, w.copy_begin, k1, budget_s=a.budget_s,
                     log=lambda s: print(s, flush=True))
        r["key"] = workload_key(text, w.upper_mask, bits, w.copy_begin, k1)
        r["device"] = torch.cuda.get_device_name(0)
        store["workloads"][name] = r
        print(f"  best {r['opts']}: {r['ms']:.3f} ms (cost-model defaults {r['default_ms']:.3f} ms)",
              flush=True)
        with open(a.out, "w") as f:
            json.dump(store, f, indent=1)
            f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
