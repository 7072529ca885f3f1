#!/usr/bin/env python
"""Throughput of the CZ-partition hot path on one MI355X.

A step is one pass of the whole hot path over the workload: every copy of
both half circuits simulated on the GPU (qs_run_halves over [0, 2^c)), then
the assembly amp(u, l) = sum_k U_k[u] L_k[l] and the FP64 probability sums
(qs_amplitudes_device).  The bitstrings are registered (uploaded) before the
timed region and the amplitudes stay in HBM, so the timed work is device work
plus its host-side launches.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--prec fp32|bf16x3] [--no-cpu-baseline] [--no-plain]

Prints one JSON line.  ``value`` is output amplitudes per second.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {0: 157.3, 1: 2500.0}   # FP32 MFMA; dense BF16 MFMA


def _kernel_source_hash() -> str:
    path = os.path.join(ROOT, "paper_1802_06952_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic_from_profile(kernel_family: str, workload: str):
    """HBM bytes per launch from a committed counter summary, if it matches the current kernels."""
    path = os.path.join(ROOT, "profiles", f"{kernel_family}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except Exception:
        return None
    if d.get("kernels_hip_sha256_16") != _kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def _oracle_subtree(args):
    """One worker of the oracle baseline: the FP64 partition oracle on copies
    [k0, k1) (a subtree of the copy tree: its shared prefix is recomputed),
    its partial amplitudes on the gathered values."""
    text, mask, u, l, k0, k1 = args
    import torch
    torch.set_num_threads(1)
    from oracle import circuit as OC, partition as P
    A, B = P.gathered_halves(OC.parse(text), mask, u, l, k0, k1)
    return A @ B.T


def _worker_init():
    import torch
    torch.set_num_threads(1)
    import oracle.partition  # noqa: F401  (imports before the timed region)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_copies: int, n_values: int, workers: int):
    """The FP64 oracle on the host on a bounded sample of the same workload:
    copies [0, n_copies) split into aligned subtrees, one worker process per
    subtree (each recomputes the prefix it shares with the others, as a GPU
    of a multi-GPU run would), partial amplitudes summed at the end."""
    import multiprocessing as mp
    import numpy as np
    from oracle import circuit as OC, partition as P
    from workloads import product_bitstrings

    text = w.circuit_text()
    c = len(P.find_cuts(OC.parse(text), w.upper_mask))
    total = 1 << c
    k1 = min(total, n_copies)
    workers = max(1, min(workers, k1))
    while k1 % workers:
        workers -= 1
    _, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    u = u[:n_values].astype(np.int64)
    l = l[:n_values].astype(np.int64)
    per = k1 // workers
    jobs = [(text, w.upper_mask, u, l, i * per, (i + 1) * per) for i in range(workers)]
    ctx = mp.get_context("spawn")   # the parent holds a GPU context: never fork it
    with ctx.Pool(workers, initializer=_worker_init) as pool:
        pool.map(_worker_init_probe, range(workers))   # every worker started and imported
        t0 = time.perf_counter()
        parts = pool.map(_oracle_subtree, jobs)
        dt = time.perf_counter() - t0
    C = sum(parts)
    assert C.shape == (len(u), len(l))
    # the gathered set size hardly matters (full half states are simulated);
    # the whole job runs every copy: scale the time by the copy count
    scaled = dt * total / k1
    m = w.n_u * w.n_l
    return {"value": m / scaled, "unit": "amplitudes/s", "cores": workers, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"FP64 oracle on copies [0, {k1}) of {total} in {workers} worker processes "
                      f"(one thread each; aligned subtrees of {per} copies, both halves, prefix "
                      f"reuse over cut layers inside a subtree, each worker recomputing the prefix "
                      f"its subtree shares with the others; {len(u)} upper x {len(l)} lower values "
                      f"gathered): {dt:.2f} s, extrapolated linearly by {total}/{k1} copies to the "
                      f"whole job of {m} amplitudes"}


def tuned_knobs(Q, names) -> dict:
    """Knobs the autotuner stored for the named workloads
    (paper_1802_06952_amd/tuned.json), for those whose stored key still
    matches the circuit, cut, copy range and bitstrings; the others are left
    to the cost model."""
    from paper_1802_06952_amd.autotune import tuned_opts, workload_key
    from workloads import product_bitstrings, workload
    out = {}
    for name in names:
        w = workload(name)
        text = w.circuit_text()
        bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
        p = Q.Plan(text, w.upper_mask)
        k1 = w.copy_end if w.copy_end is not None else (1 << p.n_cuts)
        p.close()
        o = tuned_opts(name, workload_key(text, w.upper_mask, bits, w.copy_begin, k1))
        if o is not None:
            out[name] = o
    return out


def _worker_init_probe(_):
    return os.getpid()


def controlled_variant(Q, w, bits, prec, k0, k1, a, stream, d_out, d_sums) -> dict:
    """Amplitudes/s of the workload's grid, depth, cut and bitstrings with
    every two-qubit gate drawn from CZ, CNOT and CY and a random control
    (controlled-U cuts, Supp. Eq. 1)."""
    import torch
    from workloads.circuits import random_grid_circuit
    m = int(bits.size)
    ctext = random_grid_circuit(w.rows, w.cols, w.depth, w.seed, "mixed", "random")
    cp = Q.Plan(ctext, w.upper_mask, one_stream=a.one_stream)
    try:
        ck1 = k1 if w.copy_end is not None else (1 << cp.n_cuts)

        def cstep(p):
            cp.reset(keep_bitstrings=True)
            cp.run_halves(k0, ck1, None, stream)
            cp.amplitudes_device(p, d_out.data_ptr(), d_sums.data_ptr(), stream)

        cp.run_halves(k0, ck1, bits, stream)
        cp.amplitudes_device(prec, d_out.data_ptr(), d_sums.data_ptr(), stream)
        for _ in range(a.warmup):
            cstep(prec)
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        for _ in range(a.steps):
            cstep(prec)
        torch.cuda.synchronize()
        cms = (time.perf_counter() - tc0) * 1000.0 / a.steps
        return {"value": round(m / (cms / 1000.0), 1), "unit": "amplitudes/s",
                "ms_per_step": round(cms, 4), "cuts": cp.n_cuts,
                "workload": f"{w.name} with CZ, CNOT and CY drawn per gate, random controls "
                            f"(same grid, depth, cut and bitstrings)"}
    finally:
        cp.close()


def executed_updates(dump: dict, n_values) -> dict:
    """Gate-amplitude updates the schedule executes per step (metric (ii)'s
    executed count, next to the flat one): every gate of a full-state pass on
    every amplitude of every state it runs on (the last pass counted in full,
    although it computes only the tiles the leaf stage reads), plus the 2x2
    and diagonal gates of the leaf levels on the light-cone rows (2^q
    amplitudes per row, one row per leaf path prefix and requested value)."""
    passes = leaf = 0.0
    for s, S in zip(dump["sides"], n_values):
        n, ops, levels = s["n"], s["ops"], s["levels"]
        gate = lambda i: ops[i][0] != "cut"
        for pp in s["passes"]:
            li = pp["level_in"]
            passes += 2.0 ** n * levels[li]["nodes"] * sum(1 for i in pp["ops_in"] if gate(i))
            for st, so in enumerate(pp["stages"]):
                passes += 2.0 ** n * levels[li + st + 1]["nodes"] * sum(1 for i in so if gate(i))
        q = len(s["Q"])
        paths = 1.0
        for lv in reversed(levels[s["lstar"] + 1:]):
            leaf += S * paths * sum(1 for i in lv["ops"] if gate(i)) * 2.0 ** q
            paths *= 2.0 ** len(lv["cuts"])
    return {"passes": passes, "leaf_rows": leaf, "total": passes + leaf}


def error_stats(a, ref) -> dict:
    """Errors of computed amplitudes a against the FP64 oracle's ref: the
    norm-wise relative error, the largest absolute error, that over the rms
    amplitude, and the median of the per-amplitude relative errors."""
    import numpy as np
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    d = np.abs(a - ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return {"norm_rel": float(np.linalg.norm(a - ref) / np.linalg.norm(ref)),
            "max_abs": float(d.max()), "max_over_rms": float(d.max() / rms),
            "median_rel": float(np.median(d / np.maximum(np.abs(ref), 1e-300))),
            "n": int(a.size)}


def time_workload(Q, w, prec, steps, warmup, stream, knobs=None, one_stream=False,
                  graph=False) -> dict:
    """Amplitudes/s of one workload on its own: run_halves over its copy range
    and the assembly per step, bitstrings registered and outputs in HBM; with
    graph, also the same step replayed as one library-captured HIP graph."""
    import numpy as np
    import torch
    from workloads import product_bitstrings
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    m = int(bits.size)
    p = Q.Plan(w.circuit_text(), w.upper_mask, one_stream=one_stream, **(knobs or {}))
    try:
        k0 = w.copy_begin
        k1 = w.copy_end if w.copy_end is not None else (1 << p.n_cuts)
        d_out = torch.empty(2 * m, dtype=torch.float32, device="cuda")
        d_sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        p.run_halves(k0, k1, bits, stream)
        p.amplitudes_device(prec, d_out.data_ptr(), d_sums.data_ptr(), stream)

        def step():
            p.reset(keep_bitstrings=True)
            p.run_halves(k0, k1, None, stream)
            p.amplitudes_device(prec, d_out.data_ptr(), d_sums.data_ptr(), stream)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        r = {"value": round(m / (ms / 1000.0), 1), "unit": "amplitudes/s",
             "ms_per_step": round(ms, 4), "bitstrings": m, "copies": k1 - k0,
             "halves": [p.n_upper, p.n_lower], "cuts": p.n_cuts,
             "amplitudes": d_out.cpu().numpy().view(np.complex64)}
        if graph:
            gs = torch.cuda.Stream()   # a graph cannot be captured on the null stream
            p.run_graph(k0, k1, prec, d_out.data_ptr(), d_sums.data_ptr(), gs)
            for _ in range(warmup):
                p.run_graph(k0, k1, prec, d_out.data_ptr(), d_sums.data_ptr(), gs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                p.run_graph(k0, k1, prec, d_out.data_ptr(), d_sums.data_ptr(), gs)
            torch.cuda.synchronize()
            gms = (time.perf_counter() - t0) * 1000.0 / steps
            r["graph"] = {"value": round(m / (gms / 1000.0), 1), "ms_per_step": round(gms, 4),
                          "note": "the same step replayed as one HIP graph (qs_run_graph)"}
        return r
    finally:
        p.close()


def coscheduled_pair(Q, names, prec, steps, warmup, knobs) -> dict:
    """Two circuits cut into uneven halves, each plan on a stream of its own
    (and each plan's lower half on the plan's second stream), launched
    together every step: four half sizes in flight at once."""
    import numpy as np
    import torch
    from workloads import product_bitstrings, workload
    ws = [workload(n) for n in names]
    streams = [torch.cuda.Stream() for _ in ws]    # default priority
    plans, outs, ranges, ms_alone = [], [], [], []
    try:
        for w in ws:
            bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
            p = Q.Plan(w.circuit_text(), w.upper_mask, **knobs.get(w.name, {}))
            plans.append(p)
            k1 = w.copy_end if w.copy_end is not None else (1 << p.n_cuts)
            ranges.append((w.copy_begin, k1, int(bits.size)))
            outs.append((torch.empty(2 * bits.size, dtype=torch.float32, device="cuda"),
                         torch.zeros(2, dtype=torch.float64, device="cuda")))
            p.run_halves(w.copy_begin, k1, bits, streams[len(plans) - 1])
        torch.cuda.synchronize()

        def launch(i):
            p, (k0, k1, _), (o, sm), st = plans[i], ranges[i], outs[i], streams[i]
            p.reset(keep_bitstrings=True)
            p.run_halves(k0, k1, None, st)
            p.amplitudes_device(prec, o.data_ptr(), sm.data_ptr(), st)

        for i in range(len(plans)):   # each alone, for reference
            for _ in range(warmup):
                launch(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                launch(i)
            torch.cuda.synchronize()
            ms_alone.append((time.perf_counter() - t0) * 1000.0 / steps)
        for _ in range(warmup):
            for i in range(len(plans)):
                launch(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for i in range(len(plans)):
                launch(i)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        mtot = sum(r[2] for r in ranges)
        return {"value": round(mtot / (ms / 1000.0), 1), "unit": "amplitudes/s", "ms_per_step": round(ms, 4),
                "ms_alone_sum": round(sum(ms_alone), 4),
                "circuits": [{"workload": w.name, "halves": [p.n_upper, p.n_lower], "cuts": p.n_cuts,
                              "bitstrings": r[2], "ms_alone": round(t, 4),
                              "amplitudes_per_s_coscheduled": round(r[2] / (ms / 1000.0), 1),
                              "knobs": knobs.get(w.name, {}) or "cost model defaults"}
                             for w, p, r, t in zip(ws, plans, ranges, ms_alone)],
                "schedule": "each plan on its own stream, its lower half on the plan's second "
                            "stream: four half sizes in flight"}
    finally:
        for p in plans:
            p.close()


def per_pass_table(recs) -> list:
    """Every full-state pass launch of a step with its time averaged over the
    timed steps: [half, first pass, input level, stages, tiles, MB, us, GB/s,
    passes run by the launch]."""
    acc = {}
    for r in recs:
        k = (r["side"], r["pass"])
        e = acc.setdefault(k, [r["level_in"], r["stages"], r["tiles"], r["bytes"], 0.0, 0,
                               r.get("passes", 1)])
        e[4] += r["ms"]
        e[5] += 1
    rows = []
    for (side, pi), (li, st, tiles, b, ms, cnt, npass) in sorted(acc.items()):
        us = ms * 1000.0 / cnt
        rows.append([side, pi, li, st, tiles, round(b / 1e6, 2), round(us, 2),
                     round(b / (us * 1e3), 1), npass])
    return rows


def chain_variant(Q, a, stream) -> dict:
    """Amplitudes/s of a partition into four parts (Sec. 3, Fig. 3): the 8x8
    grid (64 qubits) at depth 10 cut into row bands of 16 qubits, 32 values
    per band (2^20 product-set bitstrings), inputs resident in HBM."""
    import numpy as np
    import torch
    from workloads.circuits import grid_rows_mask, random_grid_circuit
    rows, cols, depth = 8, 8, 10
    bands = [[0, 1], [2, 3], [4, 5], [6, 7]]
    text = random_grid_circuit(rows, cols, depth, 0)
    rng = np.random.default_rng(3000)
    bits = np.zeros(1, dtype=np.uint64)
    for b in bands:
        v = rng.choice(1 << 16, size=32, replace=False).astype(np.uint64)
        bits = (bits[:, None] | (v[None, :] << np.uint64(b[0] * cols))).reshape(-1)
    m = int(bits.size)
    cp = Q.ChainPlan(text, [grid_rows_mask(rows, cols, b) for b in bands])
    try:
        d_out = torch.empty(2 * m, dtype=torch.float32, device="cuda")
        d_sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        cp.register(bits)
        for _ in range(max(1, a.warmup)):
            cp.amplitudes_device(d_out.data_ptr(), d_sums.data_ptr(), stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            cp.amplitudes_device(d_out.data_ptr(), d_sums.data_ptr(), stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / a.steps
        sums = d_sums.cpu().numpy()
        return {"value": round(m / (ms / 1000.0), 1), "unit": "amplitudes/s", "ms_per_step": round(ms, 4),
                "parts": cp.t, "part_qubits": cp.part_qubits, "link_cuts": cp.link_cuts,
                "bitstrings": m, "mean_p_times_2n": float(sums[0] / m * 2.0 ** (rows * cols)),
                "workload": "8x8 grid (64 qubits), depth 10, seed 0, four row bands of 16 qubits; "
                            "32 values per band"}
    finally:
        cp.close()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid6x7_d20")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-controlled", action="store_true",
                    help="skip the controlled-U variant of the workload (CZ, CNOT and CY mixed)")
    ap.add_argument("--no-chain", action="store_true",
                    help="skip the four-part chain partition of the 64-qubit depth-10 circuit")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (36-qubit, the co-scheduled uneven pair, the "
                         "64-qubit slice)")
    ap.add_argument("--plain-copies", type=int, default=16)
    ap.add_argument("--cpu-copies", type=int, default=256)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="worker processes of the oracle baseline (at most the host's CPUs)")
    ap.add_argument("--autotune", action="store_true",
                    help="time a grid of schedule knobs first and run with the fastest")
    ap.add_argument("--one-stream", action="store_true",
                    help="run the two halves one after the other on one stream (as the "
                         "per-kernel timing does) instead of concurrently")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="after the steps, copy a tensor of this size (for counter calibration)")
    a = ap.parse_args()

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (the copies of a half circuit are independent, but "
              "splitting them over several GPUs is not implemented); use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_1802_06952_amd as Q
    from workloads import product_bitstrings, workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    prec = 0 if a.prec == "fp32" else 1
    w = workload(a.workload)
    text = w.circuit_text()
    bits, u_vals, l_vals = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    m = int(bits.size)
    c = Q.Plan(text, w.upper_mask).n_cuts
    k0 = w.copy_begin
    k1 = w.copy_end if w.copy_end is not None else (1 << c)
    tuned = None
    if a.autotune:
        from paper_1802_06952_amd.autotune import autotune
        tuned = autotune(text, w.upper_mask, bits, k0, k1, budget_s=90.0)
        knobs = tuned["opts"]
    else:
        # knobs the autotuner stored for this workload, if measured on the same inputs
        knobs = tuned_knobs(Q, (w.name,)).get(w.name, {})
    plan = Q.Plan(text, w.upper_mask, one_stream=a.one_stream, **knobs)
    stream = torch.cuda.current_stream()
    d_out = torch.empty(2 * m, dtype=torch.float32, device="cuda")
    d_sums = torch.zeros(2, dtype=torch.float64, device="cuda")

    t_setup = time.perf_counter()
    plan.run_halves(k0, k1, bits, stream)           # registers bitstrings, plans and uploads
    plan.amplitudes_device(prec, d_out.data_ptr(), d_sums.data_ptr(), stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup

    def step(p):
        plan.reset(keep_bitstrings=True)
        plan.run_halves(k0, k1, None, stream)
        plan.amplitudes_device(p, d_out.data_ptr(), d_sums.data_ptr(), stream)

    for _ in range(a.warmup):
        step(prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / a.steps
    value = m / (ms_per_step / 1000.0)

    # Per-kernel-family device time with HIP events on the launch stream, on a
    # plan that runs the halves one after the other: every kernel then runs
    # alone and its average launch time is its own (concurrent halves share
    # the GPU).  Same kernels and work as the timed region.
    tplan = Q.Plan(text, w.upper_mask, one_stream=True, **knobs)

    def tstep(p):
        tplan.reset(keep_bitstrings=True)
        tplan.run_halves(k0, k1, None, stream)
        tplan.amplitudes_device(p, d_out.data_ptr(), d_sums.data_ptr(), stream)

    tplan.run_halves(k0, k1, bits, stream)
    tplan.amplitudes_device(prec, d_out.data_ptr(), d_sums.data_ptr(), stream)
    for _ in range(a.warmup):
        tstep(prec)
    torch.cuda.synchronize()
    tplan.set_timing(2)
    ts0 = time.perf_counter()
    for _ in range(a.steps):
        tstep(prec)
    torch.cuda.synchronize()
    ms_one_stream = (time.perf_counter() - ts0) * 1000.0 / a.steps
    tm = tplan.timing()
    pass_table = per_pass_table(tplan.pass_timing())
    tplan.set_timing(False)
    tplan.close()
    fam_ms = {"pass": tm["pass_ms"], "tail": tm["tail_ms"], "gemm": tm["gemm_ms"], "other": tm["other_ms"]}
    per_step = {k: v / a.steps for k, v in fam_ms.items()}
    launches = {"pass": tm["pass_launches"] / a.steps, "tail": tm["tail_launches"] / a.steps,
                "gemm": tm["gemm_launches"] / a.steps, "other": tm["other_launches"] / a.steps}
    dominant = max(("pass", "tail", "gemm"), key=lambda k: fam_ms[k])
    roofs = {}
    # leaf evaluation: 2x2-gate rows on the vector units and per-value
    # contractions on FP32 MFMA; priced against the FP32 peak
    t = per_step["tail"] / 1000.0
    if t > 0:
        achieved = tm["tail_flops"] / a.steps / t / 1e12
        roofs["tail"] = {"kernel": "k_tail_ws+k_tail_fused", "bound": "alu", "achieved": round(achieved, 3),
                         "peak": 157.3, "unit": "TFLOP/s", "frac": round(achieved / 157.3, 4),
                         "traffic": _traffic_from_profile("k_tail_ws+k_tail_fused", w.name),
                         "note": "14 flops per amplitude per 2x2 gate on the light-cone rows, "
                                 "8 per complex multiply-add in the per-value contraction"}
    # layer and branch passes: algorithmic bytes = 8 B read + 8 B written per
    # amplitude of every state a pass reads or writes
    bytes_per_step = tm["pass_bytes"] / a.steps
    avg_launch_s = per_step["pass"] / 1000.0 / max(1.0, launches["pass"])
    per_launch = bytes_per_step / max(1.0, launches["pass"])
    achieved = per_launch / avg_launch_s / 1e9
    roofs["pass"] = {"kernel": "k_wpass+k_xpass", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": _traffic_from_profile("k_wpass+k_xpass", w.name),
                     "algorithmic_bytes_per_launch": per_launch, "avg_launch_us": avg_launch_s * 1e6}
    # assembly: executed MFMA flops (FP32: three real products per complex
    # one, 6 M N K; split-BF16: twelve BF16 products, 24 M N K) over the GEMM
    # and split-reduce time
    t = per_step["gemm"] / 1000.0
    cplx = tm["gemm_flops"] / a.steps          # 8 M N K, the complex-product count
    executed = cplx * (0.75 if prec == 0 else 3.0)
    peak = MFMA_PEAK_TFLOPS[prec]
    roofs["gemm"] = {"kernel": "k_zgemm_nt_f32d" if prec == 0 else "k_zgemm_nt_bf16x3", "bound": "mfma",
                     "achieved": round(executed / t / 1e12, 2), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(executed / t / 1e12 / peak, 4),
                     "traffic": _traffic_from_profile("k_zgemm_nt_f32d" if prec == 0 else "k_zgemm_nt_bf16x3",
                                                      w.name),
                     "complex_8mnk_tflops": round(cplx / t / 1e12, 2),
                     "note": "executed MFMA flops: 6 M N K (FP32, 3 real products) or 24 M N K (BF16)"}
    roof = roofs[dominant]

    # executed and flat (paper accounting) amp-updates
    oc_gates = [ln.split() for ln in text.splitlines() if ln and ln[0].isdigit()]
    n_u, n_l = plan.n_upper, plan.n_lower
    g_side = [0, 0]
    upper = w.upper_mask
    for g in oc_gates:
        qs = [int(x) for x in g[2:]]
        sides = {0 if (upper >> q) & 1 else 1 for q in qs}
        for s in sides:
            g_side[s] += 1
    flat_updates = (k1 - k0) * (g_side[0] * 2.0 ** n_u + g_side[1] * 2.0 ** n_l)
    amp_updates_per_s = flat_updates / (ms_per_step / 1000.0)
    ex = executed_updates(plan.dump(k0, k1), (len(np.unique(u_vals)), len(np.unique(l_vals))))

    out = {
        "metric": "output amplitudes/s and half-circuit amp-updates/s at 42q d20; HBM/MFMA %peak",
        "value": round(value, 1),
        "unit": "amplitudes/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.rows}x{w.cols} grid ({w.n} qubits), depth {w.depth}, seed "
                               f"{w.seed}; {n_u}+{n_l} halves, {c} cut CZ, copies [{k0}, {k1}); "
                               f"{w.n_u} x {w.n_l} product-set bitstrings",
                   "qubits": w.n, "depth": w.depth, "cuts": c, "copies": k1 - k0, "bitstrings": m,
                   "assembly": "fp32 mfma" if prec == 0 else "split-bf16 (3 products) mfma"},
        "amp_updates_per_s_flat": amp_updates_per_s,
        "amp_updates_flat_note": "the paper's Table 3 accounting (2^c copies times each half's gate "
                                 "count times 2^n_half), not work done: the copy tree, the light "
                                 "cone and the folded end cuts execute "
                                 "amp_updates_executed_per_step of them",
        "amp_updates_per_s_executed": ex["total"] / (ms_per_step / 1000.0),
        "amp_updates_executed_per_step": ex,
        "passes_per_s": launches["pass"] / (ms_per_step / 1000.0),
        "device_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "launches_per_step": launches,
        "setup_s": round(setup_s, 3),
        "roofline": roof,
        "roofline_by_family": roofs,
        "pass_launches": {"columns": ["half", "pass", "level_in", "stages", "tiles", "MB", "us", "GB/s", "passes"],
                          "rows": pass_table},
        "schedule": "halves on one stream" if a.one_stream else "halves on two streams, concurrent",
        "ms_per_step_one_stream_timed": round(ms_one_stream, 4),
        "knobs": knobs or "cost model defaults",
    }
    if tuned:
        out["autotune"] = {"best_ms": round(tuned["ms"], 3), "default_ms": round(tuned["default_ms"], 3),
                           "candidates": len(tuned["tried"])}
    elif knobs:
        out["knobs_source"] = "paper_1802_06952_amd/tuned.json (autotuner, same inputs)"

    # the same step as one HIP graph per step (qs_run_graph), on a stream of
    # its own (a graph cannot be captured on the null stream)
    gs = torch.cuda.Stream()
    plan.run_graph(k0, k1, prec, d_out.data_ptr(), d_sums.data_ptr(), gs)   # eager step + capture
    for _ in range(a.warmup):
        plan.run_graph(k0, k1, prec, d_out.data_ptr(), d_sums.data_ptr(), gs)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(a.steps):
        plan.run_graph(k0, k1, prec, d_out.data_ptr(), d_sums.data_ptr(), gs)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - tg0) * 1000.0 / a.steps
    out["graph"] = {"value": round(m / (gms / 1000.0), 1), "unit": "amplitudes/s",
                    "ms_per_step": round(gms, 4),
                    "note": "the same step captured once into a HIP graph by the library "
                            "(qs_run_graph) and replayed: one launch per step"}
    step(prec)
    torch.cuda.synchronize()

    # split-BF16 assembly on the same simulated halves
    if prec == 0:
        for _ in range(2):
            step(1)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for _ in range(a.steps):
            step(1)
        torch.cuda.synchronize()
        out["value_split_bf16"] = round(m / ((time.perf_counter() - tb0) / a.steps), 1)
        step(prec)
        torch.cuda.synchronize()

    # host-API rate: bitstrings from host memory, amplitudes back to host memory
    hp = Q.Plan(text, w.upper_mask, one_stream=a.one_stream)
    hp.run_halves(k0, k1, bits)
    hp.amplitudes(bits, prec)
    th0 = time.perf_counter()
    for _ in range(2):
        hp.reset(keep_bitstrings=False)
        hp.run_halves(k0, k1, bits)
        amp_h, _ = hp.amplitudes(bits, prec)
    out["host_api_value"] = round(m / ((time.perf_counter() - th0) / 2), 1)
    hp.close()

    # the same grid, depth, cut and bitstrings with every two-qubit gate drawn
    # from CZ, CNOT and CY and a random control (controlled-U cuts, Supp. Eq. 1)
    if not a.no_controlled and w.two_qubit == "cz":
        try:
            out["controlled_u"] = controlled_variant(Q, w, bits, prec, k0, k1, a, stream, d_out, d_sums)
        except Q.QSError as e:  # reported, not fatal: the CZ workload is the metric
            out["controlled_u"] = {"error": str(e)}
        # the checked output below is the CZ workload's
        step(prec)
        torch.cuda.synchronize()


    if not a.no_chain:
        try:
            out["chain_4part"] = chain_variant(Q, a, stream)
        except Q.QSError as e:  # reported, not fatal: the two-part workload is the metric
            out["chain_4part"] = {"error": str(e)}
        step(prec)
        torch.cuda.synchronize()

    if not a.no_configs and a.workload == "grid6x7_d20":
        from workloads import workload as _wl
        tk = tuned_knobs(Q, ("grid6x6_d16", "grid6x7_d20_cols", "grid6x6_d16_stair",
                             "grid8x8_d22_slice64"))
        # 36 qubits, 18+18 halves, all 4096 copies, 2^16 bitstrings: small enough that launch
        # latency, not bandwidth, sets its time
        r = time_workload(Q, _wl("grid6x6_d16"), 0, a.steps, a.warmup, stream, tk.get("grid6x6_d16"),
                          graph=True)
        r["knobs"] = tk.get("grid6x6_d16") or "cost model defaults"
        r.pop("amplitudes")
        r["workload"] = "grid6x6_d16: 6x6 grid (36 qubits), depth 16, rows 0-2 | 3-5, FP32 assembly"
        out["config2"] = r
        # the uneven pair, co-scheduled
        out["config4"] = coscheduled_pair(Q, ("grid6x7_d20_cols", "grid6x6_d16_stair"), 0, a.steps,
                                          a.warmup, tk)
        # one GPU's slice of the 64-qubit circuit (32+32 halves, copies [0, 64) of 65536)
        c5 = {}
        for p_, name in ((0, "fp32"), (1, "split_bf16")):
            # the plans take their memory budget from the free device memory:
            # hand back what the caching allocator holds from the runs before
            torch.cuda.empty_cache()
            r = time_workload(Q, _wl("grid8x8_d22_slice64"), p_, max(2, a.steps // 5), 1, stream,
                              tk.get("grid8x8_d22_slice64"))
            r.pop("amplitudes")
            c5[name] = r
        c5["knobs"] = tk.get("grid8x8_d22_slice64") or "cost model defaults"
        c5["workload"] = ("grid8x8_d22_slice64: 8x8 grid (64 qubits), depth 22, rows 0-3 | 4-7, "
                          "copies [0, 64) of 65536, 1024 x 1024 bitstrings, partial amplitudes")
        out["config5"] = c5
        torch.cuda.empty_cache()
        step(prec)
        torch.cuda.synchronize()

    if not a.no_check:
        gpath = os.path.join(ROOT, "tests", "golden", f"{w.name}.npz")
        sums = d_sums.cpu().numpy()
        out["stats"] = {"sum_p": float(sums[0]), "2^n mean p": float(np.ldexp(sums[0] / m, w.n)),
                        "2^2n mean p^2": float(np.ldexp(sums[1] / m, 2 * w.n))}
        if os.path.exists(gpath):
            g = np.load(gpath)
            nu, nl = len(g["u"]), len(g["l"])
            chk = {"subset": f"first {nu} upper x first {nl} lower values", "reference": "FP64 oracle"}
            for p_, name in ((0, "fp32"), (1, "split_bf16")):
                step(p_)
                torch.cuda.synchronize()
                amp = d_out.cpu().numpy().view(np.complex64).reshape(w.n_u, w.n_l)
                chk[name] = error_stats(amp[:nu, :nl], g["amp"])
            out["check"] = chk
        step(prec)
        torch.cuda.synchronize()

    if not a.no_plain:
        pc = min(a.plain_copies, k1 - k0)
        pp = Q.Plan(text, w.upper_mask, plain=True)
        pp.run_halves(k0, k0 + pc, bits)
        torch.cuda.synchronize()
        pp.reset(keep_bitstrings=True)
        tp0 = time.perf_counter()
        pp.run_halves(k0, k0 + pc, None, stream)
        pp.amplitudes_device(0, d_out.data_ptr(), d_sums.data_ptr(), stream)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        scaled = tp * (k1 - k0) / pc
        out["plain_fp32"] = {"value": round(m / scaled, 2), "unit": "amplitudes/s",
                             "sample": f"flat per-copy form (no shared prefix, one gate per pass, "
                                       f"full leaf states) on {pc} of {k1 - k0} copies: {tp:.3f} s, "
                                       f"extrapolated linearly"}
        pp.close()

    if a.calib_copy_gib > 0:
        nbytes = int(a.calib_copy_gib * (1 << 30))
        x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nbytes
        del x, y

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_copies, 64, min(a.cpu_workers, os.cpu_count() or 1))

    plan.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
