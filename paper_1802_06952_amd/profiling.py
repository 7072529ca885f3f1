"""Summaries of rocprofv3 output databases (kernel traces and PMC counters).

rocprofv3 writes one SQLite database per run.  Two summaries are made here:

* ``trace``: per-kernel call count, total and average duration from a
  ``--kernel-trace --stats`` run, plus each kernel's register and LDS use;
* ``sq``: per-kernel MFMA utilisation and instruction counts from one ``--pmc``
  run of SQ and GRBM counters;
* ``launches``: one step dispatch by dispatch, durations from a trace run and
  instruction counts from a ``--pmc`` run of the same command;
* ``counters``: HBM bytes per dispatch of one kernel family from two ``--pmc``
  runs (``FETCH_SIZE``, then ``WRITE_SIZE``, both in KiB per dispatch).  Each
  counter is divided by what it reads for a plain copy of known size made in
  the same run (the largest copy-like dispatch), which turns it into bytes.

Usage::

    python -m paper_1802_06952_amd.profiling trace DIR --cmd "..." > summary.md
    python -m paper_1802_06952_amd.profiling counters FETCH_DIR WRITE_DIR \\
        --kernel k_wpass --workload grid6x7_d20 --calib-bytes N --cmd "..."
"""

from __future__ import annotations

import argparse
import collections
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _db(d: str) -> sqlite3.Connection:
    files = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))
    if not files:
        raise SystemExit(f"no rocprofv3 database under {d}")
    return sqlite3.connect(files[0])


def short_name(n: str) -> str:
    n = re.sub(r"\(.*", "", n).replace("void ", "")
    return n


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_1802_06952_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def trace_summary(d: str, cmd: str) -> str:
    con = _db(d)
    out = [f"Command: `{cmd}`", "",
           "rocprofv3 `--kernel-trace --stats` summary (durations in microseconds, all dispatches "
           "of the run).", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, c, t, a, p in con.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        out.append(f"| `{short_name(n)}` | {c} | {t:.1f} | {a:.2f} | {p:.1f} |")
    out += ["", "Resources per kernel:", "", "| kernel | vgpr | agpr | sgpr | lds | scratch |",
            "|---|---|---|---|---|---|"]
    for n, v, acc, sg, lds, scr in con.execute(
            "select name, vgpr_count, accum_vgpr_count, sgpr_count, lds_size, scratch_size "
            "from kernels group by name"):
        out.append(f"| `{short_name(n)}` | {v} | {acc} | {sg} | {lds} | {scr} |")
    out.append("")
    out.append(f"kernels.hip sha256[:16] = {kernel_source_hash()}")
    return "\n".join(out) + "\n"


def _pmc(d: str):
    con = _db(d)
    vals = collections.defaultdict(dict)
    names = {}
    for disp, kname, cname, val in con.execute(
            "select dispatch_id, name, counter_name, counter_value from pmc_events"):
        vals[disp][cname] = vals[disp].get(cname, 0.0) + float(val)
        names[disp] = short_name(kname)
    return vals, names


def _is_copy(name: str) -> bool:
    return "copy" in name.lower() or "elementwise" in name.lower()


def _in_family(name: str, kernels) -> bool:
    """Whether a dispatch name (``qs::k_x<...>``) is one of the kernels named."""
    return name.split("<")[0] in {f"qs::{k}" for k in kernels}


def counter_summary(fetch_dir: str, write_dir: str, kernel: str, calib_bytes: int) -> dict:
    """HBM bytes per dispatch of a kernel family; ``kernel`` names one kernel
    or several joined by ``+`` (their dispatches are averaged together)."""
    ks = kernel.split("+")
    f, fn = _pmc(fetch_dir)
    w, wn = _pmc(write_dir)

    def calib(vals, names, counter):
        cand = [vals[k].get(counter, 0.0) for k in vals if _is_copy(names[k])]
        if not cand:
            raise SystemExit("no copy dispatch found for calibration")
        return max(cand) * 1024.0 / calib_bytes   # counter KiB -> bytes, over the true bytes

    cf = calib(f, fn, "FETCH_SIZE")
    cw = calib(w, wn, "WRITE_SIZE")
    fk = [f[k].get("FETCH_SIZE", 0.0) for k in f if _in_family(fn[k], ks)]
    wk = [w[k].get("WRITE_SIZE", 0.0) for k in w if _in_family(wn[k], ks)]
    if not fk or not wk:
        raise SystemExit(f"no dispatch of {kernel}")
    fetch = sum(fk) / len(fk) * 1024.0 / cf
    write = sum(wk) / len(wk) * 1024.0 / cw
    return {"kernel": kernel, "dispatches": len(fk),
            "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "hbm_bytes_per_launch": fetch + write,
            "calibration": {"copy_bytes": calib_bytes, "fetch_factor": cf, "write_factor": cw,
                            "note": "counter bytes read for a plain copy of copy_bytes, divided "
                                    "by copy_bytes; kernel counters are divided by it"},
            "kernels_hip_sha256_16": kernel_source_hash()}


def sq_summary(d: str, cmd: str, simds: int = 1024, xcds: int = 8) -> str:
    """Per-kernel averages of SQ/GRBM counters from one --pmc run: MFMA busy
    cycles against the dispatch's GPU cycles times the SIMD count (MFMA
    utilisation; GRBM_GUI_ACTIVE comes summed over the XCDs, each with its own
    GRBM), MFMA flops (each MOPS unit is 512 flops), and the VALU, SALU and
    LDS instruction counts per dispatch."""
    vals, names = _pmc(d)
    per = collections.defaultdict(list)
    for disp, cs in vals.items():
        per[names[disp]].append(cs)
    cols = ["SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_F32",
            "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
            "SQ_WAVES"]
    out = [f"Command: `{cmd}`", "",
           "rocprofv3 `--pmc` counters, averaged over the dispatches of each kernel. MFMA "
           f"utilisation = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {xcds} XCDs x {simds} "
           "SIMDs); MFMA GFLOP = (MOPS_F32 + MOPS_BF16) x 512 / 1e9.", "",
           "| kernel | dispatches | MFMA util | MFMA GFLOP (F32) | MFMA GFLOP (BF16) | VALU insts | "
           "SALU insts | LDS insts | waves |", "|---|---|---|---|---|---|---|---|---|"]
    for n in sorted(per, key=lambda k: -sum(x.get("GRBM_GUI_ACTIVE", 0) for x in per[k])):
        rows = per[n]
        avg = {c: sum(r.get(c, 0.0) for r in rows) / len(rows) for c in cols}
        util = avg["SQ_VALU_MFMA_BUSY_CYCLES"] / max(1.0, avg["GRBM_GUI_ACTIVE"] / xcds * simds)
        out.append(f"| `{n}` | {len(rows)} | {100 * util:.1f} % | "
                   f"{avg['SQ_INSTS_VALU_MFMA_MOPS_F32'] * 512 / 1e9:.2f} | "
                   f"{avg['SQ_INSTS_VALU_MFMA_MOPS_BF16'] * 512 / 1e9:.2f} | "
                   f"{avg['SQ_INSTS_VALU']:.3g} | {avg['SQ_INSTS_SALU']:.3g} | "
                   f"{avg['SQ_INSTS_LDS']:.3g} | {avg['SQ_WAVES']:.0f} |")
    out.append("")
    out.append(f"kernels.hip sha256[:16] = {kernel_source_hash()}")
    return "\n".join(out) + "\n"


def _dispatches(d: str):
    """(name, microseconds) of every dispatch of a --kernel-trace run, in start order."""
    con = _db(d)
    return [(short_name(n), (e - b) / 1e3)
            for n, b, e in con.execute("select name, start, end from kernels order by start")]


def _last_step(seq, name_of):
    """The dispatches of the last complete step with inputs already on the
    device: a step ends with k_prob_final, and of all steps the ones with the
    fewest copies are those (a step that uploads bitstrings copies more)."""
    idx = [i for i, x in enumerate(seq) if "k_prob_final" in name_of(x)]
    steps = [seq[a + 1: b + 1] for a, b in zip(idx, idx[1:])]
    if not steps:
        raise SystemExit("fewer than two steps in the run")
    copies = [sum("copyBuffer" in name_of(x) for x in st) for st in steps]
    return [st for st, c in zip(steps, copies) if c == min(copies)][-1]


def launch_table(trace_dir: str, pmc_dir: str, cmd: str, clock_ghz: float = 2.4,
                 simds: int = 1024) -> str:
    """Every dispatch of one step: duration (from the trace run) and VALU, SALU
    and LDS instruction counts (from the --pmc run of the same command).  The
    VALU column is the share of the chip's VALU issue rate the dispatch used:
    one wave64 instruction per SIMD every 4 cycles."""
    vals, names = _pmc(pmc_dir)
    P = _last_step([(names[k], vals[k]) for k in sorted(vals)], lambda x: x[0])
    T = _last_step(_dispatches(trace_dir), lambda x: x[0])
    if len(P) != len(T) or any(a[0] != b[0] for a, b in zip(P, T)):
        raise SystemExit("the two runs dispatched different kernels")
    out = [f"Command: `{cmd}`", "",
           "One step, dispatch by dispatch: duration from the `--kernel-trace` run; instruction "
           "counts from the `--pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS ...` run of the same "
           f"command. VALU % = SQ_INSTS_VALU x 4 cycles / ({simds} SIMDs x duration x "
           f"{clock_ghz} GHz).", "",
           "| # | kernel | us | VALU insts | VALU % | SALU insts | LDS insts |",
           "|---|---|---|---|---|---|---|"]
    for i, ((n, c), (_, us)) in enumerate(zip(P, T)):
        valu = c.get("SQ_INSTS_VALU", 0.0)
        frac = valu * 4 / simds / (us * 1e-6 * clock_ghz * 1e9) if us > 0 else 0.0
        out.append(f"| {i} | `{n}` | {us:.2f} | {valu:.3g} | {100 * frac:.1f} | "
                   f"{c.get('SQ_INSTS_SALU', 0.0):.3g} | {c.get('SQ_INSTS_LDS', 0.0):.3g} |")
    out.append("")
    out.append(f"kernels.hip sha256[:16] = {kernel_source_hash()}")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--calib-bytes", type=int, required=True)
    c.add_argument("--cmd", required=True)
    q = sub.add_parser("sq")
    q.add_argument("dir")
    q.add_argument("--cmd", required=True)
    lt = sub.add_parser("launches")
    lt.add_argument("trace_dir")
    lt.add_argument("pmc_dir")
    lt.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.what == "trace":
        sys.stdout.write(trace_summary(a.dir, a.cmd))
    elif a.what == "sq":
        sys.stdout.write(sq_summary(a.dir, a.cmd))
    elif a.what == "launches":
        sys.stdout.write(launch_table(a.trace_dir, a.pmc_dir, a.cmd))
    else:
        d = counter_summary(a.fetch_dir, a.write_dir, a.kernel, a.calib_bytes)
        d["workload"] = a.workload
        d["command"] = a.cmd
        json.dump(d, sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()
