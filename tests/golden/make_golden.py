"""Write oracle amplitudes for the larger workloads into tests/golden/.

Calls only ``oracle`` (FP64) and ``workloads`` (seeded inputs).  Usage::

    python tests/golden/make_golden.py grid6x6_d16 [--workers 4] [--threads 2]
    python tests/golden/make_golden.py grid6x7_d20 --nu 64 --nl 64

For each workload the file ``<name>.npz`` holds the upper and lower half
values (``u``, ``l``: packed half indices), the copy range, and ``amp``, the
FP64 amplitudes of the product set (row-major over u then l).  ``--nu`` /
``--nl`` keep only the first values of the workload's bitstring draw.
"""

from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _part(args):
    name, lo, hi, u, l, threads, cache = args
    if cache:
        path = os.path.join(cache, f"{name}_{lo}_{hi}_{len(u)}_{len(l)}.npz")
        if os.path.exists(path):
            d = np.load(path)
            return lo, d["A"], d["B"]
    import torch
    torch.set_num_threads(threads)
    from oracle import circuit as OC, partition as P
    from workloads import workload
    w = workload(name)
    c = OC.parse(w.circuit_text())
    A, B = P.gathered_halves(c, w.upper_mask, u, l, lo, hi)
    if cache:
        np.savez(path + ".tmp.npz", A=A, B=B)
        os.replace(path + ".tmp.npz", path)
    return lo, A, B


def make(name: str, nu: int | None, nl: int | None, workers: int, threads: int, parts: int,
         cache: str | None = None) -> str:
    from oracle import circuit as OC, partition as P
    from workloads import workload, product_bitstrings
    w = workload(name)
    c = OC.parse(w.circuit_text())
    ncut = len(P.find_cuts(c, w.upper_mask))
    k0 = w.copy_begin
    k1 = w.copy_end if w.copy_end is not None else (1 << ncut)
    _, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    u = u[: nu or len(u)].astype(np.int64)
    l = l[: nl or len(l)].astype(np.int64)
    step = max(1, (k1 - k0) // parts)
    if cache:
        os.makedirs(cache, exist_ok=True)
    jobs = [(name, a, min(a + step, k1), u, l, threads, cache) for a in range(k0, k1, step)]
    t0 = time.time()
    A = np.zeros((len(u), k1 - k0), dtype=np.complex128)
    B = np.zeros((len(l), k1 - k0), dtype=np.complex128)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for lo, a, b in ex.map(_part, jobs):
            A[:, lo - k0: lo - k0 + a.shape[1]] = a
            B[:, lo - k0: lo - k0 + b.shape[1]] = b
            print(f"  copies from {lo}: done ({time.time() - t0:.0f} s)", flush=True)
    amp = (A @ B.T).reshape(-1)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, u=u, l=l, copy_begin=k0, copy_end=k1, amp=amp,
                        upper_mask=np.uint64(w.upper_mask))
    print(f"wrote {path}: {len(u)} x {len(l)} amplitudes, copies [{k0}, {k1}), "
          f"{time.time() - t0:.0f} s", flush=True)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--nu", type=int, default=None)
    ap.add_argument("--nl", type=int, default=None)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--threads", type=int, default=2)
    ap.add_argument("--parts", type=int, default=64)
    ap.add_argument("--cache", default=None, help="directory for per-part results (resumable runs)")
    a = ap.parse_args()
    make(a.name, a.nu, a.nl, a.workers, a.threads, a.parts, a.cache)


if __name__ == "__main__":
    main()
