"""Write oracle amplitudes for the larger workloads into tests/golden/.

Calls only ``oracle`` (FP64) and ``workloads`` (seeded inputs).  Usage::

    python tests/golden/make_golden.py grid6x6_d16 [--workers 4] [--threads 2]
    python tests/golden/make_golden.py grid6x7_d20 --nu 64 --nl 64
    python tests/golden/make_golden.py grid8x8_d22_bands --bands

For each workload the file ``<name>.npz`` holds the upper and lower half
values (``u``, ``l``: packed half indices), the copy range, and ``amp``, the
FP64 amplitudes of the product set (row-major over u then l).  ``--nu`` /
``--nl`` keep only the first values of the workload's bitstring draw.

``--bands`` (a circuit of independent row bands, one of them holding every cut
gate): the file holds the factors ``fu``, ``A``, ``B``, ``fl`` of
``band_factors`` instead, and the amplitudes are
``fu[:, None] * (A @ B.T) * fl[None, :]``.
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


def independent_blocks(circ):
    """Qubit sets of the circuit's independent blocks: the connected components
    of the graph whose edges are the two-qubit gates (a block's state is a
    tensor factor of the whole state at every layer)."""
    parent = list(range(circ.n))

    def find(q):
        while parent[q] != q:
            parent[q] = parent[parent[q]]
            q = parent[q]
        return q

    for _, _, qs in circ.gates:
        if len(qs) == 2:
            parent[find(qs[0])] = find(qs[1])
    blocks: dict[int, list[int]] = {}
    for q in range(circ.n):
        blocks.setdefault(find(q), []).append(q)
    return sorted(blocks.values())


def restrict(circ, qubits):
    """The gates of ``circ`` on ``qubits`` (all of them inside the set),
    relabelled to 0..len-1 in ascending order."""
    from oracle.circuit import Circuit
    loc = {q: i for i, q in enumerate(sorted(qubits))}
    gates = [(t, name, tuple(loc[q] for q in qs)) for t, name, qs in circ.gates
             if all(q in loc for q in qs)]
    return Circuit(len(loc), gates)


def band_factors(text: str, upper_mask: int, u_values, l_values, copy_begin: int, copy_end: int):
    """Partial amplitudes of a copy slice for a circuit made of independent
    blocks, exactly one of which holds cut gates.

    The whole state is the tensor product of the blocks' states, so a copy's
    upper half state is the cut block's upper half state of that copy times
    the states of the blocks that lie wholly in the upper half (and likewise
    for the lower half), and the slice's partial amplitude at (u, l) is
      fu[u] * sum_k U'_k[u'] L'_k[l'] * fl[l],
    with U', L' the cut block's halves (oracle partition over the same copy
    range: relabelling the qubits in ascending order keeps the cut order) and
    fu, fl the products of the other blocks' amplitudes (oracle state
    vectors).  Returns (fu, A, B, fl) with A[i, k] = U'_k, B[j, k] = L'_k."""
    from oracle import circuit as OC, partition as P, statevector as SV
    circ = OC.parse(text)
    n = circ.n
    full = (1 << n) - 1
    uq = P.half_qubits(n, upper_mask)
    lq = P.half_qubits(n, full & ~upper_mask)
    u_values = np.asarray(u_values, dtype=np.int64)
    l_values = np.asarray(l_values, dtype=np.int64)

    def pack(values, half, qubits):
        pos = {q: i for i, q in enumerate(half)}
        out = np.zeros(values.shape, dtype=np.int64)
        for j, q in enumerate(sorted(qubits)):
            out |= ((values >> pos[q]) & 1) << j
        return out

    cut_blocks = []
    fu = np.ones(len(u_values), dtype=np.complex128)
    fl = np.ones(len(l_values), dtype=np.complex128)
    for blk in independent_blocks(circ):
        inside = [(upper_mask >> q) & 1 for q in blk]
        if all(inside) or not any(inside):
            psi = SV.simulate(restrict(circ, blk))
            if all(inside):
                fu *= psi[pack(u_values, uq, blk)]
            else:
                fl *= psi[pack(l_values, lq, blk)]
        else:
            cut_blocks.append(blk)
    if len(cut_blocks) != 1:
        raise ValueError("exactly one block may hold cut gates")
    blk = cut_blocks[0]
    sub = restrict(circ, blk)
    sub_mask = sum(1 << i for i, q in enumerate(sorted(blk)) if (upper_mask >> q) & 1)
    bu = [q for q in blk if (upper_mask >> q) & 1]
    bl = [q for q in blk if not (upper_mask >> q) & 1]
    A, B = P.gathered_halves(sub, sub_mask, pack(u_values, uq, bu), pack(l_values, lq, bl),
                             copy_begin, copy_end)
    return fu, A, B, fl


def make_bands(name: str) -> str:
    """Golden factors of a workload made of independent row bands."""
    from workloads import workload, product_bitstrings
    w = workload(name)
    _, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    t0 = time.time()
    fu, A, B, fl = band_factors(w.circuit_text(), w.upper_mask, u, l, w.copy_begin, w.copy_end)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, u=u.astype(np.int64), l=l.astype(np.int64), copy_begin=w.copy_begin,
                        copy_end=w.copy_end, fu=fu, A=A, B=B, fl=fl,
                        upper_mask=np.uint64(w.upper_mask))
    print(f"wrote {path}: factors of {len(u)} x {len(l)} amplitudes, copies "
          f"[{w.copy_begin}, {w.copy_end}), {time.time() - t0:.0f} s", flush=True)
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
    ap.add_argument("--bands", action="store_true",
                    help="the workload is made of independent row bands: store the factors "
                         "(band_factors) instead of the amplitudes")
    a = ap.parse_args()
    if a.bands:
        make_bands(a.name)
    else:
        make(a.name, a.nu, a.nl, a.workers, a.threads, a.parts, a.cache)


if __name__ == "__main__":
    main()
