"""Partitions into t parts (Sec. 3, Fig. 3), in complex128.

Test infrastructure: only the tests, the golden-value script and the
benchmark's CPU baseline use this module; the HIP library never does.

The qubits are split into t parts.  Every two-qubit gate with its endpoints
in two parts is a cut gate and is rewritten by Eq. (1): a sum over b of a
factor on each endpoint.  With c cut gates the circuit is the sum of 2^c
copies, each the tensor product of t part circuits, and the amplitude of a
bitstring is the sum over copies of the product of the t part amplitudes
(the two-part scheme of Sec. 2.1 with t factors instead of two).

Readings where the paper is silent (it only shows the schemes, Fig. 3):

* the parts form a chain: every cut gate joins parts i and i+1 (row bands of
  a grid do);
* cut j is the j-th cut gate ordered by (layer, endpoint in the lower-numbered
  part); copy k carries bit s_j = (k >> (c-1-j)) & 1;
* a cut CZ puts P_b on its endpoint in the even-numbered part and Z^b on the
  one in the odd-numbered part (CZ is symmetric, Eq. 1 holds either way; for
  two parts this is the upper/lower rule of the two-part scheme); a cut
  controlled-U (cx, cy) follows Supp. Eq. 1: P_b on the control, U^b on the
  target;
* part p sees only the cuts that touch it, numbered in cut order; its copy
  index has their bits, the first the most significant.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .circuit import Circuit
from .partition import half_qubits, pack_bits, tree_states


@dataclass(frozen=True)
class PartCut:
    index: int      # position in cut order
    cycle: int
    lo_part: int    # the two parts it joins (hi_part = lo_part + 1)
    q_lo: int       # endpoint in lo_part
    q_hi: int       # endpoint in hi_part
    gate: str
    control: int    # -1 for cz


def part_of(n: int, part_masks) -> list[int]:
    owner = [-1] * n
    for p, m in enumerate(part_masks):
        for q in half_qubits(n, m):
            if owner[q] >= 0:
                raise ValueError("parts overlap")
            owner[q] = p
    if min(owner) < 0:
        raise ValueError("parts do not cover every qubit")
    if any(m == 0 for m in part_masks):
        raise ValueError("empty part")
    return owner


def chain_cuts(circ: Circuit, part_masks) -> list[PartCut]:
    owner = part_of(circ.n, part_masks)
    raw = []
    for t, name, qs in circ.gates:
        if len(qs) != 2 or owner[qs[0]] == owner[qs[1]]:
            continue
        a, b = qs
        if owner[a] > owner[b]:
            a, b = b, a
        if owner[b] != owner[a] + 1:
            raise ValueError("the parts do not form a chain: a cut gate joins parts "
                             f"{owner[a]} and {owner[b]}")
        raw.append((t, a, owner[a], b, name, -1 if name == "cz" else qs[0]))
    raw.sort()
    return [PartCut(j, t, pa, a, b, name, ctl) for j, (t, a, pa, b, name, ctl) in enumerate(raw)]


def part_cuts(cuts, p: int) -> list[PartCut]:
    """The cut gates touching part p, in cut order."""
    return [k for k in cuts if p in (k.lo_part, k.lo_part + 1)]


def part_factor(cut: PartCut, p: int, b: int) -> str:
    q = cut.q_lo if p == cut.lo_part else cut.q_hi
    if cut.gate == "cz":
        return ("p1" if b else "p0") if p % 2 == 0 else ("z" if b else "i")
    if q == cut.control:
        return "p1" if b else "p0"
    return {"cx": "x", "cy": "y"}[cut.gate] if b else "i"


def part_program(circ: Circuit, part_masks, p: int):
    """(n_p, ops, local cuts): ops as (cycle, name, local qubits, local cut or None)."""
    cuts = chain_cuts(circ, part_masks)
    mine = part_cuts(cuts, p)
    qs = half_qubits(circ.n, part_masks[p])
    loc = {q: i for i, q in enumerate(qs)}
    local = {(k.cycle, k.q_lo if p == k.lo_part else k.q_hi): i for i, k in enumerate(mine)}
    prog = []
    for t, name, gq in circ.gates:
        inside = [q for q in gq if q in loc]
        if not inside:
            continue
        if len(gq) == 2 and len(inside) == 1:
            prog.append((t, "cut", (loc[inside[0]],), local[(t, inside[0])]))
        else:
            prog.append((t, name, tuple(loc[q] for q in gq), None))
    return len(qs), prog, mine


def part_states(circ: Circuit, part_masks, p: int, select=None) -> np.ndarray:
    """Part p's amplitudes at the local indices ``select`` for every local copy:
    shape (len(select), 2^c_p), column = local copy index."""
    nloc, prog, mine = part_program(circ, part_masks, p)
    return tree_states(nloc, prog, len(mine), lambda j, b: part_factor(mine[j], p, b), select)


def amplitudes(circ: Circuit, part_masks, bitstrings, chunk: int | None = None) -> np.ndarray:
    """amp(x) = sum over the 2^c copies k of prod_p X_p[x_p, k restricted to p]."""
    cuts = chain_cuts(circ, part_masks)
    c = len(cuts)
    t = len(part_masks)
    bits = np.asarray(bitstrings, dtype=np.uint64)
    amp = np.zeros(bits.shape, dtype=np.complex128)
    vals, states, glob = [], [], []
    for p in range(t):
        v = pack_bits(bits, half_qubits(circ.n, part_masks[p]))
        uv, inv = np.unique(v, return_inverse=True)
        vals.append(inv)
        states.append(part_states(circ, part_masks, p, uv))
        glob.append([k.index for k in part_cuts(cuts, p)])
    if chunk is None:
        chunk = max(1, (1 << 22) // max(1, bits.size))  # about 64 MB per product block
    for k0 in range(0, 1 << c, chunk):
        ks = np.arange(k0, min(k0 + chunk, 1 << c), dtype=np.int64)
        prod = np.ones((bits.size, ks.size), dtype=np.complex128)
        for p in range(t):
            cp = len(glob[p])
            local = np.zeros(ks.size, dtype=np.int64)
            for i, j in enumerate(glob[p]):
                local |= ((ks >> (c - 1 - j)) & 1) << (cp - 1 - i)
            prod *= states[p][vals[p]][:, local]
        amp += prod.sum(axis=1)
    return amp
