"""The partition scheme in complex128 (Sec. 2.1; Sec. 2.3.1-2.3.2; Supp. A, Eq. 1-8).

Steps, in the paper's order:

1. Split the qubits into an upper set V1 and a lower set V2 (Supp. A, the
   division of V_t into V_{1,t} and V_{2,t}).  The two-qubit gates with one
   end in each set form E_int (the cut gates); the others stay inside a half.
2. Rewrite every cut CZ as P0 x I + P1 x Z (Eq. 1 / Supp. Eq. 2): P_b goes on
   the upper endpoint and Z^b on the lower endpoint.  A cut controlled-U with
   U = X or Y ("cx", "cy") is rewritten by Supp. Eq. 1: P_b on the control,
   U^b on the target, whichever half each is in.  With c cut gates the
   circuit becomes the sum of 2^c copies, each the tensor product of an upper
   and a lower half circuit (Supp. Eq. 7-8).
3. Simulate every copy's two halves from H on |0...0>.  States shared by
   copies up to a cut layer are computed once: a depth-first recursion over
   the cut layers, the plain form of the prefix reuse of Sec. 2.3.2.
4. The output amplitude of bitstring x is the sum over copies of the upper
   amplitude at the upper bits of x times the lower amplitude at the lower
   bits of x (Sec. 2.3.1: sample, take the tensor product, add).

Readings taken where the paper is silent: cut j is the j-th cut gate ordered
by (layer, upper endpoint id); copy k carries bit s_j = (k >> (c-1-j)) & 1,
so the earliest cut is the most significant bit; inside a half the qubits are
numbered in ascending global id (bit i of a half index is the i-th qubit of
the half).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import statevector as SV
from .circuit import Circuit


@dataclass(frozen=True)
class Cut:
    index: int
    cycle: int
    upper: int
    lower: int
    gate: str = "cz"   # the cut two-qubit gate
    control: int = -1  # its control qubit (cx, cy); -1 for cz


def half_qubits(n: int, mask: int) -> list[int]:
    return [q for q in range(n) if (mask >> q) & 1]


def find_cuts(circ: Circuit, upper_mask: int) -> list[Cut]:
    """The two-qubit gates of E_int (one endpoint in each half), in cut order."""
    raw = []
    for t, name, qs in circ.gates:
        if len(qs) != 2:
            continue
        a, b = qs
        ia, ib = (upper_mask >> a) & 1, (upper_mask >> b) & 1
        if ia != ib:
            up, lo = (a, b) if ia else (b, a)
            raw.append((t, up, lo, name, -1 if name == "cz" else a))
    raw.sort()
    return [Cut(j, *r) for j, r in enumerate(raw)]


def cut_factor(cut: Cut, upper: bool, b: int) -> str:
    """The one-qubit factor of copy bit b that cut gate ``cut`` puts on the
    endpoint in the given half: Eq. 1 (CZ: P_b upper, Z^b lower) or Supp. Eq. 1
    (controlled-U: P_b on the control, U^b on the target)."""
    if cut.gate == "cz":
        return ("p1" if b else "p0") if upper else ("z" if b else "i")
    on_control = (cut.upper if upper else cut.lower) == cut.control
    if on_control:
        return "p1" if b else "p0"
    return {"cx": "x", "cy": "y"}[cut.gate] if b else "i"


def copy_bit(k: int, j: int, c: int) -> int:
    return (k >> (c - 1 - j)) & 1


def half_program(circ: Circuit, upper_mask: int, upper: bool):
    """Ops of one half as (cycle, name, local qubits, cut index or None).

    Cut gates appear as ``cut`` ops on the half's endpoint; once the copy
    fixes b they become the factor ``cut_factor`` names (P_b, Z^b or U^b).
    """
    n = circ.n
    full = (1 << n) - 1
    mask = upper_mask if upper else (full & ~upper_mask)
    qs = half_qubits(n, mask)
    loc = {q: i for i, q in enumerate(qs)}
    cuts = find_cuts(circ, upper_mask)
    cut_of = {(c.cycle, c.upper if upper else c.lower): c.index for c in cuts}
    prog = []
    for t, name, gq in circ.gates:
        inside = [q for q in gq if q in loc]
        if not inside:
            continue
        if len(gq) == 2 and len(inside) == 1:
            prog.append((t, "cut", (loc[inside[0]],), cut_of[(t, inside[0])]))
        else:
            prog.append((t, name, tuple(loc[q] for q in gq), None))
    return len(qs), prog


def _apply_op(psi, op, bits: dict, factor) -> None:
    """Apply one program op; ``factor(j, b)`` names cut j's factor for bit b."""
    t, name, lq, j = op
    if name == "cut":
        SV.apply_gate(psi, factor(j, bits[j]), lq)
    else:
        SV.apply_gate(psi, name, lq)


def half_state_plain(circ: Circuit, upper_mask: int, upper: bool, k: int) -> np.ndarray:
    """One copy's half state, simulated from scratch (no prefix reuse)."""
    nloc, prog = half_program(circ, upper_mask, upper)
    cuts = find_cuts(circ, upper_mask)
    c = len(cuts)
    bits = {j: copy_bit(k, j, c) for j in range(c)}
    psi = SV.zero_state(nloc)
    for op in prog:
        _apply_op(psi, op, bits, lambda j, b: cut_factor(cuts[j], upper, b))
    return psi


def half_states(circ: Circuit, upper_mask: int, upper: bool, select=None,
                copy_begin: int = 0, copy_end: int | None = None) -> np.ndarray:
    """Gathered half amplitudes of every copy in [copy_begin, copy_end).

    Returns an array of shape (len(select), copy_end - copy_begin) whose column
    k - copy_begin holds the half state of copy k at the local indices in
    ``select`` (all 2^n_half indices when ``select`` is None).  Copies share
    their state up to each cut layer: the recursion branches at a layer that
    holds cuts into one child per assignment of that layer's cut bits.
    """
    nloc, prog = half_program(circ, upper_mask, upper)
    cuts = find_cuts(circ, upper_mask)
    return tree_states(nloc, prog, len(cuts), lambda j, b: cut_factor(cuts[j], upper, b),
                       select, copy_begin, copy_end)


def tree_states(nloc: int, prog, c: int, factor, select=None, copy_begin: int = 0,
                copy_end: int | None = None) -> np.ndarray:
    """The prefix-reuse recursion of Sec. 2.3.2 over a program with c cut ops
    (cut j's factor for bit b is ``factor(j, b)``); columns are copies
    k = sum_j b_j 2^(c-1-j) in [copy_begin, copy_end)."""
    total = 1 << c
    if copy_end is None:
        copy_end = total
    if not (0 <= copy_begin <= copy_end <= total):
        raise ValueError("bad copy range")
    sel = np.arange(1 << nloc) if select is None else np.asarray(select, dtype=np.int64)
    out = np.zeros((len(sel), copy_end - copy_begin), dtype=np.complex128)
    cycles = sorted({op[0] for op in prog})
    by_cycle = {t: [op for op in prog if op[0] == t] for t in cycles}

    def rec(psi, ci, bits, nassigned):
        # the copies under this node: the first nassigned cut bits are fixed
        prefix = 0
        for j in range(nassigned):
            prefix = (prefix << 1) | bits[j]
        lo = prefix << (c - nassigned)
        hi = (prefix + 1) << (c - nassigned)
        if hi <= copy_begin or lo >= copy_end:
            return
        while ci < len(cycles):
            ops = by_cycle[cycles[ci]]
            cut_js = sorted(op[3] for op in ops if op[1] == "cut")
            if cut_js:
                m = len(cut_js)
                for b in range(1 << m):
                    child_bits = dict(bits)
                    for pos, j in enumerate(cut_js):
                        child_bits[j] = (b >> (m - 1 - pos)) & 1
                    child = psi.copy()
                    for op in ops:
                        _apply_op(child, op, child_bits, factor)
                    rec(child, ci + 1, child_bits, nassigned + m)
                return
            for op in ops:
                _apply_op(psi, op, bits, factor)
            ci += 1
        k = lo
        out[:, k - copy_begin] = psi[sel]

    rec(SV.zero_state(nloc), 0, {}, 0)
    return out


def pack_bits(bitstrings, qubits) -> np.ndarray:
    """Half index of each bitstring: bit i is the value of qubits[i]."""
    b = np.asarray(bitstrings, dtype=np.uint64)
    out = np.zeros(b.shape, dtype=np.int64)
    for i, q in enumerate(qubits):
        out |= ((b >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << i
    return out


def amplitudes(circ: Circuit, upper_mask: int, bitstrings, copy_begin: int = 0,
               copy_end: int | None = None) -> np.ndarray:
    """amp(x) = sum over copies k in the range of U_k[u(x)] * L_k[l(x)].

    Over all copies this is the amplitude of the whole circuit; over a slice
    it is that slice's partial sum.
    """
    n = circ.n
    full = (1 << n) - 1
    uq = half_qubits(n, upper_mask)
    lq = half_qubits(n, full & ~upper_mask)
    if not uq or not lq:
        raise ValueError("upper mask must be a non-empty proper subset")
    u = pack_bits(bitstrings, uq)
    lo = pack_bits(bitstrings, lq)
    uu, iu = np.unique(u, return_inverse=True)
    ll, il = np.unique(lo, return_inverse=True)
    A = half_states(circ, upper_mask, True, uu, copy_begin, copy_end)
    B = half_states(circ, upper_mask, False, ll, copy_begin, copy_end)
    C = A @ B.T
    return C[iu, il]


def gathered_halves(circ: Circuit, upper_mask: int, u_values, l_values,
                    copy_begin: int = 0, copy_end: int | None = None):
    """(A, B): A[i, k] = U_k[u_i], B[j, k] = L_k[l_j] over the copy range."""
    A = half_states(circ, upper_mask, True, np.asarray(u_values, dtype=np.int64), copy_begin, copy_end)
    B = half_states(circ, upper_mask, False, np.asarray(l_values, dtype=np.int64), copy_begin, copy_end)
    return A, B
