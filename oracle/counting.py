"""Counting identities of the partition scheme (Sec. 2.2, Sec. 3, Table 1, Table 2).

* Each cut CZ doubles the number of copies: 2^c copies, 2^(c+1) half circuits.
* Equivalent qubits N_e = n_half + log2(number of half circuits) (Sec. 3,
  first paragraph; the 8-qubit example gives 4 + log2 8 = 7).
* Time estimate of Eq. (2): sum over layers of n_i gates times m half circuits
  times t seconds per gate, divided by s nodes.  Sec. 2.2 fixes n_1 = 1,
  n_2 = n_3 = 2 and n_i = 8, 10, 12 for i > 3 for the 56-, 64- and 72-qubit
  half circuits.
"""

from __future__ import annotations

from .circuit import Circuit
from .partition import find_cuts


def cuts_per_cycle(circ: Circuit, upper_mask: int) -> dict[int, int]:
    out: dict[int, int] = {}
    for c in find_cuts(circ, upper_mask):
        out[c.cycle] = out.get(c.cycle, 0) + 1
    return out


def equivalent_qubits(n_half: int, c: int) -> int:
    """N_e for two halves of n_half qubits and c cut gates: n_half + c + 1."""
    half_circuits = 2 ** (c + 1)
    return n_half + (half_circuits.bit_length() - 1)


def eq2_time(depth: int, c: int, gates_per_layer_after_3: int, t_gate: float, nodes: int) -> float:
    """Eq. (2) with m = 2^(c+1) equivalent half circuits."""
    n_i = [1, 2, 2] + [gates_per_layer_after_3] * max(0, depth - 3)
    m = 2 ** (c + 1)
    return sum(n_i[:depth]) * m * t_gate / nodes
