"""Circuit text parser of the oracle (its own; the HIP library has a separate C++ one).

A circuit is the layered form of Supp. A: a sequence of layers (cycles), each a
set of gates on disjoint qubits; an edge of the layer graph is a CZ.  The
controlled gates of Supp. Eq. 1 with U = X and U = Y ("cx", "cy") list the
control qubit first.
"""

from __future__ import annotations

from dataclasses import dataclass, field

ONE_QUBIT = ("h", "t", "sx", "sy")
TWO_QUBIT = ("cz", "cx", "cy")


@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)   # (cycle, name, (qubits...)) in file order

    def cycles(self) -> list[int]:
        return sorted({g[0] for g in self.gates})

    def gates_in_cycle(self, t: int) -> list:
        return [g for g in self.gates if g[0] == t]


def parse(text: str) -> Circuit:
    n = None
    gates = []
    last_cycle = -1
    used: dict[int, set] = {}
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "qubits":
            n = int(tok[1])
            if n < 1:
                raise ValueError(f"line {lineno}: qubit count must be positive")
            continue
        if tok[0] == "grid":
            continue
        if n is None:
            raise ValueError(f"line {lineno}: gate before 'qubits'")
        t = int(tok[0])
        name = tok[1]
        qs = tuple(int(x) for x in tok[2:])
        if t < last_cycle:
            raise ValueError(f"line {lineno}: cycles must not decrease")
        last_cycle = t
        if name in ONE_QUBIT:
            if len(qs) != 1:
                raise ValueError(f"line {lineno}: {name} takes one qubit")
        elif name in TWO_QUBIT:
            if len(qs) != 2 or qs[0] == qs[1]:
                raise ValueError(f"line {lineno}: {name} takes two distinct qubits")
        else:
            raise ValueError(f"line {lineno}: unknown gate {name!r}")
        for q in qs:
            if not 0 <= q < n:
                raise ValueError(f"line {lineno}: qubit {q} out of range")
            s = used.setdefault(t, set())
            if q in s:
                raise ValueError(f"line {lineno}: qubit {q} used twice in cycle {t}")
            s.add(q)
        gates.append((t, name, qs))
    if n is None:
        raise ValueError("missing 'qubits' line")
    return Circuit(n, gates)
