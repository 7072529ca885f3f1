"""Seeded universal random grid circuits (paper Sec. 3, Fig. 4; Supp. A).

The paper builds its circuits with the rules of its Ref. [6] (Boixo et al.,
"Characterizing quantum supremacy in near-term devices") on an r x q grid and
prints no circuit, so the rules below are our reading of them:

* qubit id ``q = row * cols + col``;
* cycle 0 applies H to every qubit; the depth ``d`` counts the CZ cycles
  1..d after it (the paper gives the first layer one gate, Sec. 2.2);
* cycle t >= 1 fires the CZ class at position ``((t - 1) mod 8) + 1`` of an
  8-cycle pattern; the two classes that cross the centre line between rows
  ``R/2 - 1`` and ``R/2`` sit at positions 7 and 8, so only cycles 8a+7 and
  8a+8 hold CZ gates between the two halves (Supp. A);
* a one-qubit gate goes on qubit q in cycle t >= 2 iff q was in a CZ at t-1
  and is in none at t; the first such gate on q is T, later ones are drawn
  uniformly from {sqrt(X), sqrt(Y), T} minus the previous one-qubit gate of q.

This reading reproduces the CZ counts of Table 2 and the CZ totals of Fig. 4
exactly.  The one-qubit totals of Fig. 4 are not reproduced exactly (the
figure, which fixes the pattern order, is missing from the text).

CNOT-style variants (the controlled-U gates of Supp. Eq. 1): with
``two_qubit`` = "cx" or "cy" every CZ of the pattern becomes that gate, with
"mixed" each one is drawn from {cz, cx, cy}; ``orient`` = "random" draws
which endpoint is the control, "low" makes it the smaller qubit id.  These
draws use a second generator, so the CZ circuits are unchanged.
"""

from __future__ import annotations

import numpy as np

GATE_NAMES = ("h", "t", "sx", "sy", "cz", "cx", "cy")


def _hp(rows: int) -> int:
    return (rows // 2 - 1) % 2


def cz_pattern(rows: int, cols: int, position: int, drop_rows=()) -> list[tuple[int, int]]:
    """CZ pairs (q0 < q1) of pattern position 1..8 on a rows x cols grid.
    ``drop_rows``: rows r whose vertical bonds to row r + 1 never fire."""
    hp = _hp(rows)
    pairs: list[tuple[int, int]] = []

    def vert(row_parity_eq_hp: bool, col_parity: int) -> None:
        for r in range(rows - 1):
            if ((r % 2) == hp) != row_parity_eq_hp or r in drop_rows:
                continue
            for c in range(cols):
                if c % 2 == col_parity:
                    pairs.append((r * cols + c, (r + 1) * cols + c))

    def horiz(col_parity: int, row_parity: int) -> None:
        for r in range(rows):
            if r % 2 != row_parity:
                continue
            for c in range(cols - 1):
                if c % 2 == col_parity:
                    pairs.append((r * cols + c, r * cols + c + 1))

    if position == 1:
        vert(False, 0)
    elif position == 2:
        vert(False, 1)
    elif position == 3:
        horiz(0, 0)
    elif position == 4:
        horiz(1, 1)
    elif position == 5:
        horiz(1, 0)
    elif position == 6:
        horiz(0, 1)
    elif position == 7:
        vert(True, 1)
    elif position == 8:
        vert(True, 0)
    else:
        raise ValueError(f"pattern position must be 1..8, got {position}")
    return pairs


def random_grid_circuit_gates(rows: int, cols: int, depth: int, seed: int,
                              two_qubit: str = "cz", orient: str = "random", drop_rows=()):
    """Return the gate list [(cycle, name, qubits...)] of the seeded circuit.

    ``drop_rows``: rows r whose vertical bonds to row r + 1 are left out, which
    splits the grid into bands of rows with no gate between them (the bands
    are then independent circuits; the one-qubit gates follow the same rule
    on the remaining CZ gates)."""
    if rows < 2 or cols < 1:
        raise ValueError("grid needs at least 2 rows and 1 column")
    if two_qubit not in ("cz", "cx", "cy", "mixed") or orient not in ("random", "low"):
        raise ValueError("two_qubit must be cz, cx, cy or mixed; orient random or low")
    n = rows * cols
    rng = np.random.default_rng(seed)
    rng2 = np.random.default_rng([seed, 1])
    gates: list[tuple] = [(0, "h", q) for q in range(n)]
    prev_busy: set[int] = set()
    last_1q: dict[int, str] = {}
    for t in range(1, depth + 1):
        pairs = cz_pattern(rows, cols, ((t - 1) % 8) + 1, tuple(drop_rows))
        busy = {q for p in pairs for q in p}
        if t >= 2:
            for q in range(n):
                if q in prev_busy and q not in busy:
                    if q not in last_1q:
                        g = "t"
                    else:
                        choices = [x for x in ("sx", "sy", "t") if x != last_1q[q]]
                        g = choices[int(rng.integers(len(choices)))]
                    last_1q[q] = g
                    gates.append((t, g, q))
        for a, b in pairs:
            kind = two_qubit
            if kind == "mixed":
                kind = ("cz", "cx", "cy")[int(rng2.integers(3))]
            if kind != "cz" and orient == "random" and int(rng2.integers(2)):
                a, b = b, a
            gates.append((t, kind, a, b))
        prev_busy = busy
    return gates


def gates_to_text(n: int, gates, rows: int | None = None, cols: int | None = None,
                  comment: str | None = None) -> str:
    lines = []
    if comment:
        lines.append(f"# {comment}")
    lines.append(f"qubits {n}")
    if rows is not None:
        lines.append(f"grid {rows} {cols}")
    for g in gates:
        lines.append(" ".join(str(x) for x in g))
    return "\n".join(lines) + "\n"


def random_grid_circuit(rows: int, cols: int, depth: int, seed: int = 0,
                        two_qubit: str = "cz", orient: str = "random", drop_rows=()) -> str:
    """Circuit text of the seeded universal random circuit on a rows x cols grid."""
    gates = random_grid_circuit_gates(rows, cols, depth, seed, two_qubit, orient, drop_rows)
    extra = "" if two_qubit == "cz" else f" {two_qubit} {orient}"
    if drop_rows:
        extra += " without the vertical bonds below rows " + ",".join(str(r) for r in sorted(drop_rows))
    return gates_to_text(rows * cols, gates, rows, cols,
                         comment=f"random grid circuit {rows}x{cols} depth {depth} seed {seed}{extra}")


def grid_rows_mask(rows: int, cols: int, row_list) -> int:
    """Bit mask of the qubits in the given rows."""
    m = 0
    for r in row_list:
        for c in range(cols):
            m |= 1 << (r * cols + c)
    return m


def grid_cols_mask(rows: int, cols: int, col_list) -> int:
    """Bit mask of the qubits in the given columns."""
    m = 0
    for c in col_list:
        for r in range(rows):
            m |= 1 << (r * cols + c)
    return m
