"""The named workloads: seeded random grid circuits, cut masks and bitstring sets.

Sizes follow the paper's workloads scaled to one GPU: a 4x4 case small enough
for brute force, 6x6 and 6x7 grids (the 42-qubit 6x7 grid is the paper's
single-GPU run, Table 3), an uneven pair of cuts, and one GPU's slice of the
8x8 (64-qubit) circuit of depth 22.
"""

from __future__ import annotations

from dataclasses import dataclass, field

from .circuits import random_grid_circuit, grid_rows_mask, grid_cols_mask


@dataclass(frozen=True)
class Workload:
    name: str
    rows: int
    cols: int
    depth: int
    seed: int
    upper_mask: int
    n_u: int                 # distinct upper values requested
    n_l: int                 # distinct lower values requested
    seed_u: int
    seed_l: int
    copy_begin: int = 0
    copy_end: int | None = None   # None = all copies
    note: str = ""
    two_qubit: str = "cz"    # cz, or the controlled gates cx / cy / mixed
    orient: str = "random"   # which endpoint of a controlled gate is the control
    drop_rows: tuple = ()    # rows whose vertical bonds to the next row are left out

    @property
    def n(self) -> int:
        return self.rows * self.cols

    def circuit_text(self) -> str:
        return random_grid_circuit(self.rows, self.cols, self.depth, self.seed,
                                   self.two_qubit, self.orient, self.drop_rows)


def _all_upper_lower(rows, cols, upper_rows):
    n = rows * cols
    nu = len(upper_rows) * cols
    return 1 << nu, 1 << (n - nu)


CONFIGS: dict[str, Workload] = {}


def _add(w: Workload) -> None:
    CONFIGS[w.name] = w


_add(Workload("grid4x4_d10", 4, 4, 10, 0, grid_rows_mask(4, 4, [0, 1]), 256, 256, 1000, 2000,
              note="16 qubits, 8+8 halves, all 65536 amplitudes"))
_add(Workload("grid6x6_d16", 6, 6, 16, 0, grid_rows_mask(6, 6, [0, 1, 2]), 256, 256, 1001, 2001,
              note="36 qubits, 18+18 halves, 2^8 x 2^8 bitstrings"))
_add(Workload("grid6x7_d20", 6, 7, 20, 0, grid_rows_mask(6, 7, [0, 1, 2]), 1024, 1024, 1002, 2002,
              note="42 qubits, 21+21 halves, 2^10 x 2^10 bitstrings"))
_add(Workload("grid6x7_d20_cols", 6, 7, 20, 0, grid_cols_mask(6, 7, [0, 1, 2]), 512, 512, 1003, 2003,
              note="42 qubits cut by columns 0-2: 18+24 halves"))
_add(Workload("grid6x6_d16_stair", 6, 6, 16, 0,
              grid_rows_mask(6, 6, [0, 1]) | sum(1 << (2 * 6 + c) for c in range(4)),
              512, 512, 1004, 2004,
              note="36 qubits, rows 0-1 plus row 2 columns 0-3: 16+20 halves"))
_add(Workload("grid6x8_d22_slice64", 6, 8, 22, 0, grid_rows_mask(6, 8, [0, 1, 2]), 256, 256,
              1006, 2006, copy_begin=0, copy_end=64,
              note="48 qubits, 24+24 halves, copies [0, 64) of 65536: the slice path at a size "
                   "the oracle can check"))
_add(Workload("grid8x8_d22_slice64", 8, 8, 22, 0, grid_rows_mask(8, 8, [0, 1, 2, 3]), 1024, 1024,
              1005, 2005, copy_begin=0, copy_end=64,
              note="64 qubits, 32+32 halves, copies [0, 64) of 65536: partial amplitudes"))


_add(Workload("grid8x8_d22_bands", 8, 8, 22, 0, grid_rows_mask(8, 8, [0, 1, 2, 3]), 1024, 1024,
              1008, 2008, copy_begin=0, copy_end=64, drop_rows=(1, 5),
              note="64 qubits, 32+32 halves, copies [0, 64) of 65536, with the vertical bonds "
                   "between rows 1-2 and 5-6 left out: each half is an independent 16-qubit band "
                   "(rows 0-1, rows 6-7) times the 16 qubits next to the cut, so the FP64 oracle "
                   "pins the partial amplitudes of the 32-qubit halves from 16-qubit states"))
_add(Workload("grid6x6_d16_mixed", 6, 6, 16, 0, grid_rows_mask(6, 6, [0, 1, 2]), 256, 256,
              1007, 2007, two_qubit="mixed", orient="random",
              note="36 qubits, 18+18 halves, each two-qubit gate drawn from CZ, CNOT and CY with "
                   "a random control (Supp. Eq. 1 cuts in both orientations)"))


def workload(name: str) -> Workload:
    return CONFIGS[name]
