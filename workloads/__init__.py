"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the simulation method: it only writes
circuit text and draws bitstrings.  Both the HIP path (through its own C++
parser) and the oracle (through its own Python parser) read what it writes.

Circuit text format (one gate per line, ``#`` starts a comment)::

    qubits <n>
    grid <rows> <cols>          # optional, informational
    <cycle> h <q>
    <cycle> t <q>
    <cycle> sx <q>              # square root of X
    <cycle> sy <q>              # square root of Y
    <cycle> cz <q0> <q1>
    <cycle> cx <control> <target>   # controlled X (CNOT)
    <cycle> cy <control> <target>   # controlled Y

Cycles are non-decreasing integers; within a cycle every qubit appears at most
once, so the gates of one cycle act on disjoint qubits.
"""

from .circuits import (  # noqa: F401
    GATE_NAMES,
    cz_pattern,
    random_grid_circuit,
    grid_rows_mask,
    grid_cols_mask,
)
from .bitstrings import product_bitstrings, mask_bits, split_bits  # noqa: F401
from .configs import CONFIGS, Workload, workload  # noqa: F401
