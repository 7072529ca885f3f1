"""FP64 CPU oracle for the CZ-partition simulator (arXiv 1802.06952).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute it.  It shares no code with the HIP
library (its own parser, its own gate tables, its own simulation loops); the
only common input is the circuit text and bitstrings written by
``workloads``.

Contents (each function cites the passage it follows):

* ``circuit``     -- parser of the circuit text format.
* ``gates``       -- the gate matrices in complex128.
* ``statevector`` -- plain full state-vector simulation, one gate at a time.
* ``dense``       -- dense 2^n x 2^n unitary brute force (n <= 10).
* ``phases``      -- the per-layer fused diagonal phase of Eq. (3)-(6).
* ``partition``   -- the partition scheme: cut CZs (Eq. 1), 2^c copies of two
                     half circuits, prefix reuse by depth-first recursion over
                     cut cycles (Sec. 2.3.2), amplitude assembly as the sum
                     over copies of upper times lower amplitudes.
* ``counting``    -- cut counts, equivalent qubits (Table 2) and the time
                     estimate of Eq. (2) (Table 1).
* ``multipart``   -- partitions into t parts in a chain (Sec. 3, Fig. 3): the
                     sum over all copies of the product of t part amplitudes.

Controlled-U gates (Supp. Eq. 1, U = X or Y) are applied directly in
``statevector`` and ``dense`` and, when cut, split as P_b on the control and
U^b on the target in ``partition`` and ``multipart``.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against a value or property the paper or the mathematics fixes (see the
module headers).  The paper prints no amplitude values, so amplitude parity is
pinned by dense brute force, unit norm, partitioned-versus-unpartitioned
agreement and the Eq. (1) identity, not by printed numbers.
"""
