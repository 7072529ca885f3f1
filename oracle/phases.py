"""Fused diagonal phase of one layer (Sec. 2.4, Eq. 3-6).

All T gates of a layer act on amplitude x as ((1+i)/sqrt 2)^{m1(x)}, m1 the
number of T qubits whose bit is 1 (Eq. 4); all CZ gates of a layer act as
(-1)^{m2(x)}, m2 the number of CZ edges with both ends 1 (Eq. 6).  The cut
projectors and Z of Eq. (1) are diagonal too: P_b keeps the amplitudes whose
bit equals b and zeroes the rest, Z^b negates those with bit 1 when b = 1.
"""

from __future__ import annotations

import numpy as np

OMEGA = (1 + 1j) / np.sqrt(2.0)


def layer_phase(n: int, t_qubits, cz_edges, proj=(), zflip=()) -> np.ndarray:
    """Diagonal of the fused layer, over all 2^n indices.

    ``proj`` holds (qubit, b) pairs for P_b, ``zflip`` qubits carrying Z.
    """
    x = np.arange(1 << n, dtype=np.int64)
    m1 = np.zeros(x.shape, dtype=np.int64)
    for q in t_qubits:
        m1 += (x >> q) & 1
    m2 = np.zeros(x.shape, dtype=np.int64)
    for a, b in cz_edges:
        m2 += ((x >> a) & 1) * ((x >> b) & 1)
    d = OMEGA ** m1 * (-1.0) ** m2
    for q, b in proj:
        d = d * (((x >> q) & 1) == b)
    for q in zflip:
        d = d * np.where((x >> q) & 1, -1.0, 1.0)
    return d.astype(np.complex128)
