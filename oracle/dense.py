"""Dense brute force: the whole circuit as one 2^n x 2^n matrix (n <= 10).

Each gate is embedded with Kronecker products (qubit q is bit q of the index,
so the factor of qubit q sits at Kronecker position n-1-q); the circuit
unitary is the ordered product and the final state is its column 0.  This is
an independent route to Eq. (4) of Supp. A: it shares no indexing with the
state-vector code.
"""

from __future__ import annotations

import numpy as np

from . import gates as G
from .circuit import Circuit


def embed_1q(n: int, q: int, m: np.ndarray) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for pos in range(n - 1, -1, -1):
        out = np.kron(out, m if pos == q else G.I2)
    return out


def embed_cz(n: int, a: int, b: int) -> np.ndarray:
    d = np.ones(1 << n, dtype=np.complex128)
    for x in range(1 << n):
        if (x >> a) & 1 and (x >> b) & 1:
            d[x] = -1.0
    return np.diag(d)


def embed_controlled(n: int, c: int, t: int, u: np.ndarray) -> np.ndarray:
    """P0 x I + P1 x u on (control c, target t), Supp. Eq. 1, as Kronecker sums."""
    return embed_1q(n, c, G.P0) + embed_1q(n, c, G.P1) @ embed_1q(n, t, u)


def unitary(circ: Circuit) -> np.ndarray:
    n = circ.n
    if n > 10:
        raise ValueError("dense brute force limited to 10 qubits")
    u = np.eye(1 << n, dtype=np.complex128)
    for _, name, qs in circ.gates:
        if name == "cz":
            g = embed_cz(n, qs[0], qs[1])
        elif name in G.CONTROLLED_U:
            g = embed_controlled(n, qs[0], qs[1], G.CONTROLLED_U[name])
        else:
            g = embed_1q(n, qs[0], G.ONE_QUBIT[name])
        u = g @ u
    return u


def final_state(circ: Circuit) -> np.ndarray:
    return unitary(circ)[:, 0].copy()
