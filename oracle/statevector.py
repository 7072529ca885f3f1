"""Plain full state-vector simulation in complex128, one gate at a time.

This is Eq. (4) of Supp. A evaluated layer by layer: within a layer the gates
act on disjoint qubits, so they are applied one after another in file order.
Amplitude index convention: bit q of the index is the value of qubit q.

States are numpy complex128 arrays; the elementwise updates run through
torch CPU views of the same memory (``torch.from_numpy``) so that large
states use all host threads.  The arithmetic is the same either way.
"""

from __future__ import annotations

import numpy as np
import torch

from . import gates as G
from .circuit import Circuit


def _view(psi: np.ndarray, *shape) -> torch.Tensor:
    return torch.from_numpy(psi).view(*shape)


def apply_1q(psi: np.ndarray, q: int, m: np.ndarray) -> None:
    """psi <- (m on qubit q) psi, in place."""
    v = _view(psi, -1, 2, 1 << q)
    a = v[:, 0, :].clone()
    b = v[:, 1, :].clone()
    m = [[complex(m[i, j]) for j in range(2)] for i in range(2)]
    v[:, 0, :] = m[0][0] * a + m[0][1] * b
    v[:, 1, :] = m[1][0] * a + m[1][1] * b


def apply_diag1(psi: np.ndarray, q: int, d0: complex, d1: complex) -> None:
    """psi <- diag(d0, d1) on qubit q, in place."""
    v = _view(psi, -1, 2, 1 << q)
    if d0 != 1:
        v[:, 0, :] *= complex(d0)
    if d1 != 1:
        v[:, 1, :] *= complex(d1)


def apply_cz(psi: np.ndarray, a: int, b: int) -> None:
    """psi <- CZ(a, b) psi: negate the amplitudes with both bits set."""
    lo, hi = min(a, b), max(a, b)
    v = _view(psi, -1, 2, 1 << (hi - lo - 1), 2, 1 << lo)
    v[:, 1, :, 1, :] *= -1


def apply_controlled(psi: np.ndarray, c: int, t: int, u: np.ndarray) -> None:
    """psi <- (P0 x I + P1 x u) psi on (control c, target t) (Supp. Eq. 1):
    u acts on the target within the amplitudes whose control bit is 1."""
    lo, hi = min(c, t), max(c, t)
    v = _view(psi, -1, 2, 1 << (hi - lo - 1), 2, 1 << lo)
    # axis 1 holds bit hi, axis 3 bit lo
    sub = v.select(1, 1) if c == hi else v.select(3, 1)
    ax = 2 if c == hi else 1  # the target's axis in sub
    a = sub.select(ax, 0).clone()
    b = sub.select(ax, 1).clone()
    m = [[complex(u[i, j]) for j in range(2)] for i in range(2)]
    sub.select(ax, 0).copy_(m[0][0] * a + m[0][1] * b)
    sub.select(ax, 1).copy_(m[1][0] * a + m[1][1] * b)


def apply_gate(psi: np.ndarray, name: str, qs) -> None:
    """Apply one gate by name.

    Besides the circuit gates this accepts the one-qubit factors of the cut
    identity CZ = P0 x I + P1 x Z (Eq. 1) and of its controlled-U form (Supp.
    Eq. 1): ``p0``, ``p1``, ``z``, ``x``, ``y`` and ``i``.
    """
    if name == "cz":
        apply_cz(psi, qs[0], qs[1])
    elif name in ("cx", "cy"):
        apply_controlled(psi, qs[0], qs[1], G.CONTROLLED_U[name])
    elif name == "x":
        apply_1q(psi, qs[0], G.X)
    elif name == "y":
        apply_1q(psi, qs[0], G.Y)
    elif name == "t":
        apply_diag1(psi, qs[0], 1.0, G.T[1, 1])
    elif name == "p0":
        apply_diag1(psi, qs[0], 1.0, 0.0)
    elif name == "p1":
        apply_diag1(psi, qs[0], 0.0, 1.0)
    elif name == "z":
        apply_diag1(psi, qs[0], 1.0, -1.0)
    elif name == "i":
        pass
    else:
        apply_1q(psi, qs[0], G.ONE_QUBIT[name])


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def simulate(circ: Circuit) -> np.ndarray:
    """Final state of the whole circuit started from |0...0>."""
    if circ.n > 30:
        raise ValueError("full state vector limited to 30 qubits")
    psi = zero_state(circ.n)
    for _, name, qs in circ.gates:
        apply_gate(psi, name, qs)
    return psi


def amplitudes(circ: Circuit, bitstrings) -> np.ndarray:
    """amp(x) = psi[x] for each bitstring x."""
    psi = simulate(circ)
    idx = np.asarray(bitstrings, dtype=np.uint64).astype(np.int64)
    return psi[idx]
