"""Seeded output bitstrings.

Bit q of a bitstring (uint64) is the measured value of qubit q.  The paper
samples components of the two halves separately and takes their tensor
product (Sec. 2.3.1, Sec. 2.3.3), so a request of 2^B outcomes is drawn as a
product set: 2^(B/2) distinct uniform values for the upper qubits times
2^(B/2) distinct uniform values for the lower qubits.  Every bitstring of the
set is marginally uniform; this is not Born-rule sampling.
"""

from __future__ import annotations

import numpy as np


def mask_bits(mask: int) -> list[int]:
    """Qubit ids set in ``mask``, ascending."""
    return [q for q in range(64) if (mask >> q) & 1]


def _deposit(values: np.ndarray, bits: list[int]) -> np.ndarray:
    out = np.zeros(values.shape, dtype=np.uint64)
    v = values.astype(np.uint64)
    for j, q in enumerate(bits):
        out |= ((v >> np.uint64(j)) & np.uint64(1)) << np.uint64(q)
    return out


def split_bits(bitstrings: np.ndarray, mask: int) -> np.ndarray:
    """Pack the bits of ``bitstrings`` selected by ``mask`` (ascending order)."""
    out = np.zeros(bitstrings.shape, dtype=np.uint64)
    b = bitstrings.astype(np.uint64)
    for j, q in enumerate(mask_bits(mask)):
        out |= ((b >> np.uint64(q)) & np.uint64(1)) << np.uint64(j)
    return out


def _distinct_uniform(rng: np.random.Generator, width: int, count: int) -> np.ndarray:
    space = 1 << width
    if count > space:
        raise ValueError(f"cannot draw {count} distinct values of {width} bits")
    if space <= (1 << 22):
        return rng.permutation(space)[:count].astype(np.uint64)
    seen: set[int] = set()
    out = []
    while len(out) < count:
        x = int(rng.integers(0, space, dtype=np.uint64))
        if x not in seen:
            seen.add(x)
            out.append(x)
    return np.array(out, dtype=np.uint64)


def product_bitstrings(n: int, upper_mask: int, n_upper_values: int, n_lower_values: int,
                       seed_upper: int, seed_lower: int):
    """Product-set bitstrings.

    Returns ``(bitstrings, u_values, l_values)`` where ``bitstrings`` has
    length ``n_upper_values * n_lower_values`` in row-major (u, l) order and
    ``u_values`` / ``l_values`` are the packed half values (ascending qubit
    order inside each half).
    """
    full = (1 << n) - 1 if n < 64 else (1 << 64) - 1
    lower_mask = full & ~upper_mask
    ub = mask_bits(upper_mask)
    lb = mask_bits(lower_mask)
    u = _distinct_uniform(np.random.default_rng(seed_upper), len(ub), n_upper_values)
    lo = _distinct_uniform(np.random.default_rng(seed_lower), len(lb), n_lower_values)
    U = _deposit(u, ub)
    L = _deposit(lo, lb)
    bits = (U[:, None] | L[None, :]).reshape(-1)
    return bits, u, lo
