"""The band-factor golden writer (tests/golden/make_golden.py: band_factors)
against the plain oracle, on a 16-qubit circuit of the same shape as the
64-qubit banded workload: 8 rows of 2 columns, upper half rows 0-3, the
vertical bonds below rows 1 and 5 left out, depth 22 (4 cut gates).

Pins: over all copies the factors give the full state vector's amplitudes
(the whole circuit, no partition); over a copy slice they give the partition
oracle's partial sums on the whole circuit; the stored 64-qubit golden's
factors have the shapes and norms the construction fixes.
"""

import os
import sys

import numpy as np

from oracle import circuit as OC, partition as P, statevector as SV
from workloads import circuits as W, product_bitstrings, workload

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLDEN not in sys.path:
    sys.path.insert(0, GOLDEN)

import make_golden as MG  # noqa: E402


def _small():
    text = W.random_grid_circuit(8, 2, 22, 3, drop_rows=(1, 5))
    mask = W.grid_rows_mask(8, 2, [0, 1, 2, 3])
    return text, mask


def _amps(fu, A, B, fl):
    return fu[:, None] * (A @ B.T) * fl[None, :]


def test_blocks_of_the_banded_circuit():
    text, mask = _small()
    blocks = MG.independent_blocks(OC.parse(text))
    assert blocks == [[0, 1, 2, 3], [4, 5, 6, 7, 8, 9, 10, 11], [12, 13, 14, 15]]
    assert len(P.find_cuts(OC.parse(text), mask)) == 4


def test_band_factors_all_copies_equal_the_state_vector():
    text, mask = _small()
    bits, u, l = product_bitstrings(16, mask, 256, 256, 5, 6)
    fu, A, B, fl = MG.band_factors(text, mask, u, l, 0, 16)
    got = _amps(fu, A, B, fl).reshape(-1)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    assert np.abs(got - ref).max() < 1e-13
    assert abs(np.sum(np.abs(ref) ** 2) - 1.0) < 1e-12  # all 2^16 amplitudes


def test_band_factors_slice_equal_the_partition_oracle():
    text, mask = _small()
    bits, u, l = product_bitstrings(16, mask, 64, 64, 7, 8)
    for k0, k1 in [(0, 4), (4, 5), (9, 16)]:
        fu, A, B, fl = MG.band_factors(text, mask, u, l, k0, k1)
        got = _amps(fu, A, B, fl).reshape(-1)
        ref = P.amplitudes(OC.parse(text), mask, bits, k0, k1)
        assert np.abs(got - ref).max() < 1e-13, (k0, k1)


def test_stored_64_qubit_factors():
    w = workload("grid8x8_d22_bands")
    g = np.load(os.path.join(GOLDEN, f"{w.name}.npz"))
    _, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    assert np.array_equal(g["u"], u.astype(np.int64)) and np.array_equal(g["l"], l.astype(np.int64))
    assert g["A"].shape == (1024, 64) and g["B"].shape == (1024, 64)
    # the bands outside the cut block are 16-qubit states sampled at uniform
    # values: 2^16 mean |psi|^2 estimates 1
    for f in (g["fu"], g["fl"]):
        assert abs(np.mean(np.abs(f) ** 2) * 2 ** 16 - 1.0) < 0.2
    # the circuit's independent blocks are rows 0-1, rows 2-5 (every cut
    # gate, 16 of them, between rows 3 and 4) and rows 6-7
    circ = OC.parse(w.circuit_text())
    assert MG.independent_blocks(circ) == [list(range(16)), list(range(16, 48)), list(range(48, 64))]
    cuts = P.find_cuts(circ, w.upper_mask)
    assert len(cuts) == 16 and all(24 <= c.upper < 32 and 32 <= c.lower < 40 for c in cuts)
