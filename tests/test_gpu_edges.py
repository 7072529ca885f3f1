"""Edge cases of the HIP path against the FP64 oracle's full state vector.

Degenerate partitions (no cut, a one-qubit half, a circuit of depth 0), the
smallest and ragged bitstring sets (one bitstring, repeated bitstrings, value
grids that fill no kernel tile), the all-zero and all-one bitstrings, and both
assembly precisions.  Bounds as in test_gpu_parity (checks.assert_close):
norm-wise relative error and the largest single error against rms(a_ref),
tolerance 1e-5 for FP32 and 1e-4 for split-BF16.
"""

import sys

import numpy as np
import pytest

from checks import assert_close, errors

from oracle import circuit as OC, statevector as SV
from workloads import circuits as W, product_bitstrings

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-4}


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_06952_amd as Q
    return Q


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()



def amps(Q, text, mask, bits, prec=0, **kw):
    p = Q.Plan(text, mask, **kw)
    try:
        a, stats = p.amplitudes(np.ascontiguousarray(bits, dtype=np.uint64), prec)
    finally:
        p.close()
    return a, stats


def reference(text, bits):
    psi = SV.simulate(OC.parse(text))
    return psi[np.asarray(bits, dtype=np.int64)]


@pytest.mark.parametrize("prec", [0, 1])
def test_no_cut(prec):
    """A cut crossed by no CZ: one copy, the amplitude is U[u] L[l]."""
    Q = _lib()
    text = "qubits 4\n0 h 0\n0 h 1\n0 h 2\n0 h 3\n1 cz 0 1\n1 cz 2 3\n2 t 0\n2 sx 2\n3 sy 1\n"
    bits = np.arange(16, dtype=np.uint64)
    say(f"case no cut prec={prec}")
    p = Q.Plan(text, 0b0011)
    assert p.n_cuts == 0
    p.close()
    a, _ = amps(Q, text, 0b0011, bits, prec)
    assert_close(a, reference(text, bits), TOL[prec])


def test_depth_zero():
    """Only the H layer: every amplitude is 2^(-n/2)."""
    Q = _lib()
    text = "qubits 3\n0 h 0\n0 h 1\n0 h 2\n"
    bits = np.arange(8, dtype=np.uint64)
    say("case depth 0")
    a, stats = amps(Q, text, 0b001, bits)
    assert np.allclose(a, 2 ** -1.5, atol=1e-7)
    assert abs(stats[0] - 1.0) < 1e-6


def test_one_qubit_half():
    """The upper half is a single qubit (a corner of a 3x3 grid)."""
    Q = _lib()
    text = W.random_grid_circuit(3, 3, 12, 4)
    bits = np.arange(512, dtype=np.uint64)
    say("case one-qubit half")
    a, _ = amps(Q, text, 0b1, bits)
    assert_close(a, reference(text, bits), 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_single_bitstring(prec):
    Q = _lib()
    text = W.random_grid_circuit(4, 5, 16, 9)
    mask = W.grid_rows_mask(4, 5, [0, 1])
    bits = np.array([0b1011_0110_1100_1010_0111], dtype=np.uint64)
    say(f"case one bitstring prec={prec}")
    a, _ = amps(Q, text, mask, bits, prec)
    ref = reference(text, bits)
    assert abs(a[0] - ref[0]) <= TOL[prec] * max(abs(ref[0]), 2 ** -10)


def test_repeated_and_extreme_bitstrings():
    """Repeated entries get the same amplitude; the all-zero and all-one
    bitstrings are ordinary values."""
    Q = _lib()
    n = 20
    text = W.random_grid_circuit(4, 5, 16, 10)
    mask = W.grid_rows_mask(4, 5, [0, 1])
    full = (1 << n) - 1
    rng = np.random.default_rng(5)
    other = rng.integers(0, full, size=6, dtype=np.uint64)
    bits = np.array([0, full, other[0], 0, other[1], full, other[0]] + list(other[2:]),
                    dtype=np.uint64)
    say("case repeated and extreme bitstrings")
    a, _ = amps(Q, text, mask, bits)
    ref = reference(text, bits)
    assert_close(a, ref, 1e-5)
    assert a[0] == a[3] and a[1] == a[5] and a[2] == a[6]


@pytest.mark.parametrize("prec", [0, 1])
def test_ragged_value_grid(prec):
    """37 upper x 101 lower values: no dimension fills a GEMM or contraction tile."""
    Q = _lib()
    text = W.random_grid_circuit(4, 5, 16, 11)
    mask = W.grid_rows_mask(4, 5, [0, 1])
    bits, _, _ = product_bitstrings(20, mask, 37, 101, 21, 22)
    say(f"case ragged 37 x 101 prec={prec}")
    a, _ = amps(Q, text, mask, bits, prec)
    assert_close(a, reference(text, bits), TOL[prec])


@pytest.mark.parametrize("depth,kw", [
    (16, dict(tail_max_qubits=10, materialize_level=0)),   # q = 7, 8: fused
    (16, dict(tail_max_qubits=9, materialize_level=1)),    # q = 5 (two kernels), 7 (fused)
    (16, dict(tail_max_qubits=6)),                         # q = 5
    (20, dict(tail_max_qubits=10, materialize_level=1)),   # q = 8 over 9 leaf levels: two kernels
    (20, dict(tail_max_qubits=10, materialize_level=0)),   # q = 9: 8 amplitudes per lane
    (24, dict(tail_max_qubits=10, materialize_level=0)),   # q = 10, the largest: 16 per lane
])
def test_light_cone_sizes(depth, kw):
    """Leaf evaluation at light cones from the smallest to the largest the
    kernels take (the two-kernel form outside 6..8 qubits or beyond 8 leaf
    levels, the fused one inside)."""
    Q = _lib()
    text = W.random_grid_circuit(4, 5, depth, 12)
    mask = W.grid_rows_mask(4, 5, [0, 1])
    bits, _, _ = product_bitstrings(20, mask, 64, 64, 31, 32)
    say(f"case light cone {kw}")
    try:
        a, _ = amps(Q, text, mask, bits, **kw)
    except Q.QSError as e:
        # a limit the planner cannot meet is reported, not approximated
        assert e.status == -3, e
        pytest.skip(f"no schedule for {kw}")
    assert_close(a, reference(text, bits), 1e-5)
