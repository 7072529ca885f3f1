"""GPU parity of partitions into t parts (Sec. 3, Fig. 3) through the C ABI.

Small circuits (18-20 qubits) against the oracle's full state vector, every
amplitude; at 48 qubits, beyond the state vector, the four-part chain against
the two-part path (itself checked against the oracle at 36-48 qubits) on the
same bitstrings.  Bounds as in test_gpu_parity (checks.assert_close):
norm-wise and element-wise, tolerance 1e-5 for the FP32 path.
"""

import sys

import numpy as np
import pytest

from checks import assert_close, errors

from oracle import circuit as OC, statevector as SV
from workloads import circuits as W

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_06952_amd as Q
    return Q


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()



def band_masks(rows, cols, bands):
    return [W.grid_rows_mask(rows, cols, b) for b in bands]


def band_product_bits(rows, cols, bands, per_band, seed):
    """Product set over the bands: per_band distinct values of each band."""
    rng = np.random.default_rng(seed)
    bits = np.zeros(1, dtype=np.uint64)
    for b in bands:
        nq = len(b) * cols
        v = rng.choice(1 << nq, size=min(per_band, 1 << nq), replace=False).astype(np.uint64)
        bits = (bits[:, None] | (v[None, :] << np.uint64(b[0] * cols))).reshape(-1)
    return bits


@pytest.mark.parametrize("rows,cols,depth,bands,two_qubit", [
    (6, 3, 12, [[0, 1], [2, 3], [4, 5]], "cz"),
    (5, 4, 12, [[0, 1], [2], [3], [4]], "cz"),
    (5, 4, 12, [[0], [1, 2], [3, 4]], "mixed"),
])
def test_chain_all_amplitudes(rows, cols, depth, bands, two_qubit):
    Q = _lib()
    text = W.random_grid_circuit(rows, cols, depth, 1, two_qubit)
    n = rows * cols
    bits = np.arange(1 << n, dtype=np.uint64)
    say(f"case chain {rows}x{cols} d{depth} {bands} {two_qubit}")
    cp = Q.ChainPlan(text, band_masks(rows, cols, bands))
    try:
        assert cp.t == len(bands) and all(c > 0 for c in cp.link_cuts)
        amp, stats = cp.amplitudes(bits)
    finally:
        cp.close()
    ref = SV.simulate(OC.parse(text))
    assert_close(amp, ref, 1e-5)
    assert abs(stats[0] - 1.0) < 1e-5  # all amplitudes: the norm


def test_chain_48q_against_two_part_path():
    """8x6 grid, depth 10: four row bands of 12 qubits against the 24+24 cut."""
    Q = _lib()
    rows, cols, depth = 8, 6, 10
    bands = [[0, 1], [2, 3], [4, 5], [6, 7]]
    text = W.random_grid_circuit(rows, cols, depth, 0)
    bits = band_product_bits(rows, cols, bands, 8, 11)
    say(f"case chain 48q: {bits.size} bitstrings")
    cp = Q.ChainPlan(text, band_masks(rows, cols, bands))
    try:
        amp4, _ = cp.amplitudes(bits)
    finally:
        cp.close()
    say("case chain 48q: two-part reference")
    p = Q.Plan(text, W.grid_rows_mask(rows, cols, [0, 1, 2, 3]))
    try:
        amp2, _ = p.amplitudes(bits)
    finally:
        p.close()
    assert_close(amp4, amp2.astype(np.complex128), 1e-5)


def test_chain_repeated_and_schedule_knobs():
    """Repeated bitstrings get equal amplitudes; forced schedules agree."""
    Q = _lib()
    rows, cols, depth = 6, 3, 12
    bands = [[0, 1], [2, 3], [4, 5]]
    text = W.random_grid_circuit(rows, cols, depth, 2)
    rng = np.random.default_rng(4)
    bits = rng.integers(0, 1 << 18, size=300, dtype=np.uint64)
    bits = np.concatenate([bits, bits[:7], [0, (1 << 18) - 1]]).astype(np.uint64)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    for kw in ({}, {"tile_bits": 7}, {"materialize_level": 0}, {"tail_max_qubits": 6}):
        say(f"case chain knobs {kw}")
        cp = Q.ChainPlan(text, band_masks(rows, cols, bands), **kw)
        try:
            amp, _ = cp.amplitudes(bits)
        except Q.QSError as e:
            assert e.status == -3, e  # a limit the planner cannot meet is reported
            continue
        finally:
            cp.close()
        assert_close(amp, ref, 1e-5)
        assert np.array_equal(amp[300:307], amp[:7])


def test_chain_errors():
    Q = _lib()
    text = W.random_grid_circuit(6, 3, 12, 2)
    cp = Q.ChainPlan(text, band_masks(6, 3, [[0, 1], [2, 3], [4, 5]]))
    try:
        cp.amplitudes(np.arange(16, dtype=np.uint64))
        with pytest.raises(Q.QSError) as e:
            cp.amplitudes(np.arange(17, dtype=np.uint64))
        assert e.value.status == -6  # another set on the same plan
    finally:
        cp.close()
    with pytest.raises(Q.QSError) as e:
        Q.ChainPlan(text, band_masks(6, 3, [[0, 1], [4, 5], [2, 3]]))
    assert e.value.status == -3  # not a chain
    with pytest.raises(Q.QSError) as e:
        Q.ChainPlan(text, band_masks(6, 3, [[0, 1], [2, 3]]))
    assert e.value.status == -1  # a qubit left out


@pytest.mark.parametrize("depth,masks_fn", [
    # the link between rows 1 and 2 has no cut gate at depth 6
    (6, lambda: band_masks(4, 3, [[0], [1], [2, 3]])),
    # a one-qubit part (qubit 0, whose neighbours are all in part 1)
    (8, lambda: [0b1, W.grid_rows_mask(4, 3, [0, 1]) & ~0b1, W.grid_rows_mask(4, 3, [2, 3])]),
])
def test_chain_degenerate_parts(depth, masks_fn):
    Q = _lib()
    text = W.random_grid_circuit(4, 3, depth, 0)
    masks = masks_fn()
    bits = np.arange(1 << 12, dtype=np.uint64)
    say(f"case chain degenerate depth {depth}")
    cp = Q.ChainPlan(text, masks)
    try:
        amp, _ = cp.amplitudes(bits)
        info = (cp.part_qubits, cp.link_cuts)
    finally:
        cp.close()
    assert 0 in info[1] or 1 in info[0]
    assert_close(amp, SV.simulate(OC.parse(text)), 1e-5)


@pytest.mark.parametrize("rows,cols,depth,bands,per_band", [
    (8, 4, 10, [[0, 1], [2, 3], [4, 5], [6, 7]], 8),   # 32 qubits, 4 cuts per link
    (6, 6, 8, [[0, 1], [2, 3], [4, 5]], 16),            # 36 qubits, 6 cuts per link
])
def test_chain_against_multipart_oracle(rows, cols, depth, bands, per_band):
    """Beyond the state vector: the FP64 t-part oracle (sum over all copies of
    the product of the part amplitudes) on 4096 band-product bitstrings."""
    from oracle import multipart as MP
    Q = _lib()
    text = W.random_grid_circuit(rows, cols, depth, 0)
    masks = band_masks(rows, cols, bands)
    bits = band_product_bits(rows, cols, bands, per_band, 50 + rows)
    say(f"case chain {rows}x{cols} d{depth} against the t-part oracle: {bits.size} bitstrings")
    cp = Q.ChainPlan(text, masks)
    try:
        amp, _ = cp.amplitudes(bits)
    finally:
        cp.close()
    say("case chain: oracle")
    ref = MP.amplitudes(OC.parse(text), masks, bits)
    assert_close(amp, ref, 1e-5)
