"""Exchange groups on the GPU: runs of full-state passes that share one
launch and pass their workgroup tiles through LDS between the passes.  The
grouped schedule packs the gates differently from the one without groups
(other diagonal runs, so other rounding), so the two agree to FP32 accuracy,
not bit for bit; the grouped path is checked against the FP64 state vector."""

import sys

import numpy as np
import pytest

from checks import assert_close

from oracle import circuit as OC, statevector as SV
from workloads import circuits as W, product_bitstrings, workload

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


def _groups(plan, k0, k1):
    d = plan.dump(k0, k1)
    return [[pp["xg"] for pp in s["passes"] if pp["xg"] > 1] for s in d["sides"]]


@pytest.mark.parametrize("name,knobs", [
    ("grid6x6_d16", {"tile_bits": 9}),
    ("grid6x7_d20", {}),
    ("grid6x7_d20", {"tile_bits": 11}),
])
def test_grouped_passes_match_single_passes(name, knobs):
    Q = _lib()
    w = workload(name)
    text = w.circuit_text()
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    out = {}
    for ex in (True, False):
        say(f"case exchange {name} {knobs} grouped={ex}")
        p = Q.Plan(text, w.upper_mask, no_exchange=not ex, **knobs)
        try:
            k1 = w.copy_end if w.copy_end is not None else (1 << p.n_cuts)
            g = _groups(p, w.copy_begin, k1)
            if ex:
                assert any(g), "the planner formed no exchange group"
            else:
                assert not any(g)
            out[ex] = p.amplitudes(bits)
        finally:
            p.close()
    a, sa = out[True]
    b, sb = out[False]
    assert a.dtype == np.complex64
    assert_close(a, b, 1e-5, "grouped against single passes")


def test_grouped_passes_against_state_vector():
    """A 3x8 grid of depth 18 cut 8 + 16 (top row): with 9-bit tiles the lower
    half's passes form exchange groups (R = 3 register bits on workgroup tiles
    of 6 + 3 + 3 bits), and 4096 random amplitudes match the FP64 state vector."""
    Q = _lib()
    rows, cols, depth = 3, 8, 18
    text = W.random_grid_circuit(rows, cols, depth, 3)
    mask = W.grid_rows_mask(rows, cols, [0])
    n = rows * cols
    ref = SV.simulate(OC.parse(text))
    xs = np.random.default_rng(7).choice(1 << n, size=4096, replace=False).astype(np.uint64)
    say("case exchange 3x8 d18 state vector")
    p = Q.Plan(text, mask, tile_bits=9, min_tile_bits=9)
    try:
        assert any(_groups(p, 0, 1 << p.n_cuts))
        amp, _ = p.amplitudes(xs)
    finally:
        p.close()
    assert_close(amp, ref[xs.astype(np.int64)], 1e-5)
