"""The C ABI's resource contract on the GPU: the caller's allocator, and the
bounded cache of block plans (every amplitude against the FP64 oracle)."""

import sys

import numpy as np
import pytest

from checks import assert_close

from oracle import circuit as OC, statevector as SV
from workloads import circuits as W, product_bitstrings, workload

pytestmark = pytest.mark.gpu

GOLDEN_TOL = 1e-5


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_06952_amd as Q
    return Q


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_torch_allocator_bit_identical_and_flat():
    """A plan whose buffers come from PyTorch's caching allocator gives the
    same amplitudes, bit for bit, as one on hipMalloc; after the first step
    repeated steps allocate nothing more, and closing the plan frees every
    buffer it took."""
    Q = _lib()
    import torch
    w = workload("grid6x6_d16")
    text = w.circuit_text()
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    m = bits.size
    say("case allocator: hipMalloc plan")
    p = Q.Plan(text, w.upper_mask, alloc=None)
    ref, _ = p.amplitudes(bits)
    p.close()
    say("case allocator: torch plan")
    p = Q.Plan(text, w.upper_mask, alloc="torch")
    a = p.allocator
    d_out = torch.empty(2 * m, dtype=torch.float32, device="cuda")
    total = 1 << p.n_cuts
    counts = []
    for rep in range(5):
        if rep < 2:
            # host API; the second time after a reset that forgets the
            # bitstrings: the same set again reuses its tables and block plans
            p.reset(keep_bitstrings=False)
            got, _ = p.amplitudes(bits)
        else:
            p.reset(keep_bitstrings=True)
            p.run_halves(0, total, None)
            p.amplitudes_device(0, d_out.data_ptr(), None)
            torch.cuda.synchronize()
            got = d_out.cpu().numpy().view(np.complex64)
        assert np.array_equal(got, ref), rep
        counts.append(a.n_alloc)
    assert counts[0] > 0 and counts[1] == counts[2] == counts[3] == counts[4], counts
    p.close()
    assert a.live == 0 and a.n_free == a.n_alloc


def test_plain_form_more_blocks_than_the_plan_cache():
    """The flat per-copy form plans every copy as a block of its own; with
    4096 copies (8192 block plans of the two halves) the plan cache is
    emptied and refilled while copies run.  Every amplitude against the
    FP64 state vector."""
    Q = _lib()
    text = W.random_grid_circuit(2, 4, 24, 1)
    mask = W.grid_rows_mask(2, 4, [0])
    bits, _, _ = product_bitstrings(8, mask, 16, 16, 1, 2)
    say("case plain form, 4096 copies of a 2x4 circuit")
    p = Q.Plan(text, mask, plain=True)
    assert p.n_cuts == 12
    try:
        amp, _ = p.amplitudes(bits)
    finally:
        p.close()
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    assert_close(amp, ref, GOLDEN_TOL)
