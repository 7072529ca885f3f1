"""qs_amplitudes_device_static, the allocation-free assembly, against
qs_amplitudes_device on the same plan, through the C ABI: two calls in a row,
the second with a smaller input, both assembly precisions.  The static form
takes its scratch from the library's static region, so the plan's allocator
sees no request during the call."""

import sys

import numpy as np
import pytest

from checks import assert_close

from workloads import product_bitstrings, workload

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-4}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(Q, torch, name):
    w = workload(name)
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    m = bits.size
    p = Q.Plan(w.circuit_text(), w.upper_mask, alloc="torch")
    try:
        k1 = w.copy_end if w.copy_end is not None else 1 << p.n_cuts
        p.run_halves(w.copy_begin, k1, bits)
        ref = torch.empty(2 * m, dtype=torch.float32, device="cuda")
        got = torch.full((2 * m,), float("nan"), dtype=torch.float32, device="cuda")
        sref = torch.zeros(2, dtype=torch.float64, device="cuda")
        sgot = torch.zeros(2, dtype=torch.float64, device="cuda")
        for prec in (0, 1):
            say(f"case no-alloc {name} m={m} prec={prec}")
            p.amplitudes_device(prec, ref.data_ptr(), sref.data_ptr())
            torch.cuda.synchronize()
            n0 = p.allocator.n_alloc
            p.amplitudes_device_static(prec, got.data_ptr(), sgot.data_ptr())
            torch.cuda.synchronize()
            assert p.allocator.n_alloc == n0
            a = got.cpu().numpy().view(np.complex64)
            r = ref.cpu().numpy().view(np.complex64)
            assert_close(a, r.astype(np.complex128), TOL[prec], what=f"{name} prec {prec}")
            # the same kernels in the same order: the same bits
            assert np.array_equal(a, r)
            assert np.array_equal(sgot.cpu().numpy(), sref.cpu().numpy())
            got.fill_(float("nan"))
    finally:
        p.close()


def test_static_assembly_matches_device_assembly():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_06952_amd as Q
    # the 42-qubit workload (2^20 amplitudes), then a smaller one (2^16)
    _case(Q, torch, "grid6x7_d20")
    _case(Q, torch, "grid6x6_d16")
