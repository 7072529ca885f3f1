"""A whole step (both halves on their two streams, fork and join events, the
assembly and the FP64 sums) can be captured into a HIP graph by a caller:
every replay gives the eager result bit for bit, with eager steps of the same
plan between the replays."""

import sys

import numpy as np
import pytest

from workloads import circuits as W, product_bitstrings

pytestmark = pytest.mark.gpu


def test_step_captured_in_a_graph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_06952_amd as Q
    text = W.random_grid_circuit(5, 6, 16, 3)
    mask = W.grid_rows_mask(5, 6, [0, 1])
    bits, _, _ = product_bitstrings(30, mask, 128, 96, 41, 42)
    m = int(bits.size)
    print("case graph capture 5x6 d16", flush=True)
    sys.stdout.flush()
    plan = Q.Plan(text, mask)
    try:
        total = 1 << plan.n_cuts
        d_out = torch.empty(2 * m, dtype=torch.float32, device="cuda")
        d_sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        side = torch.cuda.Stream()

        def step(st):
            plan.reset(keep_bitstrings=True)
            plan.run_halves(0, total, None, st)
            plan.amplitudes_device(0, d_out.data_ptr(), d_sums.data_ptr(), st)

        with torch.cuda.stream(side):
            plan.run_halves(0, total, bits, side)
            plan.amplitudes_device(0, d_out.data_ptr(), d_sums.data_ptr(), side)
            for _ in range(2):
                step(side)
        torch.cuda.synchronize()
        ref, ref_sums = d_out.clone(), d_sums.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            step(torch.cuda.current_stream())
        torch.cuda.synchronize()
        for _ in range(3):
            d_out.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(d_out, ref) and torch.equal(d_sums, ref_sums)
            with torch.cuda.stream(side):
                step(side)
            torch.cuda.synchronize()
            assert torch.equal(d_out, ref)
        # and the eager result is the library's amplitude
        amp, _ = plan.amplitudes(bits)
        assert np.array_equal(amp, ref.cpu().numpy().view(np.complex64))
    finally:
        plan.close()


def test_library_graph_step_matches_eager():
    """qs_run_graph: the step the plan captures and replays gives the eager
    step's amplitudes and sums bit for bit, over several replays with eager
    steps of the same plan in between, in both precisions, and again after
    the output pointer changes (a new capture)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_06952_amd as Q
    text = W.random_grid_circuit(5, 6, 16, 3)
    mask = W.grid_rows_mask(5, 6, [0, 1])
    bits, _, _ = product_bitstrings(30, mask, 128, 96, 41, 42)
    m = int(bits.size)
    print("case library graph 5x6 d16", flush=True)
    plan = Q.Plan(text, mask)
    try:
        total = 1 << plan.n_cuts
        side = torch.cuda.Stream()
        outs = [torch.empty(2 * m, dtype=torch.float32, device="cuda") for _ in range(2)]
        sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        with pytest.raises(Q.QSError, match="STATE"):
            plan.run_graph(0, total, 0, outs[0].data_ptr(), sums.data_ptr(), side)
        with torch.cuda.stream(side):
            plan.run_halves(0, total, bits, side)
        refs = {}
        for prec in (0, 1):
            plan.reset(keep_bitstrings=True)
            plan.run_halves(0, total, None, side)
            plan.amplitudes_device(prec, outs[0].data_ptr(), sums.data_ptr(), side)
            torch.cuda.synchronize()
            ref, ref_sums = outs[0].clone(), sums.clone()
            refs[prec] = ref
            for i in (0, 1):
                o = outs[i]
                for rep in range(3):
                    o.fill_(float("nan"))
                    sums.fill_(float("nan"))
                    plan.run_graph(0, total, prec, o.data_ptr(), sums.data_ptr(), side)
                    torch.cuda.synchronize()
                    assert torch.equal(o, ref) and torch.equal(sums, ref_sums), (prec, i, rep)
                    # an eager step of the same plan between replays, into the other output
                    plan.reset(keep_bitstrings=True)
                    plan.run_halves(0, total, None, side)
                    plan.amplitudes_device(prec, outs[1 - i].data_ptr(), None, side)
                    torch.cuda.synchronize()
                    assert torch.equal(outs[1 - i], ref)
        with pytest.raises(Q.QSError, match="ARG"):
            plan.run_graph(0, total, 0, outs[0].data_ptr(), None, 0)
        # the host-API amplitude of the same plan is the captured step's
        amp, _ = plan.amplitudes(bits, 0)
        assert np.array_equal(amp, refs[0].cpu().numpy().view(np.complex64))
    finally:
        plan.close()
