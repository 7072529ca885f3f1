"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Every comparison asserts two bounds (``checks.assert_close``): the norm-wise
relative error ||a - a_ref|| / ||a_ref|| over the evaluated amplitudes, and the
largest single error max |a - a_ref| against 8 times the tolerance in units of
rms(a_ref) (per-amplitude relative errors are ill-conditioned near the zeros of
a Porter-Thomas distribution).  Tolerances: 1e-5 for the FP32 path, 1e-4 for
the split-BF16 assembly.
"""

import os
import sys

import numpy as np
import pytest

from checks import assert_close, errors

from oracle import circuit as OC, partition as P, statevector as SV
from workloads import circuits as W, product_bitstrings, workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
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



def run_plan(Q, text, mask, bits, prec=0, **kw):
    p = Q.Plan(text, mask, **kw)
    try:
        amp, stats = p.amplitudes(bits, prec)
    finally:
        p.close()
    return amp, stats


@pytest.mark.parametrize("prec", [0, 1])
def test_grid4x4_all_amplitudes(prec):
    Q = _lib()
    w = workload("grid4x4_d10")
    text = w.circuit_text()
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    say(f"case grid4x4_d10 prec={prec} m={bits.size}")
    amp, stats = run_plan(Q, text, w.upper_mask, bits, prec)
    psi = SV.simulate(OC.parse(text))
    ref = psi[bits.astype(np.int64)]
    assert_close(amp, ref, TOL[prec])
    # every amplitude of the state: the probabilities sum to one
    assert abs(stats[0] - 1.0) < 1e-5
    assert abs(stats[1] - 1.0) < 1e-5


@pytest.mark.parametrize("rows,cols,depth,mask,seed", [
    (4, 4, 16, W.grid_cols_mask(4, 4, [0, 1]), 1),
    (3, 4, 18, W.grid_rows_mask(3, 4, [0]) | 0b0011 << 4, 2),
    (2, 6, 12, W.grid_cols_mask(2, 6, [0, 2, 4]), 3),
    (4, 5, 12, W.grid_rows_mask(4, 5, [0, 1]), 4),
    (5, 4, 14, W.grid_rows_mask(5, 4, [0, 1]), 5),
])
def test_masks_against_full_state(rows, cols, depth, mask, seed):
    Q = _lib()
    text = W.random_grid_circuit(rows, cols, depth, seed)
    n = rows * cols
    nu = bin(mask).count("1")
    bits, _, _ = product_bitstrings(n, mask, min(64, 1 << nu), min(64, 1 << (n - nu)), seed, seed + 1)
    say(f"case masks {rows}x{cols} d{depth} mask={mask:#x}")
    amp, _ = run_plan(Q, text, mask, bits)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    assert_close(amp, ref, 1e-5)


@pytest.mark.parametrize("kw", [
    dict(tile_bits=6, coalesce_bits=2),
    dict(tile_bits=9, coalesce_bits=3, materialize_level=0, tail_max_qubits=10),
    dict(tile_bits=13, coalesce_bits=6, materialize_level=2),
    dict(tile_bits=8, coalesce_bits=0, materialize_level=100),
])
def test_schedule_knobs_same_result(kw):
    Q = _lib()
    text = W.random_grid_circuit(4, 5, 16, 7)
    mask = W.grid_rows_mask(4, 5, [0, 1])
    bits, _, _ = product_bitstrings(20, mask, 128, 128, 11, 12)
    say(f"case knobs {kw}")
    amp, _ = run_plan(Q, text, mask, bits, **kw)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    assert_close(amp, ref, 1e-5)


def test_two_streams_match_one_stream():
    """The halves on two streams (the default) give bit-identical amplitudes to
    the serial order, over repeated runs of one plan (buffers change streams
    between runs) and several copy blocks."""
    Q = _lib()
    import torch
    w = workload("grid6x6_d16")
    text = w.circuit_text()
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    say("case one stream")
    p = Q.Plan(text, w.upper_mask, one_stream=True)
    total = 1 << p.n_cuts
    p.run_halves(0, total // 2, bits)
    p.run_halves(total // 2, total, bits)
    ref, _ = p.amplitudes(bits)
    p.close()
    assert_close(ref, _golden(w.name)["amp"], 1e-5)
    p = Q.Plan(text, w.upper_mask)
    stream = torch.cuda.Stream()
    d_out = torch.empty(2 * bits.size, dtype=torch.float32, device="cuda")
    for rep in range(3):
        say(f"case two streams, run {rep}")
        p.reset(keep_bitstrings=rep > 0)
        p.run_halves(0, total // 2, bits if rep == 0 else None, stream)
        p.run_halves(total // 2, total, None, stream)
        p.amplitudes_device(0, d_out.data_ptr(), None, stream)
        stream.synchronize()
        got = d_out.cpu().numpy().view(np.complex64)
        assert np.array_equal(got, ref), rep
    p.close()


def test_copy_slices_partial_sums():
    Q = _lib()
    text = W.random_grid_circuit(4, 4, 12, 5)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    oc = OC.parse(text)
    bits, _, _ = product_bitstrings(16, mask, 32, 32, 3, 4)
    p = Q.Plan(text, mask)
    total = 1 << p.n_cuts
    ranges = [(0, 3), (3, 8), (8, total - 1), (total - 1, total)]
    got = np.zeros(bits.size, dtype=np.complex128)
    for a, b in ranges:
        say(f"case slice [{a},{b})")
        q = Q.Plan(text, mask)
        q.run_halves(a, b, bits)
        amp, _ = q.amplitudes(bits)
        q.close()
        ref = P.amplitudes(oc, mask, bits, a, b)
        # partial sums of a slice can be small: both bounds with a floor
        scale = max(np.linalg.norm(ref), 1e-3)
        assert np.linalg.norm(amp - ref) <= 1e-5 * scale
        assert np.abs(amp - ref).max() <= 8 * 1e-5 * scale / np.sqrt(ref.size)
        got += amp
    full = SV.simulate(oc)[bits.astype(np.int64)]
    assert_close(got, full, 1e-5)
    # several ranges on one plan accumulate
    for a, b in ranges:
        p.run_halves(a, b, bits)
    amp, _ = p.amplitudes(bits)
    assert_close(amp, full, 1e-5)
    # a range may not run twice
    with pytest.raises(Q.QSError):
        p.run_halves(0, 1, bits)
    p.close()


def test_folded_end_cuts_on_odd_copy_counts():
    """The 42-qubit circuit's lower half has three end cuts, folded into the
    assembly as 8 groups of K / 8 copies.  Copy ranges of 8 give one copy per
    group (an odd count: the register-staged FP32 product), a range of 16 two
    (the direct-to-LDS product); the partial sums of [0, 8) and [8, 16) add up
    to [0, 16), in FP32 and in split-BF16."""
    Q = _lib()
    w = workload("grid6x7_d20")
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, 64, 64, w.seed_u, w.seed_l)
    for prec in (0, 1):
        part = {}
        for a, b in [(0, 8), (8, 16), (0, 16)]:
            say(f"case grid6x7_d20 copies [{a},{b}) prec={prec}")
            p = Q.Plan(w.circuit_text(), w.upper_mask)
            try:
                p.run_halves(a, b, bits)
                part[(a, b)], _ = p.amplitudes(bits, prec)
            finally:
                p.close()
        assert_close(part[(0, 8)] + part[(8, 16)], part[(0, 16)], TOL[prec], f"prec {prec}")


def test_argument_errors():
    Q = _lib()
    w = workload("grid4x4_d10")
    p = Q.Plan(w.circuit_text(), w.upper_mask)
    with pytest.raises(Q.QSError) as e:
        p.run_halves(0, 1 << p.n_cuts, np.array([1 << 16], dtype=np.uint64))
    assert e.value.status == -1
    with pytest.raises(Q.QSError) as e:
        p.run_halves(0, (1 << p.n_cuts) + 1, np.array([1], dtype=np.uint64))
    assert e.value.status == -1
    p.run_halves(0, 4, np.array([1, 2], dtype=np.uint64))
    with pytest.raises(Q.QSError) as e:
        p.amplitudes(np.array([1, 3], dtype=np.uint64))
    assert e.value.status == -6
    p.close()


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path)


@pytest.mark.parametrize("prec", [0, 1])
def test_grid6x6_d16_golden(prec):
    Q = _lib()
    w = workload("grid6x6_d16")
    g = _golden(w.name)
    bits, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    assert np.array_equal(g["u"], u.astype(np.int64)) and np.array_equal(g["l"], l.astype(np.int64))
    say(f"case grid6x6_d16 prec={prec}")
    amp, stats = run_plan(Q, w.circuit_text(), w.upper_mask, bits, prec)
    assert_close(amp, g["amp"], TOL[prec])


@pytest.mark.parametrize("prec", [0, 1])
def test_grid6x7_d20_full_size_subset(prec):
    """The 2^20-bitstring workload; the oracle holds the first 64 x 64 block."""
    Q = _lib()
    w = workload("grid6x7_d20")
    g = _golden(w.name)
    bits, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    nu, nl = len(g["u"]), len(g["l"])
    assert np.array_equal(g["u"], u[:nu].astype(np.int64))
    say(f"case grid6x7_d20 prec={prec} m={bits.size}")
    amp, stats = run_plan(Q, w.circuit_text(), w.upper_mask, bits, prec)
    sub = amp.reshape(w.n_u, w.n_l)[:nu, :nl].reshape(-1)
    assert_close(sub, g["amp"], TOL[prec])
    # uniform bitstrings: 2^n mean p estimates 1
    assert abs(stats[1] - 1.0) < 0.05


def test_grid6x7_d20_values_past_the_first_round():
    """1024 values per half: the leaf evaluation's persistent workgroups (one
    per compute unit) take several values each, one pipeline over all their
    chunks.  Blocks of 256 x 256 values run alone (one value per workgroup)
    give the same amplitudes as the same values inside the full set."""
    Q = _lib()
    w = workload("grid6x7_d20")
    bits, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    say(f"case grid6x7_d20 full set m={bits.size}")
    amp, _ = run_plan(Q, w.circuit_text(), w.upper_mask, bits)
    full = amp.reshape(w.n_u, w.n_l)
    B = bits.reshape(w.n_u, w.n_l)
    for ku, kl in [(1, 3), (3, 1), (2, 2), (0, 0)]:
        ru, rl = slice(256 * ku, 256 * (ku + 1)), slice(256 * kl, 256 * (kl + 1))
        say(f"case grid6x7_d20 block upper {ku} lower {kl}")
        sub, _ = run_plan(Q, w.circuit_text(), w.upper_mask, np.ascontiguousarray(B[ru, rl]).reshape(-1))
        assert_close(full[ru, rl].reshape(-1), sub, TOL[0], f"block {ku},{kl}")
    # a ragged count: 300 x 260 values, so that some workgroups take two values
    # and the others one
    ru, rl = slice(700, 1000), slice(37, 297)
    say("case grid6x7_d20 ragged 300 x 260")
    sub, _ = run_plan(Q, w.circuit_text(), w.upper_mask, np.ascontiguousarray(B[ru, rl]).reshape(-1))
    assert_close(full[ru, rl].reshape(-1), sub, TOL[0], "ragged block")


def test_plain_form_and_device_outputs():
    Q = _lib()
    import torch
    text = W.random_grid_circuit(4, 4, 12, 5)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    bits, _, _ = product_bitstrings(16, mask, 32, 32, 3, 4)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    say("case plain form")
    amp, _ = run_plan(Q, text, mask, bits, plain=True)
    assert_close(amp, ref, 1e-5)
    say("case device outputs")
    p = Q.Plan(text, mask)
    total = 1 << p.n_cuts
    p.run_halves(0, total, bits)
    d = torch.empty(2 * bits.size, dtype=torch.float32, device="cuda")
    sums = torch.zeros(2, dtype=torch.float64, device="cuda")
    p.amplitudes_device(0, d.data_ptr(), sums.data_ptr())
    torch.cuda.synchronize()
    got = d.cpu().numpy().view(np.complex64)
    assert_close(got, ref, 1e-5)
    pr = np.abs(ref) ** 2
    s = sums.cpu().numpy()
    assert abs(s[0] - pr.sum()) < 1e-5 * pr.sum()
    assert abs(s[1] - (pr ** 2).sum()) < 1e-4 * (pr ** 2).sum()
    # a second round on the registered bitstrings, split-BF16 assembly
    p.reset(keep_bitstrings=True)
    p.run_halves(0, total)
    p.amplitudes_device(1, d.data_ptr(), None)
    torch.cuda.synchronize()
    got = d.cpu().numpy().view(np.complex64)
    assert_close(got, ref, 1e-4)
    p.close()


def test_list_mode_non_product_bitstrings():
    """Bitstrings that are not a product set take the per-bitstring sum."""
    Q = _lib()
    text = W.random_grid_circuit(4, 5, 14, 9)
    mask = W.grid_rows_mask(4, 5, [0, 1])
    rng = np.random.default_rng(5)
    bits = rng.choice(1 << 20, size=3000, replace=False).astype(np.uint64)
    say("case list mode")
    amp, stats = run_plan(Q, text, mask, bits)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    assert_close(amp, ref, 1e-5)


def _golden_bits(w, g):
    """Full bitstrings of a golden file's (u, l) product set."""
    from workloads.bitstrings import mask_bits
    full = (1 << w.n) - 1
    ub, lb = mask_bits(w.upper_mask), mask_bits(full & ~w.upper_mask)
    U = np.zeros(len(g["u"]), dtype=np.uint64)
    L = np.zeros(len(g["l"]), dtype=np.uint64)
    for j, q in enumerate(ub):
        U |= ((g["u"].astype(np.uint64) >> np.uint64(j)) & np.uint64(1)) << np.uint64(q)
    for j, q in enumerate(lb):
        L |= ((g["l"].astype(np.uint64) >> np.uint64(j)) & np.uint64(1)) << np.uint64(q)
    return (U[:, None] | L[None, :]).reshape(-1)


@pytest.mark.parametrize("row_name,cut_name,sub", [
    ("grid6x7_d20", "grid6x7_d20_cols", None),
    ("grid6x6_d16", "grid6x6_d16_stair", 4096),
])
def test_cut_invariance_against_golden(row_name, cut_name, sub):
    """The same circuit cut another way (uneven halves) reproduces the oracle."""
    Q = _lib()
    wr, wc = workload(row_name), workload(cut_name)
    g = _golden(row_name)
    bits = _golden_bits(wr, g)
    ref = g["amp"]
    if sub:
        idx = np.random.default_rng(0).choice(bits.size, size=sub, replace=False)
        bits, ref = bits[idx], ref[idx]
    say(f"case cut invariance {cut_name} m={bits.size}")
    amp, _ = run_plan(Q, wc.circuit_text(), wc.upper_mask, bits)
    assert_close(amp, ref, 1e-5)


def test_coscheduled_uneven_pair_against_golden():
    """The uneven pair run together: the 42-qubit circuit cut 18+24 and the
    36-qubit circuit cut 16+20, each plan on a stream of its own (and each
    plan's lower half on the plan's second stream), launched back to back so
    that copies of all four half sizes are in flight at once.  Both results
    against the row-cut goldens of the same circuits, twice over (the second
    round reuses the registered bitstrings and cached plans)."""
    Q = _lib()
    import torch
    cases = []
    for row_name, cut_name, sub in (("grid6x7_d20", "grid6x7_d20_cols", None),
                                    ("grid6x6_d16", "grid6x6_d16_stair", 4096)):
        wr, wc = workload(row_name), workload(cut_name)
        g = _golden(row_name)
        bits = _golden_bits(wr, g)
        ref = g["amp"]
        if sub:
            idx = np.random.default_rng(0).choice(bits.size, size=sub, replace=False)
            bits, ref = bits[idx], ref[idx]
        cases.append((wc, bits, ref))
    streams = [torch.cuda.Stream() for _ in cases]
    plans = [Q.Plan(wc.circuit_text(), wc.upper_mask) for wc, _, _ in cases]
    try:
        assert [(p.n_upper, p.n_lower) for p in plans] == [(18, 24), (16, 20)]
        outs = [torch.empty(2 * b.size, dtype=torch.float32, device="cuda") for _, b, _ in cases]
        for rnd in range(2):
            say(f"case co-scheduled uneven pair, round {rnd}")
            for p, (wc, bits, _), st, o in zip(plans, cases, streams, outs):
                p.reset(keep_bitstrings=rnd > 0)
                p.run_halves(0, 1 << p.n_cuts, bits if rnd == 0 else None, st)
                p.amplitudes_device(0, o.data_ptr(), None, st)
            torch.cuda.synchronize()
            for (wc, _, ref), o in zip(cases, outs):
                amp = o.cpu().numpy().view(np.complex64)
                assert_close(amp, ref, 1e-5, what=wc.name)
    finally:
        for p in plans:
            p.close()


def test_grid6x8_slice_golden():
    """Copies [0, 64) of 65536 of a 48-qubit circuit: partial amplitudes vs the oracle."""
    Q = _lib()
    w = workload("grid6x8_d22_slice64")
    g = _golden(w.name)
    bits, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    say("case grid6x8 slice")
    p = Q.Plan(w.circuit_text(), w.upper_mask)
    p.run_halves(w.copy_begin, w.copy_end, bits)
    amp, _ = p.amplitudes(bits)
    p.close()
    assert_close(amp, g["amp"], 1e-5)


def test_grid8x8_slice_full_size():
    """64 qubits, 32+32 halves, copies [0, 64): the two sub-slices add up to the
    slice, and the split-BF16 assembly agrees with FP32."""
    Q = _lib()
    import torch
    w = workload("grid8x8_d22_slice64")
    bits, _, _ = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    text = w.circuit_text()
    say("case grid8x8 slice [0,64)")
    p = Q.Plan(text, w.upper_mask)
    p.run_halves(0, 64, bits)
    a32, _ = p.amplitudes(bits, 0)
    ab, _ = p.amplitudes(bits, 1)
    p.close()
    torch.cuda.empty_cache()
    assert np.linalg.norm(a32) > 0
    assert_close(ab, a32.astype(np.complex128), 1e-4)
    say("case grid8x8 slices [0,32) + [32,64)")
    p = Q.Plan(text, w.upper_mask)
    p.run_halves(0, 32, bits)
    p.run_halves(32, 64, bits)
    a2, _ = p.amplitudes(bits, 0)
    p.close()
    assert_close(a2, a32.astype(np.complex128), 1e-5)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5, 100])
def test_two_cuts_on_one_qubit_in_one_level(level):
    """Interleaved columns put two cuts on one qubit at the same tree level:
    P0 P1 = 0 on the upper half and Z^b0 Z^b1 = Z^(b0 xor b1) on the lower half,
    in the branch passes and in the leaf evaluation alike."""
    Q = _lib()
    text = W.random_grid_circuit(2, 6, 12, 3)
    mask = W.grid_cols_mask(2, 6, [0, 2, 4])
    bits, _, _ = product_bitstrings(12, mask, 64, 64, 3, 4)
    ref = SV.simulate(OC.parse(text))[bits.astype(np.int64)]
    say(f"case same-qubit cuts materialize_level={level}")
    amp, _ = run_plan(Q, text, mask, bits, materialize_level=level, tail_max_qubits=10)
    assert_close(amp, ref, 1e-5)


def test_grid8x8_bands_32_qubit_halves():
    """64 qubits, 32+32 halves at full size (2^32-entry half states), copies
    [0, 64) of 65536, 2^20 bitstrings: every partial amplitude against the
    FP64 oracle.  The circuit leaves out the vertical bonds below rows 1 and
    5, so each half is an independent 16-qubit band times the 16 qubits next
    to the cut; the golden holds the oracle's factors (band state vectors and
    the cut block's partition over the same copies), and every state bit of
    the halves carries entangled amplitudes."""
    Q = _lib()
    import torch
    w = workload("grid8x8_d22_bands")
    g = _golden(w.name)
    bits, u, l = product_bitstrings(w.n, w.upper_mask, w.n_u, w.n_l, w.seed_u, w.seed_l)
    assert np.array_equal(g["u"], u.astype(np.int64)) and np.array_equal(g["l"], l.astype(np.int64))
    ref = (g["fu"][:, None] * (g["A"] @ g["B"].T) * g["fl"][None, :]).reshape(-1)
    say(f"case grid8x8 bands slice [{w.copy_begin},{w.copy_end}) m={bits.size}")
    p = Q.Plan(w.circuit_text(), w.upper_mask)
    assert (p.n_upper, p.n_lower, p.n_cuts) == (32, 32, 16)
    try:
        p.run_halves(w.copy_begin, w.copy_end, bits)
        for prec in (0, 1):
            say(f"case grid8x8 bands prec={prec}")
            amp, _ = p.amplitudes(bits, prec)
            assert_close(amp, ref, TOL[prec], what=f"prec {prec}")
    finally:
        p.close()
        torch.cuda.empty_cache()
