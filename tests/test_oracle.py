"""Pins of the FP64 oracle against what the paper and the mathematics fix."""

import os

import numpy as np
import pytest

from oracle import circuit as OC
from oracle import counting, dense, gates as G, partition as P, phases, statevector as SV
from workloads import circuits as W
from workloads.bitstrings import product_bitstrings

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append(line.split())
    return out


def circ(rows, cols, depth, seed=0):
    return OC.parse(W.random_grid_circuit(rows, cols, depth, seed))


# ---------------------------------------------------------------- gates

def test_gate_closed_forms():
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]])
    for m in (G.H, G.SX, G.SY, G.T):
        assert np.allclose(m.conj().T @ m, np.eye(2), atol=1e-15)
    assert np.allclose(G.SX @ G.SX, X, atol=1e-15)
    assert np.allclose(G.SY @ G.SY, Y, atol=1e-15)
    assert np.allclose(np.linalg.matrix_power(G.T, 8), np.eye(2), atol=1e-15)
    assert np.allclose(G.T[1, 1], (1 + 1j) / np.sqrt(2))
    # sqrt(Y)|0> is |+> and sqrt(X)|0> is (|0> - i|1>)/sqrt2, up to a phase
    plus = np.array([1, 1]) / np.sqrt(2)
    mi = np.array([1, -1j]) / np.sqrt(2)
    assert abs(abs(np.vdot(plus, G.SY[:, 0])) - 1) < 1e-15
    assert abs(abs(np.vdot(mi, G.SX[:, 0])) - 1) < 1e-15


def test_eq1_cut_identity():
    # CZ = P0 x I + P1 x Z on (control, target) = (high, low) Kronecker order
    lhs = G.CZ
    rhs = np.kron(G.P0, G.I2) + np.kron(G.P1, G.Z)
    assert np.array_equal(lhs, rhs)
    # symmetric in the two qubits
    rhs2 = np.kron(G.I2, G.P0) + np.kron(G.Z, G.P1)
    assert np.array_equal(lhs, rhs2)


# ---------------------------------------------------------------- full state

def test_statevector_small_closed_forms():
    c = OC.parse("qubits 2\n0 h 0\n0 h 1\n1 cz 0 1\n")
    assert np.allclose(SV.simulate(c), np.array([1, 1, 1, -1]) / 2, atol=1e-15)
    # qubit q is bit q of the index
    c = OC.parse("qubits 3\n0 sx 2\n")
    psi = SV.simulate(c)
    assert np.allclose(psi, [0.5 + 0.5j, 0, 0, 0, 0.5 - 0.5j, 0, 0, 0], atol=1e-15)
    c = OC.parse("qubits 3\n0 h 0\n1 t 0\n2 sy 1\n")
    psi = SV.simulate(c)
    expect = np.kron(G.SY[:, 0], np.array([1, (1 + 1j) / np.sqrt(2)]) / np.sqrt(2))
    assert np.allclose(psi[:4], expect, atol=1e-15)
    assert np.allclose(psi[4:], 0)


@pytest.mark.parametrize("rows,cols,depth,seed", [
    (2, 4, 8, 0), (2, 4, 12, 1), (2, 5, 10, 2), (3, 3, 16, 3), (2, 5, 16, 4), (2, 3, 9, 5),
])
def test_dense_bruteforce_matches_statevector(rows, cols, depth, seed):
    c = circ(rows, cols, depth, seed)
    a = dense.final_state(c)
    b = SV.simulate(c)
    assert np.max(np.abs(a - b)) < 1e-13
    assert abs(np.linalg.norm(b) - 1) < 1e-13


def test_statevector_unit_norm_larger():
    for (r, cc, d) in [(4, 4, 10), (4, 5, 12)]:
        psi = SV.simulate(circ(r, cc, d))
        assert abs(np.linalg.norm(psi) - 1) < 1e-13


# ---------------------------------------------------------------- Eq. 3-6

def test_fused_phase_equals_gates():
    rng = np.random.default_rng(7)
    n = 10
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    tq = [0, 3, 7, 9]
    edges = [(1, 2), (4, 8), (5, 6)]
    psi = psi0.copy()
    for q in tq:
        SV.apply_gate(psi, "t", (q,))
    for a, b in edges:
        SV.apply_gate(psi, "cz", (a, b))
    fused = phases.layer_phase(n, tq, edges) * psi0
    assert np.max(np.abs(fused - psi)) < 1e-14
    # closed forms of Eq. 4 and Eq. 6 at single indices
    d = phases.layer_phase(n, tq, edges)
    x = (1 << 0) | (1 << 3) | (1 << 4) | (1 << 8)   # two T qubits set, edge (4,8) set
    assert abs(d[x] - ((1 + 1j) / np.sqrt(2)) ** 2 * -1) < 1e-15
    # projectors and Z of Eq. 1
    psi = psi0.copy()
    SV.apply_gate(psi, "p1", (2,))
    SV.apply_gate(psi, "z", (5,))
    ref = phases.layer_phase(n, [], [], proj=[(2, 1)], zflip=[5]) * psi0
    assert np.max(np.abs(ref - psi)) < 1e-15


# ---------------------------------------------------------------- partition

def _all_bitstrings(n):
    return np.arange(1 << n, dtype=np.uint64)


@pytest.mark.parametrize("rows,cols,depth,mask", [
    (4, 4, 10, W.grid_rows_mask(4, 4, [0, 1])),
    (4, 4, 12, W.grid_cols_mask(4, 4, [0, 1])),
    (4, 5, 10, W.grid_rows_mask(4, 5, [0, 1])),
    (4, 4, 16, W.grid_rows_mask(4, 4, [0]) | 0b0011 << 4),     # staircase
    (2, 6, 12, W.grid_cols_mask(2, 6, [0, 2, 4])),              # interleaved columns
])
def test_partition_equals_full_state(rows, cols, depth, mask):
    c = circ(rows, cols, depth)
    n = rows * cols
    bits = _all_bitstrings(n)
    amp = P.amplitudes(c, mask, bits)
    psi = SV.simulate(c)
    assert np.max(np.abs(amp - psi)) < 1e-12
    assert len(P.find_cuts(c, mask)) > 0


def test_partition_full_size_sample_6x4():
    c = circ(6, 4, 16)
    mask = W.grid_rows_mask(6, 4, [0, 1, 2])
    bits, _, _ = product_bitstrings(24, mask, 16, 16, 5, 6)
    amp = P.amplitudes(c, mask, bits)
    psi = SV.simulate(c)
    assert np.max(np.abs(amp - psi[bits.astype(np.int64)])) < 1e-12


def test_prefix_recursion_equals_plain_copies():
    c = circ(4, 4, 10)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    ncut = len(P.find_cuts(c, mask))
    for upper in (True, False):
        S = P.half_states(c, mask, upper)
        for k in range(1 << ncut):
            ref = P.half_state_plain(c, mask, upper, k)
            assert np.max(np.abs(S[:, k] - ref)) < 1e-14


def test_eq1_per_cut_gate():
    # replacing one cut CZ by its two-branch sum reproduces the circuit
    c = circ(4, 4, 10)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    psi = SV.simulate(c)
    for cut in P.find_cuts(c, mask):
        tot = np.zeros_like(psi)
        for b in (0, 1):
            gates = []
            for g in c.gates:
                if g[1] == "cz" and g[0] == cut.cycle and set(g[2]) == {cut.upper, cut.lower}:
                    gates.append((g[0], "p1" if b else "p0", (cut.upper,)))
                    gates.append((g[0], "z" if b else "i", (cut.lower,)))
                else:
                    gates.append(g)
            s = SV.zero_state(c.n)
            for _, name, qs in gates:
                SV.apply_gate(s, name, qs)
            tot += s
        assert np.max(np.abs(tot - psi)) < 1e-14


def test_partition_invariants():
    c = circ(6, 4, 16)
    mask = W.grid_rows_mask(6, 4, [0, 1, 2])
    U = P.half_states(c, mask, True)
    L = P.half_states(c, mask, False)
    # P_0 + P_1 = I and the gates are unitary: the upper copies split the norm
    assert abs(np.sum(np.abs(U) ** 2) - 1) < 1e-12
    # Z is unitary: every lower copy keeps unit norm
    assert np.max(np.abs(np.linalg.norm(L, axis=0) - 1)) < 1e-12


def test_copy_slices_sum_to_whole():
    c = circ(4, 4, 12)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    bits = _all_bitstrings(16)[::37]
    total = 1 << len(P.find_cuts(c, mask))
    whole = P.amplitudes(c, mask, bits)
    parts = sum(P.amplitudes(c, mask, bits, a, min(a + 3, total)) for a in range(0, total, 3))
    assert np.max(np.abs(parts - whole)) < 1e-14


def test_sum_over_copies_alternate_cut_rule():
    # putting P on the lower endpoint and Z on the upper one changes U_k and
    # L_k but not their sum (CZ is symmetric); compare against the full state
    c = circ(4, 4, 10)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    lower_mask = ((1 << 16) - 1) & ~mask
    bits = _all_bitstrings(16)
    a1 = P.amplitudes(c, lower_mask, bits)   # swap the roles of the halves
    psi = SV.simulate(c)
    assert np.max(np.abs(a1 - psi)) < 1e-12


# ---------------------------------------------------------------- counting

def test_table2_cut_counts_56q():
    c = circ(8, 7, 38)
    mask = W.grid_rows_mask(8, 7, [0, 1, 2, 3])
    per = counting.cuts_per_cycle(c, mask)
    for lo, hi, in_range, total, ne in (map(int, r) for r in _rows("table2_56q_cuts.txt")):
        assert sum(per.get(t, 0) for t in range(lo, hi + 1)) == in_range
        assert sum(v for t, v in per.items() if t <= hi) == total
        assert counting.equivalent_qubits(28, total) == ne


def test_fig4_cz_totals():
    for n, r, cc, d, tot in (map(int, x) for x in _rows("fig4_cz_totals.txt")):
        c = circ(r, cc, d)
        assert sum(1 for g in c.gates if g[1] == "cz") == tot


def test_table1_eq2_estimates():
    per_gate = {28: 0.25, 32: 0.38, 36: 0.67}
    gates_after3 = {56: 8, 64: 10, 72: 12}
    unit = {"s": 1, "min": 60, "h": 3600, "d": 86400}
    for n, r, cc, d, val, u in _rows("table1_estimates.txt"):
        n, r, cc, d = int(n), int(r), int(cc), int(d)
        c = circ(r, cc, d)
        mask = W.grid_rows_mask(r, cc, range(r // 2))
        ncut = len(P.find_cuts(c, mask))
        est = counting.eq2_time(d, ncut, gates_after3[n], per_gate[n // 2], 24576) / unit[u]
        printed = float(val)
        # printed to three significant figures
        assert abs(est - printed) <= 0.5 * 10 ** (np.floor(np.log10(printed)) - 2) + 1e-12, (n, d, est, printed)


def test_fig1_example_counts():
    # an 8-qubit example with two cut CZ gates gives 4 copies, 8 half circuits
    # of 4 qubits and N_e = 7 (Sec. 2.1, Sec. 3)
    assert counting.equivalent_qubits(4, 2) == 7


# ---------------------------------------------------------------- controlled-U cuts (Supp. Eq. 1)

def test_supp_eq1_controlled_gates():
    """P0 x I + P1 x U for U = X, Y, Z against the textbook 4x4 matrices in
    the basis |control target> = 00, 01, 10, 11."""
    cnot = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    cy = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, -1j], [0, 0, 1j, 0]])
    cz = np.diag([1, 1, 1, -1]).astype(complex)
    for name, ref in (("cx", cnot), ("cy", cy), ("cz", cz)):
        got = np.kron(G.P0, G.I2) + np.kron(G.P1, G.CONTROLLED_U[name])
        assert np.array_equal(got, ref), name


def test_controlled_gates_in_statevector():
    """CNOT on |+>|0> is the Bell state; CY maps |1>|0> to i|1>|1>; both are
    involutions; the target may sit above or below the control."""
    psi = SV.zero_state(2)
    SV.apply_gate(psi, "h", (1,))
    SV.apply_gate(psi, "cx", (1, 0))
    assert np.allclose(psi, [2 ** -0.5, 0, 0, 2 ** -0.5], atol=1e-15)
    psi = SV.zero_state(3)
    SV.apply_gate(psi, "h", (0,))
    SV.apply_gate(psi, "cx", (0, 2))
    assert np.allclose(psi[[0, 5]], [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    psi = np.zeros(4, dtype=complex)
    psi[0b01] = 1  # control (qubit 0) = 1, target (qubit 1) = 0
    SV.apply_gate(psi, "cy", (0, 1))
    assert np.allclose(psi, [0, 0, 0, 1j], atol=1e-15)
    rng = np.random.default_rng(7)
    for name in ("cx", "cy"):
        v = rng.normal(size=32) + 1j * rng.normal(size=32)
        w = v.copy()
        SV.apply_gate(w, name, (3, 1))
        assert not np.allclose(w, v)
        SV.apply_gate(w, name, (3, 1))
        assert np.allclose(w, v, atol=1e-14)


@pytest.mark.parametrize("two_qubit,seed", [("cx", 0), ("cy", 1), ("mixed", 2)])
def test_controlled_dense_bruteforce(two_qubit, seed):
    c = OC.parse(W.random_grid_circuit(3, 3, 12, seed, two_qubit))
    assert any(g[1] == two_qubit or (two_qubit == "mixed" and g[1] in ("cx", "cy")) for g in c.gates)
    assert np.allclose(SV.simulate(c), dense.final_state(c), atol=1e-12)


@pytest.mark.parametrize("rows,cols,depth,two_qubit,orient,seed,mask", [
    (4, 4, 12, "cx", "random", 6, W.grid_rows_mask(4, 4, [0, 1])),
    (4, 4, 12, "cy", "random", 5, W.grid_cols_mask(4, 4, [0, 1])),
    (3, 5, 14, "mixed", "random", 5, W.grid_rows_mask(3, 5, [0]) | 0b11 << 5),
    (4, 5, 10, "mixed", "low", 5, W.grid_rows_mask(4, 5, [0, 1])),
])
def test_partition_controlled_equals_full_state(rows, cols, depth, two_qubit, orient, seed, mask):
    """Supp. Eq. 1 cuts (P_b on the control, U^b on the target, either half)
    summed over copies give the full-state amplitudes."""
    c = OC.parse(W.random_grid_circuit(rows, cols, depth, seed, two_qubit, orient))
    cuts = P.find_cuts(c, mask)
    assert any(k.gate != "cz" for k in cuts)
    if orient == "random":
        # both orientations occur among the cut gates
        sides = {k.control == k.upper for k in cuts if k.gate != "cz"}
        assert sides == {True, False}
    n = rows * cols
    x = np.arange(1 << n)
    assert np.allclose(P.amplitudes(c, mask, x), SV.simulate(c), atol=1e-12)


def test_controlled_prefix_recursion_equals_plain_copies():
    c = OC.parse(W.random_grid_circuit(3, 4, 12, 6, "mixed"))
    mask = W.grid_rows_mask(3, 4, [0])
    ncut = len(P.find_cuts(c, mask))
    assert ncut >= 3
    for upper in (True, False):
        tree = P.half_states(c, mask, upper)
        for k in range(1 << ncut):
            plain = P.half_state_plain(c, mask, upper, k)
            assert np.allclose(tree[:, k], plain, atol=1e-13)


# ---------------------------------------------------------------- partitions into t parts (Sec. 3, Fig. 3)

def _bands(rows, cols, bands):
    return [W.grid_rows_mask(rows, cols, b) for b in bands]


@pytest.mark.parametrize("rows,cols,depth,bands,two_qubit", [
    (6, 3, 10, [[0, 1], [2, 3], [4, 5]], "cz"),
    (8, 2, 12, [[0, 1], [2, 3], [4, 5], [6, 7]], "cz"),
    (6, 3, 10, [[0], [1, 2, 3], [4, 5]], "mixed"),
])
def test_multipart_equals_full_state(rows, cols, depth, bands, two_qubit):
    from oracle import multipart as MP
    c = OC.parse(W.random_grid_circuit(rows, cols, depth, 1, two_qubit))
    masks = _bands(rows, cols, bands)
    cuts = MP.chain_cuts(c, masks)
    assert {k.lo_part for k in cuts} == set(range(len(bands) - 1))  # every link is cut
    x = np.random.default_rng(3).integers(0, 1 << (rows * cols), size=2000)
    assert np.allclose(MP.amplitudes(c, masks, x), SV.simulate(c)[x], atol=1e-12)


def test_multipart_two_parts_is_the_two_part_scheme():
    """t = 2: part 0 carries P_b, part 1 Z^b, copy for copy as in Sec. 2.1."""
    from oracle import multipart as MP
    c = circ(4, 4, 12, 2)
    m = W.grid_rows_mask(4, 4, [0, 1])
    for p, upper in ((0, True), (1, False)):
        assert np.array_equal(MP.part_states(c, [m, 0xFFFF & ~m], p), P.half_states(c, m, upper))


def test_multipart_rejects_non_chains():
    from oracle import multipart as MP
    c = circ(6, 3, 10, 1)
    with pytest.raises(ValueError, match="chain"):
        MP.chain_cuts(c, _bands(6, 3, [[0, 1], [4, 5], [2, 3]]))
    with pytest.raises(ValueError):
        MP.chain_cuts(c, _bands(6, 3, [[0, 1], [2, 3]]))  # qubits left out
