"""CPU checks of the cut score and the cut chooser (qs_score_cut, qs_choose_cut).

The cut count and the equivalent qubits are pinned to the paper's Table 2 (the
56-qubit circuit cut between rows 3 and 4, at every depth the table lists);
the half sizes and cut counts of other masks to the oracle's partition; the
flat Eq. 2-style update count to a count written here from the oracle's parsed
gates; and the chooser to the minimum of the individual scores.
"""

import os

import numpy as np
import pytest

import paper_1802_06952_amd as Q
from oracle import circuit as OC, partition as P
from workloads import circuits as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _score(text, mask, n_values=256):
    c = Q.qs_load_circuit(text)
    try:
        return Q.qs_score_cut(c, mask, n_values)
    finally:
        Q.qs_circuit_free(c)


def test_table2_cuts_and_equivalent_qubits():
    """Table 2: cut gates up to each depth and N_e of the 56-qubit circuit."""
    mask = W.grid_rows_mask(8, 7, [0, 1, 2, 3])
    for lo, hi, in_range, total, ne in (map(int, r) for r in _rows("table2_56q_cuts.txt")):
        if total == 0 or hi > 22:
            continue  # depth 22 is the deepest circuit the planner is asked to cost here
        sc = _score(W.random_grid_circuit(8, 7, hi, 0), mask)
        assert sc["n_cuts"] == total, (hi, sc)
        assert sc["n_upper"] == sc["n_lower"] == 28
        assert sc["equivalent_qubits"] == ne, (hi, sc)


def _flat_updates(oc, mask, c):
    """Every copy runs every gate of each half on its full state."""
    n = oc.n
    g = [0, 0]
    for _, _, qs in oc.gates:
        sides = {0 if (mask >> q) & 1 else 1 for q in qs}
        for s in sides:
            g[s] += 1
    nu = bin(mask).count("1")
    return float(2 ** c) * (g[0] * 2.0 ** nu + g[1] * 2.0 ** (n - nu))


@pytest.mark.parametrize("rows,cols,depth,seed,mask_fn", [
    (4, 5, 16, 1, lambda: W.grid_rows_mask(4, 5, [0, 1])),
    (6, 7, 20, 0, lambda: W.grid_cols_mask(6, 7, [0, 1, 2])),
    (5, 6, 12, 2, lambda: W.grid_rows_mask(5, 6, [0]) | 0b111),
    (3, 4, 10, 3, lambda: 0b1),
])
def test_score_against_oracle(rows, cols, depth, seed, mask_fn):
    text = W.random_grid_circuit(rows, cols, depth, seed)
    mask = mask_fn()
    oc = OC.parse(text)
    c = len(P.find_cuts(oc, mask))
    nu = bin(mask).count("1")
    sc = _score(text, mask)
    assert sc["n_cuts"] == c
    assert (sc["n_upper"], sc["n_lower"]) == (nu, oc.n - nu)
    assert sc["equivalent_qubits"] == max(nu, oc.n - nu) + c + 1
    assert sc["flat_updates"] == _flat_updates(oc, mask, c)
    assert 0 < sc["plan_cost"] < float("inf")


def test_plan_cost_grows_with_requested_values():
    text = W.random_grid_circuit(6, 7, 20, 0)
    mask = W.grid_rows_mask(6, 7, [0, 1, 2])
    costs = [_score(text, mask, v)["plan_cost"] for v in (16, 256, 4096)]
    assert costs[0] < costs[1] < costs[2]


def test_choose_cut_is_the_minimum_score():
    text = W.random_grid_circuit(6, 7, 20, 0)
    masks = ([W.grid_rows_mask(6, 7, list(range(j + 1))) for j in range(5)] +
             [W.grid_cols_mask(6, 7, list(range(j + 1))) for j in range(6)] +
             [(1 << k) - 1 for k in (17, 19, 23)])
    c = Q.qs_load_circuit(text)
    try:
        scores = []
        for m in masks:
            try:
                scores.append(Q.qs_score_cut(c, m, 1024))
            except Q.QSError:
                scores.append(None)
        assert any(s is None for s in scores)  # halves over 32 qubits are skipped
        for crit, key in ((0, "flat_updates"), (1, "plan_cost")):
            best, sc = Q.qs_choose_cut(c, masks, 1024, crit)
            vals = [s[key] if s else np.inf for s in scores]
            assert best == int(np.argmin(vals))
            assert sc == scores[best]
        # both criteria pick the equal halves of the paper's 42-qubit run (rows 0-2)
        assert Q.qs_choose_cut(c, masks, 1024, 0)[0] == 2
        assert Q.qs_choose_cut(c, masks, 1024, 1)[0] == 2
    finally:
        Q.qs_circuit_free(c)


def test_choose_cut_errors():
    c = Q.qs_load_circuit(W.random_grid_circuit(3, 4, 8, 0))
    try:
        for args in (([], 16, 0), ([0b11], 0, 0), ([0b11], 16, 2)):
            with pytest.raises(Q.QSError) as e:
                Q.qs_choose_cut(c, *args)
            assert e.value.status == -1
        with pytest.raises(Q.QSError) as e:
            Q.qs_choose_cut(c, [0, (1 << 12) - 1], 16, 0)  # empty and full masks only
        assert e.value.status == -3
        with pytest.raises(Q.QSError) as e:
            Q.qs_score_cut(c, 0b11, 0)
        assert e.value.status == -1
    finally:
        Q.qs_circuit_free(c)
