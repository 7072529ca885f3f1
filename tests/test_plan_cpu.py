"""CPU checks of the library's host side: exported symbols, the partition, and
the copy-tree schedule.

The schedule test replays the plan the library prints (initial product
state, tree levels with their branch factors, cuts applied at the output) with
a small numpy interpreter written here, and compares every copy's half state
with the oracle.  No GPU is involved: only the planner's reordering of the
half programs is under test.
"""

import os
import re

import numpy as np
import pytest

import paper_1802_06952_amd as Q
from oracle import circuit as OC, partition as P, statevector as SV
from workloads import CONFIGS, circuits as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "qs.h")


def test_library_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(qs_[a-z_]+)\s*\(", text))
    assert declared, "no declarations found"
    lib = Q.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(Q.EXPORTED)


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding against the C header, compiled by
    gcc: size and field offsets of qs_options, qs_allocator and qs_cut_score."""
    import ctypes
    import subprocess
    src = tmp_path / "layout.c"
    fields = {"qs_options": [f for f, _ in Q.qs_options._fields_],
              "qs_allocator": [f for f, _ in Q.qs_allocator._fields_],
              "qs_cut_score": [f for f, _ in Q.qs_cut_score._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for fld in fs:
            lines.append(f'  printf("{st} {fld} %zu\\n", offsetof({st}, {fld}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        st, key, val = ln.split()
        got[(st, key)] = int(val)
    for st, fs in fields.items():
        cls = getattr(Q, st)
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for fld in fs:
            assert got[(st, fld)] == getattr(cls, fld).offset, (st, fld)


def test_copies_per_launch_blocks():
    """copies_per_launch caps the block the dump (and qs_run_halves) takes;
    it must be a power of two."""
    text = W.random_grid_circuit(4, 4, 16, 1)
    mask = W.grid_rows_mask(4, 4, [0, 1])
    p = Q.Plan(text, mask, alloc=None)
    c = p.n_cuts
    assert p.dump()["block"] == {"k0": 0, "p": 0}
    p.close()
    p = Q.Plan(text, mask, copies_per_launch=4, alloc=None)
    assert p.dump()["block"] == {"k0": 0, "p": c - 2}
    p.close()
    with pytest.raises(Q.QSError) as e:
        Q.Plan(text, mask, copies_per_launch=6, alloc=None)
    assert e.value.status == -1


def test_parse_errors():
    for bad in ["", "qubits 0\n", "qubits 65\n", "qubits 2\n0 cz 0 0\n", "qubits 2\n0 h 2\n",
                "qubits 2\n1 h 0\n0 h 1\n", "qubits 2\n0 h 0\n0 t 0\n", "qubits 2\n0 foo 1\n",
                "0 h 0\n"]:
        with pytest.raises(Q.QSError) as e:
            Q.qs_load_circuit(bad)
        assert e.value.status == -2
    c = Q.qs_load_circuit("qubits 3 # three\n0 h 0\n0 h 1\n1 cz 0 1\n")
    assert Q.qs_circuit_info(c) == (3, 3)
    Q.qs_circuit_free(c)


def test_partition_errors():
    text = W.random_grid_circuit(4, 4, 10, 0)
    c = Q.qs_load_circuit(text)
    for mask in (0, (1 << 16) - 1, 1 << 16):
        with pytest.raises(Q.QSError) as e:
            Q.qs_partition(c, mask)
        assert e.value.status == -1
    Q.qs_circuit_free(c)


@pytest.mark.parametrize("name", list(CONFIGS))
def test_partition_matches_oracle_cuts(name):
    w = CONFIGS[name]
    text = w.circuit_text()
    p = Q.Plan(text, w.upper_mask)
    d = p.dump()
    oc = OC.parse(text)
    cuts = P.find_cuts(oc, w.upper_mask)
    assert p.n_cuts == len(cuts)
    assert [tuple(x) for x in d["cuts"]] == [(k.cycle, k.upper, k.lower) for k in cuts]
    full = (1 << w.n) - 1
    assert d["sides"][0]["qubits"] == P.half_qubits(w.n, w.upper_mask)
    assert d["sides"][1]["qubits"] == P.half_qubits(w.n, full & ~w.upper_mask)
    for s in d["sides"]:
        # every op runs at exactly one tree level
        if "levels" in s:
            seen = sorted(i for lv in s["levels"] for i in lv["ops"])
            ncut_ops = sum(1 for o in s["ops"] if o[0] == "cut")
            assert len(seen) == len(set(seen)) == len(s["ops"]) - ncut_ops


# ---------------------------------------------------------------- schedule replay

SQ = np.sqrt(0.5)
MATS = {"h": np.array([[SQ, SQ], [SQ, -SQ]], dtype=complex),
        "sx": 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]]),
        "sy": 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]])}


def _bit(n, q):
    return (np.arange(1 << n) >> q) & 1


def _apply(psi, n, op):
    name, q0, q1 = op[0], op[1], op[2]
    if name in MATS:
        m = MATS[name]
        b = _bit(n, q0)
        i0 = np.nonzero(b == 0)[0]
        i1 = i0 | (1 << q0)
        a0, a1 = psi[i0].copy(), psi[i1].copy()
        psi[i0] = m[0, 0] * a0 + m[0, 1] * a1
        psi[i1] = m[1, 0] * a0 + m[1, 1] * a1
    elif name[0] == "t":  # "t" or "t<k>" = T^k
        k = int(name[1:]) if len(name) > 1 else 1
        psi *= np.where(_bit(n, q0) == 1, ((1 + 1j) * SQ) ** k, 1.0)
    elif name == "cz":
        psi *= np.where((_bit(n, q0) & _bit(n, q1)) == 1, -1.0, 1.0)
    else:
        raise AssertionError(op)


def _cut_factor(psi, n, q, b, upper):
    if upper:
        psi *= (_bit(n, q) == b)
    elif b:
        psi *= np.where(_bit(n, q) == 1, -1.0, 1.0)


def replay(side, cuts, c):
    n = side["n"]
    qubits = side["qubits"]
    upper = side["upper"]
    loc = {g: i for i, g in enumerate(qubits)}
    cq = [loc[(k[1] if upper else k[2])] for k in cuts]
    psi0 = np.zeros(1 << n, dtype=complex)
    h = side["hinit"]
    x = np.arange(1 << n)
    psi0[(x & ~h) == 0] = 2.0 ** (-bin(h).count("1") / 2)
    out = np.zeros((1 << n, 1 << c), dtype=complex)
    levels = side["levels"]

    def rec(psi, li, k):
        if li == len(levels):
            ends = side["end_cuts"]
            for e in range(1 << len(ends)):
                s = psi.copy()
                kk = k
                for i, j in enumerate(ends):
                    b = (e >> (len(ends) - 1 - i)) & 1
                    _cut_factor(s, n, cq[j], b, upper)
                    kk |= b << (c - 1 - j)
                out[:, kk] = s
            return
        lv = levels[li]
        m = len(lv["cuts"])
        for b in range(1 << m):
            s = psi.copy()
            kk = k
            for i, j in enumerate(lv["cuts"]):
                bb = (b >> (m - 1 - i)) & 1
                _cut_factor(s, n, cq[j], bb, upper)
                kk |= bb << (c - 1 - j)
            for oi in lv["ops"]:
                _apply(s, n, side["ops"][oi])
            rec(s, li + 1, kk)

    rec(psi0, 0, 0)
    return out


@pytest.mark.parametrize("rows,cols,depth,mask", [
    (4, 4, 10, W.grid_rows_mask(4, 4, [0, 1])),
    (4, 4, 16, W.grid_cols_mask(4, 4, [0, 1])),
    (3, 4, 18, W.grid_rows_mask(3, 4, [0]) | 0b0011 << 4),
    (2, 6, 12, W.grid_cols_mask(2, 6, [0, 2, 4])),
])
def test_tree_schedule_replays_to_oracle(rows, cols, depth, mask):
    text = W.random_grid_circuit(rows, cols, depth, 3)
    p = Q.Plan(text, mask)
    d = p.dump()
    oc = OC.parse(text)
    c = p.n_cuts
    assert c > 0
    for si, upper in enumerate((True, False)):
        side = d["sides"][si]
        got = replay(side, d["cuts"], c)
        ref = P.half_states(oc, mask, upper)
        assert np.max(np.abs(got - ref)) < 1e-12


def _run_op(psi, side, cq, oi, fixed):
    """One half op; a cut op inside an op list is a cut fixed by the block."""
    op = side["ops"][oi]
    if op[0] == "cut":
        _cut_factor(psi, side["n"], cq[op[3]], fixed(op[3]), side["upper"])
    else:
        _apply(psi, side["n"], op)


def _level_states(side, cuts, upto, fixed):
    """States of every node of tree levels 0..upto, level by level."""
    n = side["n"]
    loc = {g: i for i, g in enumerate(side["qubits"])}
    cq = [loc[(k[1] if side["upper"] else k[2])] for k in cuts]
    h = side["hinit"]
    x = np.arange(1 << n)
    psi0 = np.zeros(1 << n, dtype=complex)
    psi0[(x & ~h) == 0] = 2.0 ** (-bin(h).count("1") / 2)
    levels = side["levels"]
    cur = {0: psi0}
    for oi in levels[0]["ops"]:
        _run_op(cur[0], side, cq, oi, fixed)
    for li in range(1, upto + 1):
        lv = levels[li]
        m = len(lv["cuts"])
        nxt = {}
        for node, psi in cur.items():
            for b in range(1 << m):
                s = psi.copy()
                for i, j in enumerate(lv["cuts"]):
                    _cut_factor(s, n, cq[j], (b >> (m - 1 - i)) & 1, side["upper"])
                for oi in lv["ops"]:
                    _run_op(s, side, cq, oi, fixed)
                nxt[(node << m) | b] = s
        cur = nxt
    return cur, cq


def _pass_states(side, cq, fixed):
    """States of the last materialised level as the passes compute them: each
    pass runs ops_in on every node of its level, then descends one level per
    branch stage (cut factors of that level's cuts, then the stage's ops)."""
    n = side["n"]
    levels = side["levels"]
    h = side["hinit"]
    x = np.arange(1 << n)
    cur = None
    for pp in side["passes"]:
        li = pp["level_in"]
        if pp["init"]:
            psi0 = np.zeros(1 << n, dtype=complex)
            psi0[(x & ~h) == 0] = 2.0 ** (-bin(h).count("1") / 2)
            cur = {0: psi0}
        for psi in cur.values():
            for oi in pp["ops_in"]:
                _run_op(psi, side, cq, oi, fixed)
        for st, so in enumerate(pp["stages"]):
            lv = levels[li + st + 1]
            m = len(lv["cuts"])
            nxt = {}
            for node, psi in cur.items():
                for b in range(1 << m):
                    s = psi.copy()
                    for i, j in enumerate(lv["cuts"]):
                        _cut_factor(s, n, cq[j], (b >> (m - 1 - i)) & 1, side["upper"])
                    for oi in so:
                        _run_op(s, side, cq, oi, fixed)
                    nxt[(node << m) | b] = s
            cur = nxt
    return cur


@pytest.mark.parametrize("rows,cols,depth,mask,kw", [
    (4, 4, 12, W.grid_rows_mask(4, 4, [0, 1]), {}),
    (4, 4, 16, W.grid_cols_mask(4, 4, [0, 1]), {"tile_bits": 7}),
    (3, 6, 16, W.grid_rows_mask(3, 6, [0]), {"tile_bits": 7, "materialize_level": 6}),
    (4, 5, 14, W.grid_rows_mask(4, 5, [0, 1]), {"tile_bits": 8, "materialize_level": 4}),
    (2, 6, 12, W.grid_cols_mask(2, 6, [0, 2, 4]), {"materialize_level": 3}),
    (4, 5, 14, W.grid_rows_mask(4, 5, [0, 1]), {"plain": True}),
])
def test_pass_schedule_matches_tree_levels(rows, cols, depth, mask, kw):
    """Every op of the materialised levels runs exactly once, in an order the
    tree allows, when the passes (with their multi-level branch stages) are
    replayed: the last materialised level comes out as the level-by-level
    replay gives it, node for node."""
    text = W.random_grid_circuit(rows, cols, depth, 5)
    p = Q.Plan(text, mask, **kw)
    d = p.dump(0, 1 << p.n_cuts)
    p.close()
    for side in d["sides"]:
        ls = side["lstar"]
        every = [i for lv in side["levels"][: ls + 1] for i in lv["ops"]]
        ran = [i for pp in side["passes"] for i in pp["ops_in"] + [j for so in pp["stages"] for j in so]]
        assert sorted(ran) == sorted(every)
        assert all(pp["level_in"] + pp["branch"] <= ls for pp in side["passes"])
        c = len(d["cuts"])
        k0 = d["block"]["k0"]
        fixed = lambda j: (k0 >> (c - 1 - j)) & 1
        ref, cq = _level_states(side, d["cuts"], ls, fixed)
        got = _pass_states(side, cq, fixed)
        assert sorted(got) == sorted(ref)
        for k in ref:
            assert np.max(np.abs(got[k] - ref[k])) < 1e-12


def test_multi_level_passes_are_used():
    """On the 42-qubit workload the planner lands the passes two levels apart
    where the ops fit, so fewer tree levels are written than materialised."""
    from workloads import workload
    w = workload("grid6x7_d20")
    p = Q.Plan(w.circuit_text(), w.upper_mask)
    d = p.dump(0, 1 << p.n_cuts)
    one = Q.Plan(w.circuit_text(), w.upper_mask, max_stages=1).dump(0, 1 << p.n_cuts)
    p.close()
    for s2, s1 in zip(d["sides"], one["sides"]):
        assert max(pp["branch"] for pp in s2["passes"]) == 2
        assert max(pp["branch"] for pp in s1["passes"]) == 1
        written = {pp["level_in"] + pp["branch"] for pp in s2["passes"] if pp["branch"]}
        assert len(written) < s2["lstar"]


X_WAVE_BITS = 3  # wave bits of an exchange group's workgroup tile


@pytest.mark.parametrize("name,knobs", [
    ("grid6x7_d20", {}),
    ("grid6x6_d16", {"tile_bits": 9}),
    ("grid8x8_d22_slice64", {"tile_bits": 11}),
])
def test_exchange_groups_are_well_formed(name, knobs):
    """Every exchange group in the dump: consecutive phases without a branch
    on one level, each phase's tile is the six lane bits plus R register bits
    of the group's R + 3 bits, every 2x2 gate of a phase acts on its tile, the
    first phase alone may start from the product state, and no group ends a
    side's schedule.  With no_exchange every pass stands alone and the ops are
    the same, in the same order."""
    from workloads import workload
    w = workload(name)
    p = Q.Plan(w.circuit_text(), w.upper_mask, **knobs)
    k1 = w.copy_end if w.copy_end is not None else (1 << p.n_cuts)
    d = p.dump(w.copy_begin, k1)
    p.close()
    q = Q.Plan(w.circuit_text(), w.upper_mask, no_exchange=True, **knobs)
    d0 = q.dump(w.copy_begin, k1)
    q.close()
    groups = 0
    for s, s0 in zip(d["sides"], d0["sides"]):
        ps = s["passes"]
        assert all(pp["xg"] == 1 for pp in s0["passes"])
        flat = [i for pp in ps for st in [pp["ops_in"]] + pp["stages"] for i in st]
        flat0 = [i for pp in s0["passes"] for st in [pp["ops_in"]] + pp["stages"] for i in st]
        assert sorted(flat) == sorted(flat0)
        assert ps[-1]["xg"] == 1
        i = 0
        while i < len(ps):
            G = ps[i]["xg"]
            assert G >= 1
            if G == 1:
                i += 1
                continue
            groups += 1
            R = len(ps[i]["tile"]) - 6
            U = set()
            for k in range(i, i + G):
                pp = ps[k]
                assert pp["xg"] == (G if k == i else 0)
                assert pp["branch"] == 0 and pp["level_in"] == ps[i]["level_in"]
                assert pp["init"] == (k == 0 and ps[i]["init"] == 1) or pp["init"] == 0
                t = pp["tile"]  # local qubit ids; perm gives their state bits
                tb = sorted(s["perm"][x] for x in t)
                assert tb[:6] == list(range(6)) and len(tb) == 6 + R and len(set(tb)) == len(tb)
                U |= set(tb[6:])
                for op in pp["ops_in"]:
                    o = s["ops"][op]
                    if o[0] in ("h", "sx", "sy"):
                        assert o[1] in t
            assert len(U) <= R + X_WAVE_BITS
            i += G
    assert groups >= 1


@pytest.mark.parametrize("rows,cols,depth,two_qubit,mask", [
    (4, 4, 12, "cx", W.grid_rows_mask(4, 4, [0, 1])),
    (4, 4, 14, "cy", W.grid_rows_mask(4, 4, [0])),
    (3, 5, 16, "mixed", W.grid_rows_mask(3, 5, [0])),
])
def test_controlled_u_schedule_replays_to_oracle(rows, cols, depth, two_qubit, mask):
    """Controlled-U cuts whose control is in the upper half: every copy of
    both halves equals the oracle's Supp. Eq. 1 split."""
    text = W.random_grid_circuit(rows, cols, depth, 4, two_qubit, "low")
    p = Q.Plan(text, mask)
    d = p.dump()
    oc = OC.parse(text)
    c = p.n_cuts
    assert [tuple(x) for x in d["cuts"]] == [(k.cycle, k.upper, k.lower) for k in P.find_cuts(oc, mask)]
    assert any(k.gate != "cz" for k in P.find_cuts(oc, mask))
    for si, upper in enumerate((True, False)):
        got = replay(d["sides"][si], d["cuts"], c)
        ref = P.half_states(oc, mask, upper)
        assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("two_qubit,mask", [
    ("cx", W.grid_rows_mask(4, 4, [0, 1])),
    ("mixed", W.grid_cols_mask(4, 4, [0, 1])),
])
def test_controlled_u_any_orientation_sums_to_oracle(two_qubit, mask):
    """Controls on either side: the copies may differ from the oracle's split
    (the mirrored one), their sum over copies may not."""
    text = W.random_grid_circuit(4, 4, 12, 8, two_qubit, "random")
    p = Q.Plan(text, mask)
    d = p.dump()
    oc = OC.parse(text)
    c = p.n_cuts
    U = replay(d["sides"][0], d["cuts"], c)
    L = replay(d["sides"][1], d["cuts"], c)
    x = np.arange(1 << 16)
    u = P.pack_bits(x, P.half_qubits(16, mask))
    lo = P.pack_bits(x, P.half_qubits(16, ((1 << 16) - 1) & ~mask))
    amp = np.einsum("ik,ik->i", U[u], L[lo])
    assert np.max(np.abs(amp - SV.simulate(oc))) < 1e-12


def test_controlled_u_counts_written_gates():
    c = Q.qs_load_circuit("qubits 3\n0 h 0\n1 cx 0 1\n2 cy 1 2\n")
    try:
        assert Q.qs_circuit_info(c) == (3, 3)
    finally:
        Q.qs_circuit_free(c)


def test_binding_maps_one_hip_runtime():
    """Importing the binding first (before torch) still leaves one HIP and one
    HSA runtime in the process: torch's, which the library binds to."""
    import subprocess
    import sys
    code = ("import paper_1802_06952_amd, torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}),"
            " len({l.split()[-1] for l in maps if 'libhsa-runtime64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"]


def test_failed_partition_frees_the_circuit_once():
    """A plan whose partition is rejected releases its circuit exactly once
    (a second release would corrupt the heap of this process)."""
    import gc
    text = W.random_grid_circuit(6, 4, 12, 1)
    for _ in range(3):
        with pytest.raises(Q.QSError):
            Q.Plan(text, 0)
        with pytest.raises(Q.QSError):
            Q.ChainPlan(text, [W.grid_rows_mask(6, 4, b) for b in ([0, 1], [4, 5], [2, 3])])
        gc.collect()
    p = Q.Plan(text, W.grid_rows_mask(6, 4, [0, 1, 2]))
    assert p.n_cuts > 0
    p.close()


@pytest.mark.parametrize("rows,cols,depth,bands", [
    (6, 4, 12, [[0, 1], [2, 3], [4, 5]]),
    (8, 8, 10, [[0, 1], [2, 3], [4, 5], [6, 7]]),
    (5, 4, 12, [[0], [1, 2], [3, 4]]),
])
def test_chain_partition_against_oracle(rows, cols, depth, bands):
    """Part sizes and cuts per link of qs_partition_chain equal the oracle's
    chain partition (Sec. 3, Fig. 3)."""
    from oracle import multipart as MP
    text = W.random_grid_circuit(rows, cols, depth, 0)
    masks = [W.grid_rows_mask(rows, cols, b) for b in bands]
    cuts = MP.chain_cuts(OC.parse(text), masks)
    cp = Q.ChainPlan(text, masks)
    try:
        assert cp.t == len(bands)
        assert cp.part_qubits == [len(b) * cols for b in bands]
        assert cp.link_cuts == [sum(1 for k in cuts if k.lo_part == i) for i in range(len(bands) - 1)]
    finally:
        cp.close()


def test_chain_partition_errors():
    text = W.random_grid_circuit(4, 3, 8, 0)
    rows = [W.grid_rows_mask(4, 3, [r]) for r in range(4)]
    c = Q.qs_load_circuit(text)
    try:
        for masks, status in (([rows[0] | rows[1], rows[1] | rows[2], rows[3]], -1),  # overlap
                              ([rows[0], rows[1], rows[2]], -1),                      # a row left out
                              ([rows[0], 0, rows[1] | rows[2] | rows[3]], -1),        # empty part
                              ([rows[0]], -1),                                        # t = 1
                              ([rows[0], rows[2], rows[1], rows[3]], -3)):            # not a chain
            with pytest.raises(Q.QSError) as e:
                Q.qs_partition_chain(c, masks)
            assert e.value.status == status, masks
    finally:
        Q.qs_circuit_free(c)
