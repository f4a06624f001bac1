"""Pins of the check-generation oracle (oracle/checks.py): a hand-traced run of
Algorithm 4, the paper's worked set-XOR example, the GF(2) invariant
B L = B', independence of the check #3 groups, payload identities, and local
repair against brute force."""

import json
import os

import numpy as np
import pytest

from oracle import checks, codec, gf2, graph
from synth import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def G_of(k, n, **kw):
    kw.setdefault("dist", "rsd")
    return graph.build(graph.GraphParams(k=k, n=n, **kw))


def test_hand_traced_run():
    # B = [C0: {D0}, C1: {D1}, C2: {D0, D1}].  Column 2 first absorbs column 0
    # (weight 2 -> 1) and then column 1 (weight 1 -> 0): one zero column =
    # n - k ends the loop after the first sweep.
    G = graph.from_rows(2, [[0], [1], [0, 1]])
    b, L, sweeps = checks.cga(G)
    assert b == [0b01, 0b10, 0] and L == [0b001, 0b010, 0b111] and sweeps == 1
    check2, check3 = checks.split(b, L)
    assert check2 == {0: [0], 1: [1]} and check3 == [[0, 1, 2]]


def test_paper_worked_set_xor_example():
    with open(os.path.join(GOLDEN, "paper_eq1_4.json")) as fh:
        g = json.load(fh)
    c2 = g["check2"]
    assert checks.set_xor([c2["D0"], c2["D1"], c2["D2"]]) == g["check3"]


@pytest.mark.parametrize("k,n,seed,dist", [(20, 30, 1, "rsd"), (40, 70, 2, "rsd"), (30, 45, 3, "raptor"),
                                           (60, 80, 4, "rsd")])
def test_columns_stay_sums_of_original_columns(k, n, seed, dist):
    # every step XORs column i into column j in B and in L alike, so at the
    # end B' = B L over GF(2) with L invertible
    G = G_of(k, n, seed=seed, dist=dist)
    b, L, _ = checks.cga(G)
    B = gf2.dense_B(G).astype(np.int64)
    Lm = np.array([[(L[j] >> s) & 1 for j in range(n)] for s in range(n)], dtype=np.int64)
    Bp = np.array([[(b[j] >> i) & 1 for j in range(n)] for i in range(k)], dtype=np.int64)
    assert np.array_equal((B @ Lm) % 2, Bp)
    assert gf2.rank(Lm.astype(np.uint8), list(range(n))) == n
    check2, check3 = checks.split(b, L)
    zero = [j for j in range(n) if b[j] == 0]
    assert len(check3) == len(zero) <= n - gf2.rank(gf2.dense_B(G), list(range(n)))
    # the groups are independent vectors of the null space
    if check3:
        V = np.zeros((n, len(check3)), dtype=np.uint8)
        for q, grp in enumerate(check3):
            V[grp, q] = 1
        assert gf2.rank(V, list(range(len(check3)))) == len(check3)
    assert [len(g_) for g_ in check3] == sorted(len(g_) for g_ in check3)


def test_checks_hold_on_payloads():
    G = G_of(40, 70, seed=2)
    x = gen.payload(0, 5, 40, 32)
    c = codec.encode(G, x)
    b, L, _ = checks.cga(G)
    check2, check3 = checks.split(b, L)
    assert check2 and check3
    for i, members in check2.items():
        acc = np.zeros(32, np.uint8)
        for s in members:
            acc ^= c[s]
        assert np.array_equal(acc, x[i])
    for grp in check3:
        acc = np.zeros(32, np.uint8)
        for s in grp:
            acc ^= c[s]
        assert not acc.any()


def _usable(grp, s, known):
    return s in grp and not [m for m in grp if m != s and not known[m]]


def test_local_repair_against_brute_force():
    # each level's choice is checked against a direct search of the groups
    # usable with what is known at that level
    G = G_of(40, 70, seed=2)
    x = gen.payload(0, 6, 40, 16)
    c = codec.encode(G, x)
    _, check3 = checks.split(*checks.cga(G)[:2])
    rng = np.random.default_rng(3)
    deeper = 0
    for trial in range(40):
        lost = sorted(rng.choice(70, size=int(rng.integers(1, 12)), replace=False).tolist())
        er = (rng.random(70) < 0.1).astype(np.uint8)
        er[lost] = 0
        out, ok, used, lev, levels = checks.local_repair(check3, c, lost, er)
        known0 = np.ones(70, dtype=bool)
        known0[np.flatnonzero(er)] = False
        known0[lost] = False
        for l in range(levels + 1):
            known = known0.copy()
            for r, s in enumerate(lost):
                if ok[r] and lev[r] < l:
                    known[s] = True
            for r, s in enumerate(lost):
                usable = [q for q, grp in enumerate(check3) if _usable(grp, s, known)]
                if ok[r] and lev[r] == l:
                    # the first group usable at this level, and none before it
                    assert used[r] == usable[0] and np.array_equal(out[r], c[s])
                elif not ok[r] or lev[r] > l:
                    # unknown at this level: nothing usable yet (else it would be rebuilt here)
                    assert not usable or (ok[r] and lev[r] == l)
        for r, s in enumerate(lost):
            if not ok[r]:
                assert used[r] == -1 and lev[r] == -1 and not out[r].any()
        deeper += int(levels > 1)
    assert deeper > 0


def test_local_repair_closure_is_order_independent():
    # the rebuilt set equals that of a queue-driven sequential search in any
    # order (the closure of the one-unknown rule), and the one-level run is
    # the first step of it
    G = G_of(60, 110, seed=5, dist="raptor")
    x = gen.payload(0, 8, 60, 16)
    c = codec.encode(G, x)
    _, check3 = checks.split(*checks.cga(G)[:2])
    rng = np.random.default_rng(11)
    for trial in range(25):
        lost = sorted(rng.choice(110, size=int(rng.integers(2, 30)), replace=False).tolist())
        _, ok, _, _, levels = checks.local_repair(check3, c, lost)
        known = np.ones(110, dtype=bool)
        known[lost] = False
        todo = list(lost)
        rng.shuffle(todo)
        progress = True
        while progress:
            progress = False
            for s in list(todo):
                if any(_usable(grp, s, known) for grp in check3):
                    known[s] = True
                    todo.remove(s)
                    progress = True
        assert sorted(set(lost) - set(todo)) == [s for r, s in enumerate(lost) if ok[r]]
        _, ok1, _, lev1, levels1 = checks.local_repair(check3, c, lost, max_levels=1)
        assert levels1 == min(levels, 1) and set(np.flatnonzero(ok1)) == set(np.flatnonzero(lev1 == 0))


def test_check_data_reads_the_papers_example():
    # §2.7's example array: #3{13, 56, 17, 66}, #2(19; 11, 13), #3{39, 88}
    with open(os.path.join(GOLDEN, "paper_check_data.json")) as fh:
        g = json.load(fh)
    c2, c3 = checks.parse_check_data(g["array"])
    assert c3 == g["check3"]
    assert [[i, m] for i, m in c2] == g["check2"]
    check2, groups = checks.from_check_data(g["array"])
    assert check2 == {19: [11, 13]} and groups == [[39, 88], [13, 17, 56, 66]]


def test_check_data_size_formula_and_round_trip():
    # a converged run stores N = sum L_c + k + 2n integers (§2.7): k check #2
    # records of L + 3 and n - k check #3 records of L + 2
    G = graph.from_rows(2, [[0], [1], [0, 1]])
    check2, check3 = checks.split(*checks.cga(G)[:2])
    arr = checks.check_data(check2, check3)
    L = sum(len(v) for v in check2.values()) + sum(len(gr) for gr in check3)
    assert len(arr) == L + G.k + 2 * G.n == 13
    assert arr == [1, 0, 1, 0, 1, 1, 1, 1, 0, 3, 0, 1, 2]
    for k, n, seed in ((40, 70, 2), (30, 45, 3)):
        G = G_of(k, n, seed=seed)
        check2, check3 = checks.split(*checks.cga(G)[:2])
        arr = checks.check_data(check2, check3)
        L = sum(len(v) for v in check2.values()) + sum(len(gr) for gr in check3)
        assert len(arr) == L + 3 * len(check2) + 2 * len(check3)
        assert checks.from_check_data(arr) == (check2, check3)


@pytest.mark.parametrize("arr", [[2, 1, 5], [0, 3, 1, 2], [1, 4, 2, 7], [1, 4], [0]])
def test_check_data_rejects_malformed_arrays(arr):
    with pytest.raises(ValueError):
        checks.parse_check_data(arr)


def test_extra_groups_from_a_degree_one_block():
    # coded block 3 has degree one (input 0) while input 0's check #2 set is
    # {0, 1}: c_3 = x_0 = c_0 ^ c_1, so {0, 1, 3} XORs to zero
    G = graph.from_rows(2, [[0, 1], [1], [0, 1], [0]])
    extra = checks.extra_groups(G, {0: [0, 1], 1: [1]})
    assert extra == [[0, 1, 3]]
    # a degree-one block that is itself input 0's check #2 set adds nothing
    assert checks.extra_groups(G, {0: [3], 1: [1]}) == []


def test_extra_groups_hold_on_precoded_payloads():
    # every group from degree-one blocks and from the precode's check #1 sets
    # (Eqs. (1)-(4)) XORs to zero on an encoded precoded object
    from oracle import precode
    b, k, n = 85, 100, 170
    G = G_of(k, n, seed=3, dist="raptor")
    check2, check3 = checks.split(*checks.cga(G)[:2])
    c1 = precode.checks(b, k)
    data = gen.payload(0, 9, b, 32)
    x = precode.encode(b, k, data)
    c = codec.encode(G, x)
    extra = checks.extra_groups(G, check2, c1)
    from_c1 = checks.extra_groups(G, check2, c1)[len(checks.extra_groups(G, check2)):]
    assert from_c1, "no check #1 set had every member in check #2"
    for grp in extra:
        acc = np.zeros(32, np.uint8)
        for s in grp:
            acc ^= c[s]
        assert not acc.any()
    merged = checks.with_extra_groups(check3, extra)
    assert [len(gr) for gr in merged] == sorted(len(gr) for gr in merged)
    assert len({tuple(gr) for gr in merged}) == len(merged) >= len(check3)


def test_extend_local_makes_the_encoded_rows():
    # §2.9: a code grown from 140 to 160 rows; the new rows that local groups
    # reach equal the encoding of the longer code's rows (the definition),
    # the rest stay zero; with some old rows unavailable fewer are made
    G = graph.build(graph.GraphParams(k=80, n=160, dist="raptor", seed=5))
    x = gen.payload(3, 0, 80, 64)
    c = codec.encode(G, x)
    b, L, _ = checks.cga(G)
    _, groups = checks.split(b, L)
    rows, made, levels = checks.extend_local(groups, c[:140], 160)
    assert made.sum() > 0 and levels >= 1
    assert np.array_equal(rows[made == 1], c[140:][made == 1])
    assert not rows[made == 0].any()
    er = np.zeros(140, np.uint8)
    er[::7] = 1
    rows2, made2, _ = checks.extend_local(groups, c[:140], 160, er)
    assert made2.sum() <= made.sum()
    assert np.array_equal(rows2[made2 == 1], c[140:][made2 == 1])
    # a new row is made exactly when some group of it has every other member
    # known, directly or through rows made before: the closure, checked by brute force
    known = np.ones(160, bool)
    known[140:] = False
    known[:140][er == 1] = False
    changed = True
    while changed:
        changed = False
        for grp in groups:
            unk = [m for m in grp if not known[m]]
            if len(unk) == 1 and unk[0] >= 140:
                known[unk[0]] = True
                changed = True
    assert np.array_equal(made2.astype(bool), known[140:])
