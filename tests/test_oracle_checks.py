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


def test_local_repair_against_brute_force():
    G = G_of(40, 70, seed=2)
    x = gen.payload(0, 6, 40, 16)
    c = codec.encode(G, x)
    _, check3 = checks.split(*checks.cga(G)[:2])
    rng = np.random.default_rng(3)
    for trial in range(30):
        lost = sorted(rng.choice(70, size=int(rng.integers(1, 6)), replace=False).tolist())
        er = (rng.random(70) < 0.1).astype(np.uint8)
        er[lost] = 0
        out, ok, used = checks.local_repair(check3, c, lost, er)
        down = set(lost) | set(np.flatnonzero(er).tolist())
        for r, s in enumerate(lost):
            usable = [q for q, grp in enumerate(check3) if s in grp and not (set(grp) - {s}) & down]
            if usable:
                assert ok[r] == 1 and used[r] == usable[0] and np.array_equal(out[r], c[s])
            else:
                assert ok[r] == 0 and used[r] == -1 and not out[r].any()
