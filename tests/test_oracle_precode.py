"""Pins of the precode oracle (oracle/precode.py): Algorithm 2's checks against
Algorithm 2 evaluated on small codes, the cyclic-shift block structure of
array LDPC codes, girth, encodability, and the
two-stage decode against direct checks and an independent check peel."""

import itertools

import numpy as np
import pytest

from oracle import codec, graph, precode
from synth import gen

# (b, k): Table 2's k values with j' = 3, and small codes
CODES = [(28, 49), (21, 35), (55, 77), (10, 15), (925, 1036), (9919, 10246), (110, 121)]


def is_prime(q):
    return q >= 2 and all(q % d for d in range(2, int(q ** 0.5) + 1))


@pytest.mark.parametrize("k", [2, 15, 49, 97, 1024, 1036, 10246, 2 * 3 * 5 * 7 * 11, 121])
def test_largest_prime_factor(k):
    p = precode.largest_prime_factor(k)
    assert is_prime(p) and k % p == 0
    assert not any(k % q == 0 and is_prime(q) for q in range(p + 1, k + 1))


def test_check_one_equals_algorithm_2(golden):
    # Algorithm 2's index expression, evaluated term by term for small codes
    # (every row) and sampled rows of Table 2's codes
    g = golden("alg2_check_one.json")
    for code in g["codes"]:
        b, k = code["b"], code["k"]
        assert precode.array_params(b, k) == (code["p"], code["kp"], code["jp"])
        L = precode.check_one(b, k)
        assert len(L) == k - b
        for r, row in code["rows"].items():
            assert L[int(r)] == sorted(row), (b, k, r)
    assert sorted(g["codes"][0]["rows"]["0"]) == [4, 12, 20]      # the hand-worked row


@pytest.mark.parametrize("b,k", CODES)
def test_checks_are_blocks_of_cyclic_shifts(b, k):
    # Array LDPC codes are made of p x p powers of the cyclic shift: in every
    # block row the checks meet a run of consecutive block columns, each in a
    # permutation block whose column offset grows with the row by one (mod p),
    # and the run ends in the identity block of that block row's parity blocks.
    p, kp, jp = precode.array_params(b, k)
    C = precode.checks(b, k)
    assert len(C) == k - b == jp * p
    for j in range(jp):
        rows = [C[i + j * p] for i in range(p)]
        cols = [sorted({m // p for m in row}) for row in rows]
        assert all(c_ == cols[0] for c_ in cols)
        assert cols[0] == list(range(cols[0][0], cols[0][0] + kp - jp + 1))
        assert cols[0][-1] * p == b + j * p                      # parity blocks b + jp .. b + jp + p - 1
        for c in cols[0]:
            off = [next(m % p for m in row if m // p == c) for row in rows]
            assert sorted(off) == list(range(p))                 # a permutation block
            assert all((off[i] - i) % p == (off[0]) % p for i in range(p))   # a power of the shift
        assert [next(m for m in row if m // p == cols[0][-1]) for row in rows] == [b + j * p + i for i in range(p)]


@pytest.mark.parametrize("b,k", [c for c in CODES if c[1] <= 1100])
def test_no_two_checks_share_two_blocks(b, k):
    # girth at least 6 (k' <= p): the property array codes are chosen for
    p, kp, jp = precode.array_params(b, k)
    assert kp <= p
    C = [set(c) for c in precode.checks(b, k)]
    assert all(len(a & c) <= 1 for a, c in itertools.combinations(C, 2))


@pytest.mark.parametrize("b,k", CODES)
def test_parity_rows_only_use_earlier_block_rows(b, k):
    p, _, _ = precode.array_params(b, k)
    for r, row in enumerate(precode.check_one(b, k)):
        assert len(set(row)) == len(row)
        assert all(0 <= i < b + p * (r // p) for i in row)


@pytest.mark.parametrize("b,k", [(28, 49), (925, 1036)])
def test_encode_satisfies_every_check(b, k):
    data = gen.payload(0, 3, b, 16)
    x = precode.encode(b, k, data)
    assert np.array_equal(x[:b], data)
    for members in precode.checks(b, k):
        acc = np.zeros(16, np.uint8)
        for m in members:
            acc ^= x[m]
        assert not acc.any()
    # linearity: the parity of a sum is the sum of the parities
    d2 = gen.payload(0, 4, b, 16)
    assert np.array_equal(precode.encode(b, k, data ^ d2), x ^ precode.encode(b, k, d2))


def queue_check_peel(C, known):
    """Independent reference: recovered set of a queue-driven peel over the checks."""
    known = set(np.flatnonzero(known).tolist())
    changed = True
    while changed:
        changed = False
        for members in C:
            unknown = [s for s in members if s not in known]
            if len(unknown) == 1:
                known.add(unknown[0])
                changed = True
    return known


def test_precode_recovers_what_the_ldgm_decode_misses():
    b, k = 925, 1036
    G = graph.build(graph.GraphParams(k=k, n=1500, dist="raptor", seed=3))
    data = gen.payload(0, 9, b, 32)
    x = precode.encode(b, k, data)
    c = codec.encode(G, x)
    # erase every coded row on three data blocks: the LDGM decode cannot get them
    lost = [5, 400, 900]
    er = np.zeros(G.n, np.uint8)
    for i in lost:
        er[G.NT(i)] = 1
    xd, rec, st, _ = codec.decode(G, c, er)
    assert not rec[lost].any()
    got, ok, status = precode.decode_two_stage(G, b, c, er)
    assert status[0] == 1 and ok.all() and np.array_equal(got, data)
    assert status[2] == st[2] and status[3] >= 1


@pytest.mark.parametrize("seed", range(4))
def test_two_stage_decode_is_exact_and_matches_a_queue_peel(seed):
    b, k = 28, 49
    G = graph.build(graph.GraphParams(k=k, n=60, dist="rsd", seed=seed + 1))
    data = gen.payload(1, seed, b, 16)
    x = precode.encode(b, k, data)
    c = codec.encode(G, x)
    C = precode.checks(b, k)
    rng = np.random.default_rng(seed)
    for trial in range(20):
        er = (rng.random(G.n) < rng.uniform(0.0, 0.5)).astype(np.uint8)
        got, ok, status = precode.decode_two_stage(G, b, c, er)
        okb = ok.astype(bool)
        assert np.array_equal(got[okb], data[okb]) and not got[~okb].any()
        _, rec, _, _ = codec.decode(G, c, er)
        want = queue_check_peel(C, rec) if not rec[:b].all() else set(np.flatnonzero(rec).tolist())
        assert set(np.flatnonzero(okb).tolist()) == {s for s in want if s < b}
        assert status[0] == int(okb.all()) and status[1] == b - okb.sum()


def test_no_erasures_and_level_limit():
    b, k = 55, 77
    G = graph.build(graph.GraphParams(k=k, n=130, dist="rsd", seed=2))
    data = gen.payload(2, 0, b, 16)
    c = codec.encode(G, precode.encode(b, k, data))
    got, ok, status = precode.decode_two_stage(G, b, c, np.zeros(G.n, np.uint8))
    assert np.array_equal(got, data) and status[:2] == (1, 0)
    # stage two one level at a time ends where the unbounded run ends
    x, rec, _, _ = codec.decode(G, c, np.zeros(G.n, np.uint8))
    rec[:3] = 0
    full_x, full_known, L = precode.precode_bp(b, k, x, rec)
    one_x, one_known, L1 = precode.precode_bp(b, k, x, rec, maxit=1)
    assert L1 == min(L, 1) and one_known.sum() <= full_known.sum()
    assert full_known[:b].all() and np.array_equal(full_x[:b], data)


def test_two_stage_repair_rebuilds_lost_rows_exactly():
    # Table 2's smaller code with three of ten disks lost: the two-stage
    # decode brings the data back, the parity is encoded again, and every
    # lost row equals its encoding, including rows the LDGM pass alone
    # cannot rebuild
    b, k, n = 925, 1036, 2180
    G = graph.build(graph.GraphParams(k=k, n=n, dist="raptor", seed=1))
    x = precode.encode(b, k, gen.payload(0, 2, b, 16))
    c = codec.encode(G, x)
    lost = list(range(0, 3 * n // 10))
    out, ok = precode.repair_two_stage(G, b, c, np.zeros(n, np.uint8), lost)
    assert ok.all() and np.array_equal(out, c[lost])
    _, ok1 = codec.repair_conventional(G, c, np.zeros(n, np.uint8), lost)
    assert ok1.sum() < ok.sum()


def test_two_stage_repair_when_the_data_cannot_come_back():
    # six of ten disks lost: the data stays incomplete, rows are rebuilt only
    # when all their inputs were recovered, and each rebuilt row is exact
    b, k, n = 925, 1036, 2180
    G = graph.build(graph.GraphParams(k=k, n=n, dist="raptor", seed=1))
    x = precode.encode(b, k, gen.payload(0, 3, b, 16))
    c = codec.encode(G, x)
    lost = list(range(0, 6 * n // 10))
    out, ok = precode.repair_two_stage(G, b, c, np.zeros(n, np.uint8), lost)
    assert 0 < ok.sum() < len(lost)
    for r, j in enumerate(lost):
        if ok[r]:
            assert np.array_equal(out[r], c[j])
        else:
            assert not out[r].any()
