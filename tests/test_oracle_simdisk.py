"""Pins of the disk-failure sweep oracle (oracle/simdisk.py) against a worked
example, closed forms, the GF(2) rank and an independent sequential peel."""

import itertools
import math

import numpy as np
import pytest

from oracle import codec, gf2, graph, simdisk
from synth import gen


def G_of(k, n, **kw):
    kw.setdefault("dist", "rsd")
    return graph.build(graph.GraphParams(k=k, n=n, **kw))


def test_hand_example_three_disks():
    # k = 2 inputs, coded rows {0}, {1}, {0, 1}, one row per disk
    G = graph.from_rows(2, [[0], [1], [0, 1]])
    # one disk lost: the two others always determine both inputs; with row 2
    # lost both survivors have degree one (one level), otherwise the
    # surviving singleton frees the sum row at a second level
    assert simdisk.sim_disks(G, 3, 1).tolist() == [[1, 0, 2], [1, 0, 2], [1, 0, 1]]
    # two disks lost: one row is left, never enough for two inputs
    assert simdisk.sim_disks(G, 3, 2).tolist() == [[0, 2, 0], [0, 1, 1], [0, 1, 1]]
    assert simdisk.sim_disks(G, 3, 0).tolist() == [[1, 0, 1]]
    assert simdisk.sim_disks(G, 3, 3).tolist() == [[0, 2, 0]]


@pytest.mark.parametrize("n,s", [(10, 10), (2180, 10), (21800, 10), (97, 7), (5, 1), (64, 64)])
def test_striping_is_an_equal_in_order_partition(n, s):
    rows = [simdisk.disk_rows(n, s, d) for d in range(s)]
    flat = [j for r in rows for j in r]
    assert flat == list(range(n))
    sizes = {len(r) for r in rows}
    assert max(sizes) - min(sizes) <= 1 and min(sizes) == n // s
    if n % s == 0:
        assert sizes == {n // s}


@pytest.mark.parametrize("s,f", [(10, 0), (10, 2), (10, 5), (7, 7), (12, 4)])
def test_combinations_count_and_rank_order(s, f):
    combos = simdisk.combinations(s, f)
    assert len(combos) == math.comb(s, f)
    assert all(list(c) == sorted(set(c)) and len(c) == f for c in combos)
    assert combos == sorted(combos) and len(set(combos)) == len(combos)
    if f:
        assert combos[0] == tuple(range(f)) and combos[-1] == tuple(range(s - f, s))


def test_sub_range_is_a_slice_of_the_sweep():
    G = G_of(40, 70, seed=3)
    full = simdisk.sim_disks(G, 7, 3)
    assert np.array_equal(simdisk.sim_disks(G, 7, 3, first=11, count=9), full[11:20])


def test_fewer_failures_never_decode_less():
    # peeling is monotone in the surviving rows
    G = G_of(40, 60, seed=5)
    s = 6
    res = {}
    for f in range(s + 1):
        for c, st in zip(simdisk.combinations(s, f), simdisk.sim_disks(G, s, f)):
            res[c] = st
    assert res[()][0] == 1 and res[tuple(range(s))].tolist() == [0, 40, 0]
    for a in res:
        for b in res:
            if set(a) < set(b):
                assert res[b][0] <= res[a][0] and res[a][1] <= res[b][1]
    assert 0 < sum(int(v[0]) for v in res.values()) < len(res)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tolerable_patterns_have_full_rank_and_match_a_sequential_peel(seed):
    G = G_of(24, 40, seed=seed, dist="finite", finite_w=(0.1, 0.5, 0.3, 0.1))
    B = gf2.dense_B(G)
    s = 5
    for f in range(s + 1):
        for failed, st in zip(simdisk.combinations(s, f), simdisk.sim_disks(G, s, f)):
            er = simdisk.erased_mask(G.n, s, failed)
            surv = np.flatnonzero(er == 0)
            rec = codec.bp_sequential(G, er)
            assert st[1] == G.k - int(rec.sum())
            if st[0]:
                assert gf2.rank(B, surv) == G.k
            if gf2.rank(B, surv) < G.k:
                assert st[0] == 0


def test_level_limit():
    G = G_of(40, 70, seed=3)
    full = simdisk.sim_disks(G, 7, 2)
    one = simdisk.sim_disks(G, 7, 2, maxit=1)
    assert (one[:, 2] <= 1).all() and (one[:, 1] >= full[:, 1]).all()
    L = int(full[:, 2].max())
    assert np.array_equal(simdisk.sim_disks(G, 7, 2, maxit=L), full)


def test_precoded_sweep_matches_the_two_stage_decode_on_payloads():
    # the symbolic sweep against the numeric two-stage decode of a real
    # payload, pattern by pattern; the precode only ever adds tolerable patterns
    from oracle import precode
    b, k = 28, 49
    G = graph.build(graph.GraphParams(k=k, n=84, dist="rsd", seed=2))
    data = gen.payload(3, 1, b, 16)
    c = codec.encode(G, precode.encode(b, k, data))
    s = 7
    for f in range(s + 1):
        got = simdisk.sim_disks_precoded(G, b, s, f)
        plain = simdisk.sim_disks(G, s, f)
        for r, failed in enumerate(simdisk.combinations(s, f)):
            out, ok, status = precode.decode_two_stage(G, b, c, simdisk.erased_mask(G.n, s, failed))
            assert got[r].tolist() == list(status)
            assert np.array_equal(out[ok.astype(bool)], data[ok.astype(bool)])
            assert got[r][0] >= plain[r][0]
    assert simdisk.sim_disks_precoded(G, b, s, 2, first=5, count=3).tolist() == \
        simdisk.sim_disks_precoded(G, b, s, 2)[5:8].tolist()


def test_precoded_sweep_monotone():
    b, k = 28, 49
    G = graph.build(graph.GraphParams(k=k, n=70, dist="rsd", seed=4))
    s = 7
    res = {}
    for f in range(s + 1):
        for cmb, st in zip(simdisk.combinations(s, f), simdisk.sim_disks_precoded(G, b, s, f)):
            res[cmb] = st
    for a in res:
        for bb in res:
            if set(a) < set(bb):
                assert res[bb][0] <= res[a][0] and res[a][1] <= res[bb][1]
