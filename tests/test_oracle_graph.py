"""Pins of the oracle's seeded LDGM graph (CPU only)."""

import itertools

import numpy as np
from scipy import stats

from oracle import dist, gf2, graph, prng
from synth import workloads


def P(**kw):
    return graph.GraphParams(**kw)


def test_rows_sorted_distinct_in_range():
    for p in [P(k=64, n=96), P(k=1, n=5), P(k=3, n=50, dist="raptor"),
              P(k=200, n=300, dist="finite", finite_w=workloads.finite16_weights(), seed=7)]:
        G = graph.build(p)
        assert len(G.row_ptr) == p.n + 1 and G.row_ptr[0] == 0
        for j in range(p.n):
            r = G.N(j)
            assert 1 <= len(r) <= p.k
            assert np.all(np.diff(r) > 0) and r[0] >= 0 and r[-1] < p.k


def test_csc_is_transpose_of_csr():
    G = graph.build(P(k=50, n=80, seed=3, stripe_key=9))
    B = gf2.dense_B(G)
    BT = np.zeros_like(B)
    for i in range(G.k):
        rows = G.NT(i)
        assert np.all(np.diff(rows) > 0)
        BT[i, rows] = 1
    assert np.array_equal(B, BT)
    assert G.col_ptr[-1] == G.nnz


def test_prefix_stability_in_n():
    a = graph.build(P(k=100, n=120))
    b = graph.build(P(k=100, n=300))
    assert np.array_equal(a.row_ptr, b.row_ptr[:121])
    assert np.array_equal(a.col, b.col[:a.nnz])


def test_seed_and_stripe_key_change_the_graph():
    a = graph.build(P(k=100, n=120))
    for other in [P(k=100, n=120, seed=2), P(k=100, n=120, stripe_key=1)]:
        b = graph.build(other)
        assert not (np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col))


def test_degree_histogram_matches_distribution():
    p = P(k=64, n=20000, seed=11)
    G = graph.build(p)
    w, _, _ = dist.rsd_weights(64, 0.1, 0.05)
    probs = np.array(dist.probabilities(w)[1:])
    counts = np.bincount(G.degrees(), minlength=65)[1:]
    exp = probs * p.n
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    chi2 = float(((obs - ex) ** 2 / ex).sum())
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4


def test_neighbour_marginals_uniform():
    p = P(k=40, n=6000, dist="finite", finite_w=(0.0, 0.0, 0.0, 1.0), seed=5)   # all degree 4
    G = graph.build(p)
    assert np.all(G.degrees() == 4)
    counts = np.bincount(G.col, minlength=40)
    chi2, pv = stats.chisquare(counts)
    assert pv > 1e-4


def test_floyd_uniform_over_subsets():
    # all C(5,2) = 10 subsets equally likely
    seen = {}
    for s in range(20000):
        key = prng.stream_key(1234, 1, 0, s)
        sub = tuple(graph.floyd_sample(key, 2, 5))
        assert len(set(sub)) == 2
        seen[sub] = seen.get(sub, 0) + 1
    assert set(seen) == set(itertools.combinations(range(5), 2))
    chi2, pv = stats.chisquare(list(seen.values()))
    assert pv > 1e-4


def test_floyd_full_draw_is_everything():
    key = prng.stream_key(1, 1, 0, 0)
    assert graph.floyd_sample(key, 17, 17) == list(range(17))


def test_from_rows_roundtrip(golden):
    g = golden("dpg_hand_example.json")
    G = graph.from_rows(g["k"], g["rows"])
    assert [list(G.N(j)) for j in range(G.n)] == g["rows"]
    assert list(G.NT(0)) == [0, 1, 2, 4]
