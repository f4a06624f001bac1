"""Pins of the oracle's encode / peeling decode / repair / update (CPU only)."""

import itertools

import numpy as np
import pytest

from oracle import codec, gf2, graph
from synth import gen, workloads


def rand_x(k, t, seed=0, stripe=0):
    return gen.payload(seed, stripe, k, t)


def G_of(k, n, **kw):
    return graph.build(graph.GraphParams(k=k, n=n, **kw))


@pytest.mark.parametrize("k,n,kw", [(8, 12, {}), (64, 96, {}), (20, 40, dict(dist="raptor")),
                                    (30, 31, dict(dist="finite", finite_w=(0.1, 0.5, 0.4)))])
def test_encode_equals_dense_gf2_product(k, n, kw):
    G = G_of(k, n, **kw)
    x = rand_x(k, 64, seed=3)
    assert np.array_equal(codec.encode(G, x), gf2.encode_bits(gf2.dense_B(G), x))


def test_encode_linearity_and_zero():
    G = G_of(64, 96)
    x, y = rand_x(64, 128, 1), rand_x(64, 128, 2)
    assert np.array_equal(codec.encode(G, x ^ y), codec.encode(G, x) ^ codec.encode(G, y))
    assert not codec.encode(G, np.zeros_like(x)).any()


def test_encode_parity_invariant_and_copies():
    G = G_of(64, 200, seed=4)
    x = rand_x(64, 64, 5)
    c = codec.encode(G, x)
    lhs = np.bitwise_xor.reduce(c, axis=0)
    odd = [i for i in range(G.k) if len(G.NT(i)) % 2 == 1]
    rhs = np.bitwise_xor.reduce(x[odd], axis=0) if odd else np.zeros(64, np.uint8)
    assert np.array_equal(lhs, rhs)
    ones = [j for j in range(G.n) if G.deg(j) == 1]
    assert ones
    for j in ones:
        assert np.array_equal(c[j], x[G.N(j)[0]])


def test_paper_worked_xor_example(golden):
    """Eqs. (1)-(4): XOR over groups cancels repeated coded symbols."""
    g = golden("paper_eq1_4.json")
    C = gen.payload(11, 0, 100, 64)                      # coded blocks C0..C99
    rows = [g["check2"]["D0"], g["check2"]["D1"], g["check2"]["D2"], g["check3"]]
    G = graph.from_rows(100, rows)
    D = codec.encode(G, C)
    assert np.array_equal(D[0] ^ D[1] ^ D[2], D[3])
    # the symmetric difference of the three groups is exactly the check #3 group
    sym = set()
    for r in rows[:3]:
        sym ^= set(r)
    assert sorted(sym) == g["check3"]


def check_schedule_against(golden_levels, golden_status, sched):
    assert [[list(p) for p in lev] for lev in sched.levels] == golden_levels
    assert list(sched.status()) == golden_status


def test_dpg_hand_example(golden):
    g = golden("dpg_hand_example.json")
    G = graph.from_rows(g["k"], g["rows"])
    s = codec.peel_schedule(G, np.array(g["erased"], dtype=np.uint8))
    check_schedule_against(g["levels"], g["status"], s)
    e = g["with_erasure"]
    s2 = codec.peel_schedule(G, np.array(e["erased"], dtype=np.uint8))
    check_schedule_against(e["levels"], e["status"], s2)
    x = rand_x(3, 32, 9)
    c = codec.encode(G, x)
    for er in (g["erased"], e["erased"]):
        xd, rec, st, _ = codec.decode(G, c, np.array(er, dtype=np.uint8))
        assert st[0] == 1 and np.array_equal(xd, x) and rec.all()


def verify_schedule_properties(G, erased, sched):
    """Each level is exactly the set of inputs named by some weight-1 survivor,
    each paired with the minimum (degree, row) namer; F is a stopping set."""
    erased = np.asarray(erased, dtype=bool)
    F = set(range(G.k))
    for lev in sched.levels:
        namers = {}
        for h in range(G.n):
            if erased[h]:
                continue
            rem = [i for i in G.N(h) if i in F]
            if len(rem) == 1:
                namers.setdefault(rem[0], []).append((G.deg(h), h))
        assert [f for f, _ in lev] == sorted(namers)
        for f, g in lev:
            assert (G.deg(g), g) == min(namers[f])
        F -= {f for f, _ in lev}
    assert sorted(F) == list(sched.F)
    return F


def stopping_set(G, erased, F):
    for h in range(G.n):
        if not erased[h] and len([i for i in G.N(h) if i in F]) == 1:
            return False
    return True


@pytest.mark.parametrize("seed", range(6))
def test_decode_identity_and_failure_semantics(seed):
    k, n = 64, 160 if seed % 2 == 0 else 96
    G = G_of(k, n, seed=seed + 1)
    x = rand_x(k, 256, seed)
    c = codec.encode(G, x)
    er = gen.erasure_mask(seed, 0, n, 16)
    xd, rec, st, sched = codec.decode(G, c, er)
    R = rec.astype(bool)
    assert np.array_equal(xd[R], x[R])
    assert not xd[~R].any()
    assert st == (int(R.all()), int((~R).sum()), sched.L)
    F = verify_schedule_properties(G, er, sched)
    assert stopping_set(G, er.astype(bool), F)
    if st[0]:
        assert np.array_equal(xd, x)


def test_decode_succeeds_at_high_overhead():
    G = G_of(64, 200, seed=3)
    x = rand_x(64, 64, 1)
    xd, rec, st, _ = codec.decode(G, codec.encode(G, x), np.zeros(200, np.uint8))
    assert st[0] == 1 and np.array_equal(xd, x)


@pytest.mark.parametrize("seed", range(8))
def test_recovered_set_is_order_independent(seed):
    k, n = 100, 130
    G = G_of(k, n, seed=seed)
    er = gen.erasure_mask(seed + 50, 0, n, 10)
    R = codec.peel_schedule(G, er).recovered_mask().astype(bool)
    assert np.array_equal(R, codec.bp_sequential(G, er))
    for order in range(3):
        assert np.array_equal(R, codec.bp_sequential(G, er, order=order + 1))


def test_maxit_truncates_levels():
    G = G_of(64, 160, seed=1)
    er = np.zeros(160, np.uint8)
    full = codec.peel_schedule(G, er)
    assert full.L >= 3
    for m in range(1, full.L + 2):
        s = codec.peel_schedule(G, er, maxit=m)
        assert s.L == min(m, full.L)
        assert s.levels == full.levels[:s.L]


def test_forced_failure_when_all_neighbours_of_an_input_are_erased():
    G = G_of(64, 160, seed=1)
    i = 5
    er = np.zeros(160, np.uint8)
    er[G.NT(i)] = 1
    s = codec.peel_schedule(G, er)
    assert i in set(s.F) and s.status()[0] == 0


def test_degree_one_graph_is_selection():
    G = G_of(20, 30, dist="finite", finite_w=(1.0,))
    x = rand_x(20, 64, 2)
    c = codec.encode(G, x)
    xd, rec, st, s = codec.decode(G, c, np.zeros(30, np.uint8))
    covered = sorted(set(int(G.N(j)[0]) for j in range(30)))
    assert list(np.flatnonzero(rec)) == covered
    assert s.L == (1 if covered else 0)
    assert np.array_equal(xd[covered], x[covered])


def _span_by_enumeration(B, cols):
    """Every GF(2) combination of the listed columns, as k-bit ints: the XOR
    of each of the 2^|cols| subsets."""
    vecs = [sum(1 << int(i) for i in np.flatnonzero(B[:, g])) for g in cols]
    span = {0}
    for v in vecs:
        span |= {s ^ v for s in span}
    return span


def test_ml_set_small_cases():
    # rows {0,1}, {1,2}, {0,1,2}: no row has one unknown, so peeling recovers
    # nothing, yet the three rows have full rank and determine every input
    G = graph.from_rows(3, [[0, 1], [1, 2], [0, 1, 2]])
    B = gf2.dense_B(G)
    assert gf2.ml_set(B, [0, 1, 2]) == [0, 1, 2] and gf2.rank(B, [0, 1, 2]) == 3
    assert not codec.peel_schedule(G, np.zeros(3, np.uint8)).recovered_mask().any()
    # without the third row the span is {0, x0^x1, x1^x2, x0^x2}: no unit vector
    assert gf2.ml_set(B, [0, 1]) == [] and gf2.rank(B, [0, 1]) == 2
    # an input no surviving row touches is never determinable; the others are
    G2 = graph.from_rows(4, [[0], [0, 1], [1, 2], [3]])
    B2 = gf2.dense_B(G2)
    assert gf2.ml_set(B2, [0, 1, 2]) == [0, 1, 2]
    assert gf2.ml_set(B2, [0, 1, 2, 3]) == [0, 1, 2, 3]
    assert gf2.ml_set(B2, [1, 2, 3]) == [3]
    assert gf2.ml_set(B2, []) == []


def test_ml_set_and_rank_against_enumerated_span():
    # brute force: the span of the surviving columns listed element by element
    for k, n, seed in [(4, 6, 1), (5, 7, 2), (3, 6, 3), (5, 6, 4)]:
        G = G_of(k, n, seed=seed, dist="finite", finite_w=(0.3, 0.4, 0.3))
        B = gf2.dense_B(G)
        for bits in itertools.product((0, 1), repeat=n):
            surv = [j for j in range(n) if bits[j]]
            span = _span_by_enumeration(B, surv)
            assert gf2.ml_set(B, surv) == [i for i in range(k) if (1 << i) in span]
            assert 1 << gf2.rank(B, surv) == len(span)


def test_ml_set_is_all_inputs_exactly_at_full_rank():
    for seed in range(4):
        G = G_of(12, 20, seed=seed)
        B = gf2.dense_B(G)
        for m in (8, 12, 16, 20):
            surv = list(range(m))
            full = gf2.rank(B, surv) == 12
            assert (gf2.ml_set(B, surv) == list(range(12))) == full


def test_brute_force_all_erasure_patterns_tiny():
    """For tiny graphs and EVERY erasure pattern: R is within the ML-decodable
    set, ok implies full rank, F is a stopping set, values are exact."""
    cases = [(4, 7, 1), (5, 8, 2), (6, 9, 3), (6, 10, 4), (3, 6, 5)]
    for k, n, seed in cases:
        G = G_of(k, n, seed=seed, dist="finite", finite_w=(0.2, 0.4, 0.3, 0.1))
        B = gf2.dense_B(G)
        x = rand_x(k, 16, seed)
        c = codec.encode(G, x)
        for bits in itertools.product((0, 1), repeat=n):
            er = np.array(bits, dtype=np.uint8)
            xd, rec, st, sched = codec.decode(G, c, er)
            surv = [j for j in range(n) if not bits[j]]
            R = set(np.flatnonzero(rec))
            ml = set(gf2.ml_set(B, surv))
            assert R <= ml
            if st[0]:
                assert gf2.rank(B, surv) == k
            assert stopping_set(G, er.astype(bool), set(range(k)) - R)
            for i in R:
                assert np.array_equal(xd[i], x[i])


def test_repair_from_inputs_and_conventional():
    G = G_of(64, 200, seed=2)
    x = rand_x(64, 128, 4)
    c = codec.encode(G, x)
    lost = [3, 50, 199]
    assert np.array_equal(codec.repair_from_inputs(G, x, lost), c[lost])
    er = np.zeros(200, np.uint8)
    blocks, ok = codec.repair_conventional(G, c, er, lost)
    er2 = er.copy()
    er2[lost] = 1
    rec = codec.peel_schedule(G, er2).recovered_mask()
    for r, j in enumerate(lost):
        assert ok[r] == int(all(rec[i] for i in G.N(j)))
        if ok[r]:
            assert np.array_equal(blocks[r], c[j])
        else:
            assert not blocks[r].any()


def test_conventional_repair_can_succeed_when_decode_fails():
    G = G_of(64, 96, seed=2)
    x = rand_x(64, 64, 4)
    c = codec.encode(G, x)
    er = np.zeros(96, np.uint8)
    found = False
    for j in range(96):
        er2 = er.copy()
        er2[j] = 1
        s = codec.peel_schedule(G, er2)
        rec = s.recovered_mask()
        if s.status()[0] == 0 and all(rec[i] for i in G.N(j)):
            blocks, ok = codec.repair_conventional(G, c, er, [j])
            assert ok[0] == 1 and np.array_equal(blocks[0], c[j])
            found = True
            break
    assert found


def test_update_delta_equals_reencode():
    G = G_of(64, 96, seed=6)
    x = rand_x(64, 128, 1)
    c = codec.encode(G, x)
    ids = [1, 17, 40]
    new = gen.update_blocks(6, 0, ids, 128)
    x2, c2 = codec.update(G, x, ids, new)
    # delta propagation by linearity of the region XOR
    c3 = c.copy()
    for u, i in enumerate(ids):
        delta = x[i] ^ new[u]
        for h in G.NT(i):
            c3[h] ^= delta
    assert np.array_equal(c2, c3)
    changed = sorted(set(np.flatnonzero((c2 != c).any(axis=1))))
    assert set(changed) <= set(codec.affected_rows(G, ids))


def test_workload_shapes():
    s = workloads.large_stripe()
    assert (s.k, s.n, s.t, s.n_erased) == (4096, 4506, 65536, 225)
    t = workloads.tiny()
    assert (t.k, t.n, t.t, t.n_erased) == (64, 96, 4096, 16)
    r = workloads.resident256(4)
    assert all(1 <= len(sp.extra["lost"]) <= 4 and len(sp.extra["update_ids"]) == 10 for sp in r)


def _graph(k, n, seed=1, key=0, **kw):
    kw.setdefault("dist", "rsd")
    return graph.build(graph.GraphParams(k=k, n=n, seed=seed, stripe_key=key, **kw))


def test_extension_keeps_existing_blocks_and_strengthens_the_code():
    # the longer graph starts with the original rows, so the existing blocks
    # are part of the extended code unchanged; the new rows make an erasure
    # pattern decodable that the original code could not resolve
    k, n_old, n_new, t = 200, 210, 300, 16
    G0, G1 = _graph(k, n_old), _graph(k, n_new)
    x = gen.payload(0, 5, k, t)
    c_old = codec.encode(G0, x)
    new, made = codec.extend(G1, n_old, x=x)
    assert made.all() and new.shape == (n_new - n_old, t)
    assert np.array_equal(np.concatenate([c_old, new]), codec.encode(G1, x))
    er_old = gen.erasure_mask(2, 5, n_old, 10)
    _, rec0, st0, _ = codec.decode(G0, c_old, er_old)
    er_new = np.concatenate([er_old, np.zeros(n_new - n_old, np.uint8)])
    x1, rec1, st1, _ = codec.decode(G1, np.concatenate([c_old, new]), er_new)
    assert st0[0] == 0 and st1[0] == 1 and np.array_equal(x1, x)
    assert rec1.sum() > rec0.sum()


def test_extension_without_inputs_follows_the_recovered_set():
    # generated from the existing blocks: a new row is made exactly when all
    # its neighbours were recovered from the surviving old rows, and then it
    # equals the encode of the inputs; the others stay zero
    k, n_old, n_new, t = 150, 260, 320, 16
    G0, G1 = _graph(k, n_old, key=5), _graph(k, n_new, key=5)
    x = gen.payload(0, 6, k, t)
    c_old = codec.encode(G0, x)
    full, _ = codec.extend(G1, n_old, x=x)
    for n_er in (0, 30):
        er = gen.erasure_mask(2, 6, n_old, n_er)
        new, made = codec.extend(G1, n_old, c_old=c_old, erased=er)
        _, rec, _, _ = codec.decode(G0, c_old, er)
        for r, j in enumerate(range(n_old, n_new)):
            want = all(rec[i] for i in G1.N(j))
            assert bool(made[r]) == want
            assert np.array_equal(new[r], full[r] if want else np.zeros(t, np.uint8))
        if n_er == 0:
            assert rec.all() and made.all()
    assert not made.all()   # 30 of 260 rows erased: the decode stalls early
