"""GPU parity: every library result equals the oracle's, bit for bit.

All calls go through the C ABI (ctypes binding); payloads are seeded uniform
bytes.  Run on an MI355X: pytest -m gpu.
"""

import numpy as np
import pytest

from gpu_util import (check_schedule, dev, empty_i32, empty_u8, gpu_decode, gpu_peel, graphs, host,
                      oracle_decode)
from oracle import codec
from synth import gen, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07409_amd as fs
    fs.fs_reset_tune()
    yield
    fs.fs_reset_tune()


def spec_graphs(sp):
    return graphs(**sp.graph_kwargs())


def encode_case(sp):
    import paper_1702_07409_amd as fs
    g, G = spec_graphs(sp)
    x = sp.x()
    xd = dev(x)
    c = empty_u8(sp.n, sp.t)
    fs.fs_encode(g, xd, c, sp.t)
    return g, G, x, xd, c


# ---------------------------------------------------------------- encode

def test_encode_tiny():
    sp = workloads.tiny()
    g, G, x, xd, c = encode_case(sp)
    assert np.array_equal(host(c), codec.encode(G, x))


RAGGED = workloads.StripeSpec(stripe=3, k=300, n=333, t=512 * 7 + 48, dist="rsd", rsd_c=0.1,
                              rsd_delta=0.05, stripe_key=5, n_erased=20)


def test_encode_ragged_every_tuning():
    import paper_1702_07409_amd as fs
    sp = RAGGED
    g, G = spec_graphs(sp)
    x = sp.x()
    want = codec.encode(G, x)
    xd = dev(x)
    for lpr in (16, 32, 64):
        for ch in (1, 2, 4):
            for nt in (0, 1):
                for remap in (0, 1):
                    fs.fs_set_tune(lpr, ch, remap, nt)
                    c = empty_u8(sp.n, sp.t)
                    c.fill_(0x5A)
                    fs.fs_encode(g, xd, c, sp.t)
                    assert np.array_equal(host(c), want), (lpr, ch, nt, remap)
    fs.fs_reset_tune()


def test_encode_large_stripe_full_size():
    sp = workloads.large_stripe()
    g, G, x, xd, c = encode_case(sp)
    assert np.array_equal(host(c), codec.encode(G, x))


def test_encode_degree_k_rows_and_k1():
    import paper_1702_07409_amd as fs
    for kw, t in [(dict(k=8, n=20, dist="finite", finite_w=(0,) * 7 + (1.0,), seed=3), 64),
                  (dict(k=1, n=5, seed=2), 16)]:
        g, G = graphs(**kw)
        x = gen.payload(1, 0, kw["k"], t)
        c = empty_u8(kw["n"], t)
        fs.fs_encode(g, dev(x), c, t)
        assert np.array_equal(host(c), codec.encode(G, x))


@pytest.mark.parametrize("k,n,dist,t", [(10246, 21800, "raptor", 7 * 1024 + 48), (12000, 13500, "finite", 2048 + 16)])
def test_encode_sparse_graph_beyond_8192_inputs(k, n, dist, t):
    # sparse graphs of more than 8192 inputs take 512-byte slices by default:
    # several slices per block and a ragged tail
    w = workloads.finite16_weights() if dist == "finite" else ()
    sp = workloads.StripeSpec(stripe=0, k=k, n=n, t=t, dist=dist, finite_w=w, stripe_key=3, n_erased=0)
    g, G, x, xd, c = encode_case(sp)
    assert np.array_equal(host(c), codec.encode(G, x))
    import paper_1702_07409_amd as fs
    li = fs.fs_last_launch()
    assert (li["gather_kind"], li["gather_slice_bytes"]) == (1, 512), li


@pytest.mark.parametrize("k,width", [(1024, 4096), (2048, 2048), (4096, 1024), (8192, 512)])
def test_encode_rsd_default_slice_width(k, width):
    # Robust Soliton graphs take W = 4 MiB / k slices by default (within
    # [512 B, 4 KiB]); blocks of two slices and a ragged 16-byte tail
    t = 2 * width + 16
    sp = workloads.StripeSpec(stripe=0, k=k, n=round(1.08 * k), t=t, dist="rsd", rsd_c=0.05, rsd_delta=0.01,
                              stripe_key=7, n_erased=0)
    g, G, x, xd, c = encode_case(sp)
    import paper_1702_07409_amd as fs
    li = fs.fs_last_launch()
    assert (li["gather_kind"], li["gather_slice_bytes"]) == (1, width), li
    assert np.array_equal(host(c), codec.encode(G, x))


def test_encode_tiles_beyond_the_lds_edge_stage():
    # 16-row tiles of degree-200 rows hold 3200 edges: read from global memory
    import paper_1702_07409_amd as fs
    kw = dict(k=1000, n=100, dist="finite", finite_w=(0.0,) * 199 + (1.0,), seed=4)
    g, G = graphs(**kw)
    x = gen.payload(2, 0, 1000, 1024)
    for lpr in (16, 64):
        fs.fs_set_tune(lpr, 2, 1, 1)
        c = empty_u8(100, 1024)
        fs.fs_encode(g, dev(x), c, 1024)
        assert np.array_equal(host(c), codec.encode(G, x))
    fs.fs_reset_tune()


def test_encode_and_decode_rsd_heavy_tail():
    # Robust Soliton at k = 8192 has rows of degree in the thousands: they are
    # encoded as several segments combined by atomic XOR
    import paper_1702_07409_amd as fs
    sp = workloads.StripeSpec(stripe=9, k=8192, n=8847, t=512 + 64, dist="rsd", rsd_c=0.05,
                              rsd_delta=0.01, stripe_key=11, n_erased=354)
    g, G = spec_graphs(sp)
    assert int(G.degrees().max()) > 1000
    x = sp.x()
    want = codec.encode(G, x)
    for lpr, ch in ((16, 2), (64, 1), (32, 4)):
        fs.fs_set_tune(lpr, ch, 1, 1)
        c = empty_u8(sp.n, sp.t)
        c.fill_(0x77)
        fs.fs_encode(g, dev(x), c, sp.t)
        assert np.array_equal(host(c), want), (lpr, ch)
    fs.fs_reset_tune()
    decode_case(sp)


SLAB_CASES = [
    # (k, n, t, dist): the slab cases have >= 256 slices of the slab width,
    # so the LDS-slab encode runs; t is ragged against the slice width
    (500, 550, 65536 + 48, "rsd"),          # 16 lanes, 256-byte slices
    (512, 553, 65536 + 256, "rsd_heavy"),   # 16 lanes, rows split into atomic segments
    (200, 220, 131072 + 512, "finite"),     # 32 lanes
    (64, 96, 262144 + 1024, "rsd"),         # 64 lanes
    (2000, 2160, 16384 + 16, "rsd_heavy"),  # above the slab's k: the gather runs
]


@pytest.mark.parametrize("case", SLAB_CASES, ids=lambda c: "k%d-t%d-%s" % (c[0], c[2], c[3]))
@pytest.mark.parametrize("slab", [1, 0])
def test_encode_lds_slab_and_gather_match_oracle(case, slab):
    import paper_1702_07409_amd as fs
    k, n, t, kind = case
    kw = dict(stripe=80 + k % 7, k=k, n=n, t=t, stripe_key=k)
    if kind == "finite":
        sp = workloads.StripeSpec(dist="finite", finite_w=workloads.finite16_weights(), **kw)
    elif kind == "rsd_heavy":
        sp = workloads.StripeSpec(dist="rsd", rsd_c=0.05, rsd_delta=0.01, **kw)
    else:
        sp = workloads.StripeSpec(dist="rsd", **kw)
    fs.fs_set_tune(encode_slab=slab)
    try:
        g, G, x, xd, c = encode_case(sp)
        if kind == "rsd_heavy":
            assert g.max_degree > 64
        assert np.array_equal(host(c), codec.encode(G, x))
    finally:
        fs.fs_reset_tune()


def test_encode_rejects_bad_alignment():
    import paper_1702_07409_amd as fs
    g, _ = graphs(k=8, n=10, seed=1)
    x, c = empty_u8(8 * 64 + 16), empty_u8(10 * 64)
    with pytest.raises(fs.FsError):
        fs.fs_encode(g, x, c, 40)
    with pytest.raises(fs.FsError):
        fs.fs_encode(g, x[1:], c, 64)


# ---------------------------------------------------------------- peel + decode

def decode_case(sp, maxit=0):
    import paper_1702_07409_amd as fs
    g, G = spec_graphs(sp)
    x = sp.x()
    c_host = codec.encode(G, x)
    c = dev(c_host)
    er = sp.erased_mask()
    sched = codec.peel_schedule(G, er, maxit)
    check_schedule(sched, gpu_peel(g, er, maxit))
    got = gpu_decode(g, c, er, sp.t, maxit)
    xo, reco, sto, _ = oracle_decode(G, c_host, er, maxit)
    assert list(got.status) == list(sto)
    assert np.array_equal(got.recovered, reco)
    assert np.array_equal(got.x, xo)
    R = reco.astype(bool)
    assert np.array_equal(got.x[R], x[R])
    return g, G, got, sched


def test_decode_tiny():
    decode_case(workloads.tiny())


def test_decode_ragged():
    decode_case(RAGGED)


def test_decode_large_stripe_full_size():
    _, _, got, sched = decode_case(workloads.large_stripe())
    assert sched.L > 10 and 0 < got.status[1] < 4096


@pytest.mark.parametrize("maxit", [1, 2, 5])
def test_decode_maxit(maxit):
    decode_case(workloads.tiny(), maxit)


def test_decode_success_path_high_overhead():
    sp = workloads.StripeSpec(stripe=1, k=500, n=1000, t=512, dist="rsd", n_erased=100)
    _, _, got, _ = decode_case(sp)
    assert got.status[0] == 1


def test_decode_no_erasures_and_all_erased():
    for ne in (0, 96):
        sp = workloads.tiny()
        sp.n_erased = ne
        _, _, got, _ = decode_case(sp)
        if ne == 96:
            assert list(got.status) == [0, 64, 0] and not got.x.any()


def test_decode_forced_failure_of_one_input():
    sp = workloads.StripeSpec(stripe=0, k=64, n=200, t=256, dist="rsd", graph_seed=3)
    g, G = spec_graphs(sp)
    er = np.zeros(sp.n, np.uint8)
    er[G.NT(7)] = 1
    x = sp.x()
    c_host = codec.encode(G, x)
    got = gpu_decode(g, dev(c_host), er, sp.t)
    assert got.recovered[7] == 0 and not got.x[7].any()
    xo, reco, sto, _ = oracle_decode(G, c_host, er)
    assert np.array_equal(got.x, xo) and list(got.status) == list(sto)


def test_decode_k1_t16():
    sp = workloads.StripeSpec(stripe=0, k=1, n=4, t=16, dist="rsd", n_erased=2)
    decode_case(sp)


@pytest.mark.parametrize("k,n,dist", [(16384, 18022, "rsd"), (20000, 22000, "rsd"), (10246, 21800, "raptor"),
                                      (20000, 32000, "finite")])
def test_peel_state_beyond_lds_uses_workspace(k, n, dist):
    # k = 16384: the full peel state does not fit LDS, its per-row counters
    # (8 n bytes) do; n = 22000 Robust Soliton: not even those, everything
    # stays in the workspace; n = 21800 and 32000 with degrees <= 65 or 16:
    # the counters fit packed in 32 bits, and at n = 21800 the decoding row
    # of each input and the input masks as well
    w = workloads.finite16_weights() if dist == "finite" else ()
    sp = workloads.StripeSpec(stripe=0, k=k, n=n, t=16, dist=dist, finite_w=w, stripe_key=1,
                              n_erased=round(0.05 * n))
    decode_case(sp)


@pytest.mark.parametrize("prog_global", [0, 1])
def test_decode_slab_replay_program_placement(prog_global):
    # k = 1000 uses the slab replay (k x 128-byte rows in LDS); the program is
    # read from LDS or, forced by the tuning, from global memory
    import paper_1702_07409_amd as fs
    fw = tuple([0.45] + [0.0] * 22 + [0.55])
    sp = workloads.StripeSpec(stripe=4, k=1000, n=4000, t=1024 + 128, dist="finite", finite_w=fw,
                              stripe_key=2, n_erased=0)
    fs.fs_set_tune(replay_prog_global=prog_global)
    try:
        _, G, got, sched = decode_case(sp)
    finally:
        fs.fs_reset_tune()
    assert got.status[0] == 1


@pytest.mark.parametrize("prog_global", [0, 1])
def test_decode_wide_replay_program_placement(prog_global):
    import paper_1702_07409_amd as fs
    fw = tuple([0.45] + [0.0] * 22 + [0.55])
    sp = workloads.StripeSpec(stripe=4, k=4000, n=16000, t=256 * 3 + 32, dist="finite", finite_w=fw,
                              stripe_key=2, n_erased=0)
    fs.fs_set_tune(replay_prog_global=prog_global)
    try:
        _, G, got, sched = decode_case(sp)
    finally:
        fs.fs_reset_tune()
    assert got.status[0] == 1


FIN16 = workloads.finite16_weights()
LOOKAHEAD_CASES = {
    # 1585 inputs in the dependency slab: 64-byte slices, at most 215 pairs a
    # level (one per thread), ragged t (1072 = 16 slices + 48 bytes)
    "prefetched": dict(stripe=6, k=2000, n=2600, t=1024 + 48, dist="finite", finite_w=FIN16, stripe_key=5,
                       n_erased=50),
    # 32-byte slices and a first level of 741 pairs: past 512 a level's pairs
    # load their block when they run
    "wide_levels": dict(stripe=6, k=3000, n=3600, t=2048 + 128 + 32, dist="finite",
                        finite_w=tuple([0.3] + list(FIN16[1:])), stripe_key=5, n_erased=100),
    # 342 slab inputs: 128-byte slices
    "rsd": dict(stripe=7, k=2500, n=3000, t=4096 + 48, dist="rsd", stripe_key=6, n_erased=60),
    # the wide replay of blocks too short for enough 128-byte slices: 32-byte
    # slices (513, the last one 16 bytes), then 64-byte slices (513, the last
    # one 48 bytes)
    "short_32": dict(stripe=8, k=1500, n=1800, t=16384 + 16, dist="finite", finite_w=FIN16, stripe_key=7,
                     n_erased=40),
    "short_64": dict(stripe=8, k=1500, n=1800, t=32768 + 48, dist="rsd", stripe_key=8, n_erased=40),
    # 3619 slab inputs and 15203 program entries: 16-byte slices, a level of
    # 3339 pairs, no erasures
    "degree_one_heavy": dict(stripe=4, k=4000, n=16000, t=800, dist="finite",
                             finite_w=tuple([0.45] + [0.0] * 22 + [0.55]), stripe_key=2, n_erased=0),
    # 9907 slab inputs do not fit LDS beside the program: the kernel runs the
    # wide replay instead
    "slab_too_large": dict(stripe=8, k=12000, n=13500, t=160, dist="finite", finite_w=FIN16, stripe_key=7,
                           n_erased=300),
}


# slice width the wide replay must take for the short-block cases (the rule
# depends on the CU count and on how many program workgroups fit a CU, so
# the launch is checked, not assumed)
WIDE_REPLAY_WIDTH = {"short_32": 32, "short_64": 64}


@pytest.mark.parametrize("lookahead", [1, 0])
@pytest.mark.parametrize("case", sorted(LOOKAHEAD_CASES))
def test_decode_lookahead_replay(case, lookahead):
    # large k: the lookahead replay (coded blocks loaded steps ahead, the
    # inputs later pairs read kept in an LDS slab) and the wide replay both
    # equal the oracle
    import paper_1702_07409_amd as fs
    fs.fs_set_tune(replay_lookahead=lookahead)
    try:
        decode_case(workloads.StripeSpec(**LOOKAHEAD_CASES[case]))
        li = fs.fs_last_launch()
        if lookahead == 0 and case in WIDE_REPLAY_WIDTH:
            assert (li["replay_kind"], li["replay_slice_bytes"]) == (2, WIDE_REPLAY_WIDTH[case]), li
        # with the lookahead tuning its kernel is launched (it falls back to
        # wide slices inside when the slab does not fit); without, the wide one
        assert li["replay_kind"] == (3 if lookahead else 2), li
    finally:
        fs.fs_reset_tune()


@pytest.mark.parametrize("maxit", [1, 3, 7])
def test_decode_lookahead_replay_maxit(maxit):
    import paper_1702_07409_amd as fs
    fs.fs_set_tune(replay_lookahead=1)
    try:
        decode_case(workloads.StripeSpec(**LOOKAHEAD_CASES["prefetched"]), maxit)
    finally:
        fs.fs_reset_tune()


def test_decode_lookahead_replay_large_stripe():
    # the full-size stripe through the lookahead replay (32-byte slices; the
    # default wide replay is covered by the full-size test above)
    import paper_1702_07409_amd as fs
    fs.fs_set_tune(replay_lookahead=1)
    try:
        decode_case(workloads.large_stripe())
    finally:
        fs.fs_reset_tune()


def test_decode_lookahead_plan_without_its_program():
    # a plan made without the lookahead program, applied with the lookahead
    # replay asked for: the kernel finds the program unusable and runs the
    # wide replay
    import paper_1702_07409_amd as fs
    sp = workloads.StripeSpec(**LOOKAHEAD_CASES["rsd"])
    g, G = spec_graphs(sp)
    x = sp.x()
    c_host = codec.encode(G, x)
    er = sp.erased_mask()
    xo, reco, sto, _ = oracle_decode(G, c_host, er, 0)
    ws = fs.workspace(g, fs.FS_OP_DECODE, sp.t)
    rec, st = empty_u8(sp.k), empty_i32(3)
    out = empty_u8((sp.k, sp.t))
    fs.fs_decode_plan(g, dev(er), 0, rec, st, ws)
    fs.fs_set_tune(replay_lookahead=1)
    try:
        fs.fs_decode_apply(g, dev(c_host), out, sp.t, ws)
    finally:
        fs.fs_reset_tune()
    assert host(st).tolist() == list(sto)
    assert np.array_equal(host(out), xo)


def test_decode_wide_replay_with_more_than_65535_rows():
    # n > 65535: no 16-bit program, the replay reads its program from global memory
    sp = workloads.StripeSpec(stripe=5, k=2000, n=70000, t=32, dist="rsd", stripe_key=3, n_erased=7000)
    _, G, got, sched = decode_case(sp)
    assert got.status[0] == 1


def test_peel_replay_equals_decode_and_is_deterministic():
    import paper_1702_07409_amd as fs
    sp = workloads.large_stripe()
    sp = workloads.scaled(sp, 1024)
    g, G = spec_graphs(sp)
    x = sp.x()
    c = dev(codec.encode(G, x))
    er = sp.erased_mask()
    a = gpu_decode(g, c, er, sp.t)
    b = gpu_decode(g, c, er, sp.t)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.status, b.status)
    p = gpu_peel(g, er)
    x2 = empty_u8(sp.k, sp.t)
    st = dev(p.status)
    lp = empty_i32(sp.k + 1)
    lp[:len(p.level_ptr)] = dev(p.level_ptr)
    fs.fs_replay(g, c, st, lp, dev(p.dp_f), dev(p.dp_g), x2, sp.t, fs.workspace(g, fs.FS_OP_REPLAY, sp.t))
    assert np.array_equal(host(x2), a.x)


def test_decode_plan_applied_to_several_stripes():
    # one plan (schedule + replay program) serves every stripe that shares the
    # graph and the erasure pattern
    import paper_1702_07409_amd as fs
    for sp in (workloads.tiny(), workloads.scaled(workloads.large_stripe(), 2048)):
        g, G = spec_graphs(sp)
        er = sp.erased_mask()
        rec, st = empty_u8(sp.k), empty_i32(3)
        ws = fs.workspace(g, fs.FS_OP_DECODE, sp.t)
        fs.fs_decode_plan(g, dev(er), 0, rec, st, ws)
        for stripe in (0, 7):
            x = gen.payload(0, stripe, sp.k, sp.t)
            c_host = codec.encode(G, x)
            xd = empty_u8(sp.k, sp.t)
            xd.fill_(0x3C)
            fs.fs_decode_apply(g, dev(c_host), xd, sp.t, ws)
            xo, reco, sto, _ = oracle_decode(G, c_host, er)
            assert np.array_equal(host(xd), xo)
            assert np.array_equal(host(rec), reco) and host(st).tolist() == list(sto)


# ---------------------------------------------------------------- repair

def test_repair_from_inputs():
    import paper_1702_07409_amd as fs
    sp = workloads.resident256(2)[1]
    sp = workloads.scaled(sp, 4096)
    g, G = spec_graphs(sp)
    x = sp.x()
    c_host = codec.encode(G, x)
    lost = sp.extra["lost"]
    c = dev(c_host)
    c[lost] = 0
    rep, st = empty_u8(len(lost)), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_REPAIR, sp.t, len(lost))
    fs.fs_repair(g, dev(x), c, None, dev(np.array(lost, np.uint32)), len(lost), rep, st, sp.t, ws)
    assert np.array_equal(host(c), c_host)
    assert host(rep).tolist() == [1] * len(lost) and host(st).tolist() == [1, 0, 0]


@pytest.mark.parametrize("tile", [(0, 0), (16, 2), (256, 1)])
def test_repair_from_inputs_long_rows(tile):
    # lost rows of hundreds of inputs are cut into 64-edge pieces that XOR
    # into the zeroed row (with a row of exactly 64, one of 65 and short ones
    # beside them); the row-wide and default tilings and a ragged block
    import paper_1702_07409_amd as fs
    sp = workloads.StripeSpec(stripe=11, k=2000, n=2200, t=1024 + 48, dist="rsd", rsd_c=0.05, rsd_delta=0.01,
                              stripe_key=11)
    g, G = spec_graphs(sp)
    deg = G.degrees()
    heavy = [int(j) for j in np.argsort(-deg)[:3]]
    assert deg[heavy[0]] > 200
    lost = heavy + [int(j) for j in np.flatnonzero(deg == 1)[:2]]
    for d in (64, 65, 128):
        rows = np.flatnonzero(deg == d)
        if len(rows):
            lost.append(int(rows[0]))
    x = sp.x()
    c_host = codec.encode(G, x)
    c = dev(c_host)
    c[lost] = 0x5a
    rep, st = empty_u8(len(lost)), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_REPAIR, sp.t, len(lost))
    fs.fs_set_tune(tile[0], tile[1], 1, 1)
    try:
        fs.fs_repair(g, dev(x), c, None, dev(np.array(lost, np.uint32)), len(lost), rep, st, sp.t, ws)
    finally:
        fs.fs_reset_tune()
    assert np.array_equal(host(c), c_host)
    assert host(rep).tolist() == [1] * len(lost) and host(st).tolist() == [1, 0, 0]


def test_repair_conventional():
    import paper_1702_07409_amd as fs
    sp = workloads.StripeSpec(stripe=2, k=64, n=96, t=512, dist="rsd", graph_seed=2, n_erased=4)
    g, G = spec_graphs(sp)
    x = sp.x()
    c_host = codec.encode(G, x)
    er = sp.erased_mask()
    # rows that the conventional repair can and cannot rebuild
    lost = [j for j in range(sp.n) if not er[j]][:12]
    want, ok = codec.repair_conventional(G, c_host, er, lost)
    assert 0 < ok.sum() < len(lost)
    c = dev(c_host)
    c[lost] = 0x77
    rep, st = empty_u8(len(lost)), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_REPAIR_CONVENTIONAL, sp.t, len(lost))
    fs.fs_repair(g, None, c, dev(er), dev(np.array(lost, np.uint32)), len(lost), rep, st, sp.t, ws)
    got = host(c)
    assert np.array_equal(host(rep), ok)
    assert np.array_equal(got[lost], want)
    others = [j for j in range(sp.n) if j not in lost]
    assert np.array_equal(got[others], c_host[others])
    assert host(st).tolist() == [0, int(len(lost) - ok.sum()), 0]


def test_repair_rejects_bad_lost_ids_without_writing():
    import paper_1702_07409_amd as fs
    sp = workloads.tiny()
    g, G = spec_graphs(sp)
    x = sp.x()
    c_host = codec.encode(G, x)
    for lost in ([3, 96], [5, 9, 5]):
        for mode_a in (True, False):
            c = dev(c_host)
            rep, st = empty_u8(len(lost)), empty_i32(3)
            op = fs.FS_OP_REPAIR if mode_a else fs.FS_OP_REPAIR_CONVENTIONAL
            ws = fs.workspace(g, op, sp.t, len(lost))
            fs.fs_repair(g, dev(x) if mode_a else None, c, None, dev(np.array(lost, np.uint32)),
                         len(lost), rep, st, sp.t, ws)
            assert np.array_equal(host(c), c_host)
            assert host(st).tolist() == [0, len(lost), fs._lib.FS_ERR_INVALID]
            assert not host(rep).any()


# ---------------------------------------------------------------- update

def update_case(sp, ids, t=None):
    import paper_1702_07409_amd as fs
    g, G = spec_graphs(sp)
    x = sp.x()
    c_host = codec.encode(G, x)
    new = gen.update_blocks(workloads.UPDATE_DATA_SEED, sp.stripe, ids, sp.t)
    xd, cd = dev(x), dev(c_host)
    st = empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_UPDATE, sp.t, len(ids))
    fs.fs_update(g, xd, cd, dev(np.array(ids, np.uint32)), len(ids), dev(new), st, sp.t, ws)
    return G, x, c_host, new, host(xd), host(cd), host(st)


def test_update_equals_reencode():
    sp = workloads.scaled(workloads.resident256(1)[0], 8192)
    ids = sp.extra["update_ids"]
    G, x, c_host, new, xg, cg, st = update_case(sp, ids)
    x2, c2 = codec.update(G, x, ids, new)
    assert np.array_equal(xg, x2) and np.array_equal(cg, c2)
    aff = codec.affected_rows(G, ids)
    assert st.tolist() == [len(aff), sum(len(G.NT(i)) for i in ids), 0]


def test_update_rejects_bad_ids_without_writing():
    sp = workloads.tiny()
    for ids in ([1, 64], [3, 4, 3]):
        G, x, c_host, new, xg, cg, st = update_case(sp, ids)
        assert np.array_equal(xg, x) and np.array_equal(cg, c_host)
        assert st.tolist()[2] != 0


def test_update_all_inputs():
    sp = workloads.tiny()
    ids = list(range(sp.k))[::-1]
    G, x, c_host, new, xg, cg, st = update_case(sp, ids)
    x2, c2 = codec.update(G, x, ids, new)
    assert np.array_equal(xg, x2) and np.array_equal(cg, c2)
