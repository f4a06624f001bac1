"""Batched plans (one captured launch for many stripes) give the oracle's
results bit for bit; graph replays, rebinds and the autotuner keep them."""

import dataclasses
import os
import tempfile

import numpy as np
import pytest

from gpu_util import dev, empty_i32, empty_u8, graphs, host
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


def S(**kw):
    return workloads.StripeSpec(**kw)


# stripes of uneven k, block size and distribution (one graph each)
ENC = [S(stripe=20, k=64, n=96, t=4096, dist="rsd", stripe_key=20),
       S(stripe=21, k=2000, n=2160, t=1024 + 16, dist="rsd", rsd_c=0.05, rsd_delta=0.01, stripe_key=21),
       S(stripe=22, k=512, n=563, t=8192, dist="finite", finite_w=workloads.finite16_weights(), stripe_key=22)]
DEC = [S(stripe=30, k=64, n=96, t=4096, dist="rsd", stripe_key=30, n_erased=16),
       S(stripe=31, k=500, n=1000, t=512 + 32, dist="rsd", stripe_key=31, n_erased=100),
       S(stripe=32, k=3000, n=3300, t=2048, dist="finite", finite_w=workloads.finite16_weights(),
         stripe_key=32, n_erased=165)]
# repair stripes and their lost rows: short rows, and rows of hundreds of
# inputs (cut into 64-edge pieces that XOR into the zeroed row)
REP = [(S(stripe=40, k=1024, n=1126, t=4096, dist="rsd", stripe_key=40), lambda G: [5, 77, 1100]),
       (S(stripe=41, k=2000, n=2200, t=1024 + 48, dist="rsd", rsd_c=0.05, rsd_delta=0.01, stripe_key=41),
        lambda G: [int(j) for j in np.argsort(-G.degrees())[:2]] + [3])]
UPD = [S(stripe=50, k=1024, n=1126, t=2048, dist="rsd", stripe_key=50)]


class Batch:
    """Buffers of one batch and the oracle's expected outputs."""

    def __init__(self, data_seed=0):
        import paper_1702_07409_amd as fs
        self.items, self.checks = [], []
        for sp in ENC:
            g, G = graphs(**sp.graph_kwargs())
            x = gen.payload(data_seed, sp.stripe, sp.k, sp.t)
            c = empty_u8(sp.n, sp.t)
            c.fill_(0xEE)
            self.items.append(fs.work("encode", g, sp.t, x=dev(x), c=c))
            want = codec.encode(G, x)
            self.checks.append(lambda c=c, want=want: np.array_equal(host(c), want))
        for sp in DEC:
            g, G = graphs(**sp.graph_kwargs())
            x = gen.payload(data_seed, sp.stripe, sp.k, sp.t)
            c_host = codec.encode(G, x)
            er = sp.erased_mask()
            xo = empty_u8(sp.k, sp.t)
            xo.fill_(0x11)
            rec, st = empty_u8(sp.k), empty_i32(3)
            self.items.append(fs.work("decode", g, sp.t, x=xo, c=dev(c_host), erased=dev(er), recovered=rec,
                                      status=st))
            xw, recw, stw, _ = codec.decode(G, c_host, er)
            self.checks.append(lambda xo=xo, rec=rec, st=st, xw=xw, recw=recw, stw=stw:
                               np.array_equal(host(xo), xw) and np.array_equal(host(rec), recw)
                               and host(st).tolist() == list(stw))
        for sp, lost_of in REP:
            g, G = graphs(**sp.graph_kwargs())
            x = gen.payload(data_seed, sp.stripe, sp.k, sp.t)
            c_host = codec.encode(G, x)
            lost = lost_of(G)
            c = dev(c_host)
            c[lost] = 0
            rep, st = empty_u8(len(lost)), empty_i32(3)
            self.items.append(fs.work("repair", g, sp.t, x=dev(x), c=c, ids=dev(np.array(lost, np.uint32)),
                                      n_ids=len(lost), repaired=rep, status=st))
            self.checks.append(lambda c=c, want=c_host, rep=rep, st=st, m=len(lost):
                               np.array_equal(host(c), want) and host(rep).tolist() == [1] * m
                               and host(st).tolist() == [1, 0, 0])
        for sp in UPD:
            g, G = graphs(**sp.graph_kwargs())
            x = gen.payload(data_seed, sp.stripe, sp.k, sp.t)
            c_host = codec.encode(G, x)
            ids = gen.update_ids(workloads.UPDATE_IDS_SEED, sp.stripe, sp.k, 10)
            new = gen.update_blocks(workloads.UPDATE_DATA_SEED + data_seed, sp.stripe, ids, sp.t)
            xd, cd, st = dev(x), dev(c_host), empty_i32(3)
            self.items.append(fs.work("update", g, sp.t, x=xd, c=cd, ids=dev(np.array(ids, np.uint32)),
                                      n_ids=len(ids), new_blocks=dev(new), status=st))
            x2, c2 = codec.update(G, x, ids, new)
            self.checks.append(lambda xd=xd, cd=cd, x2=x2, c2=c2: np.array_equal(host(xd), x2)
                               and np.array_equal(host(cd), c2))

    def verify(self):
        bad = [i for i, ok in enumerate(self.checks) if not ok()]
        assert not bad, "items differing from the oracle: %s" % bad


def test_plan_mixed_batch_and_graph_replays():
    import paper_1702_07409_amd as fs
    import torch
    b = Batch()
    plan = fs.Plan(b.items)
    info = plan.info()
    assert info["items"] == len(b.items) and info["decode_items"] == len(DEC)
    for _ in range(3):
        plan.launch()
        torch.cuda.synchronize()
        b.verify()


def test_plan_without_graph_matches():
    import paper_1702_07409_amd as fs
    b = Batch(data_seed=3)
    plan = fs.Plan(b.items, graph=False)
    plan.launch()
    b.verify()


def test_plan_rebind_to_new_buffers():
    import paper_1702_07409_amd as fs
    a = Batch(data_seed=1)
    plan = fs.Plan(a.items)
    plan.launch()
    a.verify()
    b = Batch(data_seed=2)
    # same graphs are required: rebuild b's items on a's graphs
    items = []
    for wa, wb in zip(a.items, b.items):
        wb.graph = wa.graph
        wb._keep = wb._keep + (wa._keep[0],)
        items.append(wb)
    plan.rebind(items)
    plan.launch()
    b.verify()


# the autotuner's search space: tilings (0, 0 = the per-graph rule), XCD remap, store kind
TUNED_TILINGS = {(0, 0), (16, 1), (16, 2), (16, 4), (32, 1), (32, 2), (32, 4), (64, 1), (64, 2), (64, 4),
                 (128, 2), (256, 1), (256, 2)}


def test_plan_autotune_and_cache():
    import paper_1702_07409_amd as fs
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        b = Batch(data_seed=4)
        p1 = fs.Plan(b.items, tune_cache=path, autotune=True)
        i1 = p1.info()
        assert i1["tune_source"] == 1 and i1["tuned_ms"] > 0
        tu = i1["tune"]
        assert (tu["lanes_per_row"], tu["chunks"]) in TUNED_TILINGS
        assert tu["xcd_remap"] in (0, 1) and tu["nt_store"] in (0, 1) and tu["claim_chunk"] in (0, 1, 4, 32)
        p1.launch()
        b.verify()
        b2 = Batch(data_seed=4)
        p2 = fs.Plan(b2.items, tune_cache=path, autotune=True)
        i2 = p2.info()
        assert i2["tune_source"] == 2 and i2["tune"] == i1["tune"]
        p2.launch()
        b2.verify()


@pytest.mark.parametrize("lpr,ch", [(8, 1), (8, 2), (8, 4), (128, 1), (128, 2), (256, 1), (256, 2)])
def test_narrow_and_row_wide_tilings(lpr, ch):
    # 8 lanes per row (128-512 byte slices), and one or two rows per
    # workgroup: plans (encode, repair, the update's accumulate pass) and a
    # single-stripe encode with a ragged block
    import paper_1702_07409_amd as fs
    fs.fs_set_tune(lpr, ch, 1, 1)
    try:
        b = Batch(data_seed=6)
        fs.Plan(b.items).launch()
        b.verify()
        sp = S(stripe=23, k=300, n=450, t=8192 + 48, dist="rsd", stripe_key=23)
        g, G = graphs(**sp.graph_kwargs())
        x = gen.payload(0, sp.stripe, sp.k, sp.t)
        c = empty_u8(sp.n, sp.t)
        fs.fs_set_tune(lpr, ch, 1, 1, encode_slab=0)
        fs.fs_encode(g, dev(x), c, sp.t)
        assert np.array_equal(host(c), codec.encode(G, x))
        li = fs.fs_last_launch()
        assert (li["gather_lanes_per_row"], li["gather_chunks"]) == (lpr, ch), li
    finally:
        fs.fs_reset_tune()


def test_plan_rejects_bad_items():
    import paper_1702_07409_amd as fs
    sp = workloads.tiny()
    g, _ = graphs(**sp.graph_kwargs())
    c = empty_u8(sp.n, sp.t)
    st, rep = empty_i32(3), empty_u8(1)
    with pytest.raises(fs.FsError) as e:
        fs.Plan([fs.work("repair", g, sp.t, x=None, c=c, ids=dev(np.array([1], np.uint32)), n_ids=1,
                         repaired=rep, status=st)])
    assert e.value.status == fs._lib.FS_ERR_UNSUPPORTED
    with pytest.raises(fs.FsError) as e:
        fs.Plan([fs.work("encode", g, 4100, x=empty_u8(sp.k * 4112), c=empty_u8(sp.n * 4112))])
    assert e.value.status == fs._lib.FS_ERR_ALIGN


@pytest.mark.parametrize("staged", [False, True])
def test_plan_in_caller_memory(staged):
    import paper_1702_07409_amd as fs
    import torch
    b = Batch(data_seed=5)
    dev_bytes, stage_bytes = fs.plan_memory_size(b.items)
    assert 0 < stage_bytes < dev_bytes
    mem = torch.empty(dev_bytes, dtype=torch.uint8, device="cuda")
    stage = torch.empty(stage_bytes, dtype=torch.uint8, pin_memory=True) if staged else None
    s = torch.cuda.Stream()
    plan = fs.Plan(b.items, memory=mem, stage=stage, stream=s)
    plan.launch(stream=s)
    s.synchronize()
    b.verify()
    plan.free()
    with pytest.raises(fs.FsError) as e:
        fs.Plan(b.items, memory=mem[:1024], stream=s)
    assert e.value.status == fs._lib.FS_ERR_WORKSPACE
    if staged:
        with pytest.raises(fs.FsError) as e:
            fs.Plan(b.items, memory=mem, stage=stage[:16], stream=s)
        assert e.value.status == fs._lib.FS_ERR_WORKSPACE


def test_graph_in_caller_memory():
    import paper_1702_07409_amd as fs
    import torch
    sp = S(stripe=60, k=700, n=780, t=1024, dist="rsd", stripe_key=60)
    owned, G = graphs(**sp.graph_kwargs())
    x = dev(gen.payload(0, sp.stripe, sp.k, sp.t))
    want = codec.encode(G, host(x))
    for staged in (False, True):
        g = fs.fs_graph_build(host_only=True, **sp.graph_kwargs())
        nbytes = g.image_size()
        mem = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
        stage = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True) if staged else None
        s = torch.cuda.Stream()
        with pytest.raises(fs.FsError) as e:
            g.upload(mem[:64], stream=s)
        assert e.value.status == fs._lib.FS_ERR_WORKSPACE
        g.upload(mem, stage=stage, stream=s)
        c = empty_u8(sp.n, sp.t)
        fs.fs_encode(g, x, c, sp.t, stream=s)
        s.synchronize()
        assert np.array_equal(host(c), want)
        with pytest.raises(fs.FsError) as e:
            g.upload(mem, stream=s)
        assert e.value.status == fs._lib.FS_ERR_INVALID
        g.free()
    with pytest.raises(fs.FsError) as e:
        owned.upload(torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert e.value.status == fs._lib.FS_ERR_INVALID


def test_plan_with_large_items_and_rebind():
    """Stripes large enough to run as launches of their own (a 64 MiB encode,
    a 32 MiB decode, a device-sized update) next to small ones: the oracle's
    results on graph replays and after a rebind to new buffers."""
    import paper_1702_07409_amd as fs
    import torch
    big_enc = S(stripe=70, k=1024, n=1126, t=65536, dist="rsd", stripe_key=70)
    big_dec = S(stripe=71, k=1024, n=1126, t=32768, dist="finite", finite_w=workloads.finite16_weights(),
                stripe_key=71, n_erased=56)
    small = S(stripe=72, k=64, n=96, t=4096, dist="rsd", stripe_key=72)
    ge, Ge = graphs(**big_enc.graph_kwargs())
    gd, Gd = graphs(**big_dec.graph_kwargs())
    gs, Gs = graphs(**small.graph_kwargs())

    def make(seed):
        items, checks = [], []
        x = gen.payload(seed, big_enc.stripe, big_enc.k, big_enc.t)
        c = empty_u8(big_enc.n, big_enc.t)
        items.append(fs.work("encode", ge, big_enc.t, x=dev(x), c=c))
        want = codec.encode(Ge, x)
        checks.append(lambda c=c, want=want: np.array_equal(host(c), want))
        xd = gen.payload(seed, big_dec.stripe, big_dec.k, big_dec.t)
        cd = codec.encode(Gd, xd)
        er = big_dec.erased_mask()
        xo, rec, st = empty_u8(big_dec.k, big_dec.t), empty_u8(big_dec.k), empty_i32(3)
        items.append(fs.work("decode", gd, big_dec.t, x=xo, c=dev(cd), erased=dev(er), recovered=rec, status=st))
        xw, recw, stw, _ = codec.decode(Gd, cd, er)
        checks.append(lambda xo=xo, rec=rec, st=st, xw=xw, recw=recw, stw=stw:
                      np.array_equal(host(xo), xw) and np.array_equal(host(rec), recw)
                      and host(st).tolist() == list(stw))
        xs = gen.payload(seed, small.stripe, small.k, small.t)
        cs = empty_u8(small.n, small.t)
        items.append(fs.work("encode", gs, small.t, x=dev(xs), c=cs))
        wants = codec.encode(Gs, xs)
        checks.append(lambda cs=cs, wants=wants: np.array_equal(host(cs), wants))
        # a small decode after the large one: it shares the batched replay
        # while the large one replays on its own
        cs_host = codec.encode(Gs, xs)
        ers = dataclasses.replace(small, n_erased=12).erased_mask()
        xso, recs, sts = empty_u8(small.k, small.t), empty_u8(small.k), empty_i32(3)
        items.append(fs.work("decode", gs, small.t, x=xso, c=dev(cs_host), erased=dev(ers), recovered=recs,
                             status=sts))
        xsw, recsw, stsw, _ = codec.decode(Gs, cs_host, ers)
        checks.append(lambda xso=xso, recs=recs, sts=sts, xsw=xsw, recsw=recsw, stsw=stsw:
                      np.array_equal(host(xso), xsw) and np.array_equal(host(recs), recsw)
                      and host(sts).tolist() == list(stsw))
        return items, checks

    items, checks = make(10)
    plan = fs.Plan(items)
    assert plan.info()["gather_jobs"] == 2
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        bad = [i for i, ok in enumerate(checks) if not ok()]
        assert not bad, bad
    items2, checks2 = make(11)
    plan.rebind(items2)
    plan.launch()
    torch.cuda.synchronize()
    bad = [i for i, ok in enumerate(checks2) if not ok()]
    assert not bad, bad


def test_plan_peels_in_every_state_layout():
    """Decodes whose peel state fits LDS whole, by its 64-bit row counters,
    by its 32-bit row counters, and not at all, in one plan."""
    import paper_1702_07409_amd as fs
    specs = [S(stripe=80, k=64, n=96, t=64, dist="rsd", stripe_key=80, n_erased=10),
             S(stripe=81, k=16384, n=18022, t=16, dist="rsd", stripe_key=81, n_erased=900),
             S(stripe=82, k=10246, n=21800, t=32, dist="raptor", stripe_key=82, n_erased=1090),
             S(stripe=83, k=20000, n=22000, t=16, dist="rsd", stripe_key=83, n_erased=1100)]
    items, wants, outs = [], [], []
    for sp in specs:
        g, G = graphs(**sp.graph_kwargs())
        x = sp.x()
        c = codec.encode(G, x)
        er = sp.erased_mask()
        xo, rec, st = empty_u8(sp.k, sp.t), empty_u8(sp.k), empty_i32(3)
        items.append(fs.work("decode", g, sp.t, x=xo, c=dev(c), erased=dev(er), recovered=rec, status=st))
        wants.append(codec.decode(G, c, er)[:3])
        outs.append((xo, rec, st))
    plan = fs.Plan(items)
    for _ in range(2):
        plan.launch()
        for (xo, rec, st), (xw, recw, stw) in zip(outs, wants):
            assert host(st).tolist() == list(stw)
            assert np.array_equal(host(rec), recw) and np.array_equal(host(xo), xw)
