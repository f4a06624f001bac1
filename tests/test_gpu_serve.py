"""Serving: requests served in the mix (continuous batching, overlapping
ticks, admission by footprint) give exactly what each gives alone through the
plain one-call path, in arrival order, and what the oracle gives."""

import numpy as np
import pytest

from gpu_util import host
from oracle import codec, graph
from synth import serving, workloads

pytestmark = pytest.mark.gpu

HI = 2 << 20          # payload cap of this test (k <= 128 at 16 KiB blocks)
POOL = 10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_07409_amd as fs
    fs.fs_reset_tune()
    yield


def _served(rate, duration, budget, max_items=16):
    from paper_1702_07409_amd.serve import Request, Server
    srv = Server(budget=budget, streams=3, max_inflight=4, max_items=max_items, workers=4, keep_outputs=True)
    pool = serving.build_pool(srv, POOL, hi=HI)
    trace = workloads.serving_trace(rate=rate, duration=duration, pool_size=POOL, hi=HI)
    reqs = serving.build_requests(trace, pool, Request, hi=HI)
    stats = srv.run(reqs)
    return srv, pool, reqs, stats


def _alone(pool, reqs):
    """The same requests one at a time through the plain entry points, on a
    fresh pool, in arrival order; returns per-request outputs and the pool."""
    import torch
    import paper_1702_07409_amd as fs
    graphs, xs, cs = {}, [], []

    def G(p):
        key = (p["k"], p["n"])
        if key not in graphs:
            graphs[key] = fs.fs_graph_build(**p)
        return graphs[key]

    for sp in pool:
        p = serving.graph_params(sp)
        x = serving.payload_tensor(sp)
        c = torch.empty((sp.n, sp.t), dtype=torch.uint8, device="cuda")
        fs.fs_encode(G(p), x, c, sp.t)
        xs.append(x)
        cs.append(c)
    outs = []
    for r in reqs:
        if r.kind == "encode":
            g = G(r.params)
            c = torch.empty((g.n, r.t), dtype=torch.uint8, device="cuda")
            fs.fs_encode(g, r.x, c, r.t)
            outs.append({"c": c})
            continue
        sp = pool[r.stripe]
        g = G(serving.graph_params(sp))
        st = torch.full((3,), -7, dtype=torch.int32, device="cuda")
        if r.kind == "decode":
            out = torch.empty((g.k, r.t), dtype=torch.uint8, device="cuda")
            rec = torch.empty(g.k, dtype=torch.uint8, device="cuda")
            fs.fs_decode(g, cs[r.stripe], r.erased, 0, out, rec, st, r.t, fs.workspace(g, fs.FS_OP_DECODE, r.t))
            outs.append({"out": out, "recovered": rec, "status": st})
        elif r.kind == "repair":
            m = r.ids.numel()
            rep = torch.empty(m, dtype=torch.uint8, device="cuda")
            fs.fs_repair(g, xs[r.stripe], cs[r.stripe], None, r.ids, m, rep, st, r.t,
                         fs.workspace(g, fs.FS_OP_REPAIR, r.t, m))
            outs.append({"repaired": rep, "status": st})
        else:
            m = r.ids.numel()
            fs.fs_update(g, xs[r.stripe], cs[r.stripe], r.ids, m, r.new_blocks, st, r.t,
                         fs.workspace(g, fs.FS_OP_UPDATE, r.t, m))
            outs.append({"status": st})
    torch.cuda.synchronize()
    return outs, xs, cs


def _check_same(srv, reqs, outs, xs, cs):
    import torch
    bad = []
    for r, o in zip(reqs, outs):
        if r.kind == "encode":
            ok = torch.equal(r.c, o["c"])
        elif r.kind == "decode":
            ok = (torch.equal(r.out, o["out"]) and torch.equal(r.recovered, o["recovered"])
                  and torch.equal(r.status[:3], o["status"]))
        elif r.kind == "repair":
            ok = torch.equal(r.repaired, o["repaired"]) and torch.equal(r.status[:3], o["status"])
        else:
            ok = torch.equal(r.status[:3], o["status"])
        if not ok:
            bad.append((r.rid, r.kind))
    assert not bad, "served differs from alone: %s" % bad[:10]
    for sid, st in srv.stripes.items():
        assert torch.equal(st.x, xs[sid]) and torch.equal(st.c, cs[sid]), "resident stripe %d differs" % sid


def test_served_in_the_mix_equals_alone():
    # ~150 requests arriving within 3 ms: ticks overlap and batch several requests
    srv, pool, reqs, stats = _served(rate=50000.0, duration=0.003, budget=24 << 20)
    try:
        assert stats["requests"] == len(reqs) and len(reqs) > 100
        assert all(r.t_done is not None for r in reqs)
        assert max(srv.tick_items) > 1, "no tick batched more than one request"
        assert srv.peak_inflight > 1, "ticks never overlapped"
        kinds = {r.kind for r in reqs}
        assert kinds == {"encode", "decode", "repair", "update"}
        outs, xs, cs = _alone(pool, reqs)
        _check_same(srv, reqs, outs, xs, cs)
    finally:
        srv.close()


def test_served_small_requests_match_oracle():
    srv, pool, reqs, stats = _served(rate=20000.0, duration=0.004, budget=64 << 20)
    try:
        checked = 0
        for r in reqs:
            if r.kind == "encode" and r.params["k"] * r.t <= (1 << 20):
                G = graph.build(graph.GraphParams(**{k: v for k, v in r.params.items()}))
                assert np.array_equal(host(r.c), codec.encode(G, host(r.x))), "encode %d" % r.rid
                checked += 1
        assert checked >= 5
        # decodes of stripes that no update touched before them: compare with
        # the oracle decode of the stripe's original encoding
        touched = set()
        dec_checked = 0
        for r in reqs:
            if r.kind == "update":
                touched.add(r.stripe)
            elif r.kind == "decode" and r.stripe not in touched:
                sp = pool[r.stripe]
                if sp.k * sp.t > (2 << 20):
                    continue
                G = graph.build(graph.GraphParams(**serving.graph_params(sp)))
                x0 = host(serving.payload_tensor(sp))
                xw, recw, stw, _ = codec.decode(G, codec.encode(G, x0), host(r.erased))
                assert np.array_equal(host(r.out), xw) and np.array_equal(host(r.recovered), recw)
                assert host(r.status)[:3].tolist() == list(stw)
                dec_checked += 1
        assert dec_checked >= 1
    finally:
        srv.close()


def test_request_larger_than_budget_is_served_alone():
    srv, pool, reqs, stats = _served(rate=20000.0, duration=0.002, budget=1 << 20, max_items=4)
    try:
        assert all(r.t_done is not None for r in reqs)
        outs, xs, cs = _alone(pool, reqs)
        _check_same(srv, reqs, outs, xs, cs)
    finally:
        srv.close()


def test_budget_beyond_device_memory_skips_the_reservation():
    # run() reserves the budget in torch's caching allocator first; a budget
    # larger than the device is left unreserved and the requests are served
    from paper_1702_07409_amd.serve import Request, Server
    srv = Server(budget=1 << 50, streams=2, max_inflight=2, max_items=8, workers=2, keep_outputs=True)
    try:
        pool = serving.build_pool(srv, 4, hi=HI)
        trace = workloads.serving_trace(rate=20000.0, duration=0.001, pool_size=4, hi=HI)
        reqs = serving.build_requests(trace, pool, Request, hi=HI)
        stats = srv.run(reqs)
        assert stats["requests"] == len(reqs) and all(r.t_done is not None for r in reqs)
        outs, xs, cs = _alone(pool, reqs)
        _check_same(srv, reqs, outs, xs, cs)
    finally:
        srv.close()
