"""Helpers for the GPU parity tests: device tensors, and the same stripe built
by the library and by the oracle."""

import numpy as np

from oracle import codec, graph


def torch():
    import torch as _t
    return _t


def dev(a, dtype=None):
    t = torch()
    arr = np.ascontiguousarray(a)
    out = t.from_numpy(arr).to("cuda")
    return out if dtype is None else out.to(dtype)


def host(t):
    torch().cuda.synchronize()
    return t.detach().cpu().numpy()


def empty_u8(*shape):
    return torch().empty(*shape, dtype=torch().uint8, device="cuda")


def empty_i32(*shape):
    return torch().empty(*shape, dtype=torch().int32, device="cuda")


def graphs(**kw):
    """(library graph, oracle graph) for the same parameters.  The seed is
    always passed explicitly: the two builders' defaults differ."""
    import paper_1702_07409_amd as fs
    kw.setdefault("seed", graph.GraphParams(k=1, n=1).seed)
    g = fs.fs_graph_build(**kw)
    G = graph.build(graph.GraphParams(**kw))
    return g, G


class Decoded:
    def __init__(self, x, recovered, status, level_ptr=None, dp_f=None, dp_g=None):
        self.x, self.recovered, self.status = x, recovered, status
        self.level_ptr, self.dp_f, self.dp_g = level_ptr, dp_f, dp_g


def gpu_peel(g, erased, maxit=0):
    import paper_1702_07409_amd as fs
    k = g.k
    rec, st = empty_u8(k), empty_i32(3)
    lp, df, dg = empty_i32(k + 1), empty_i32(k), empty_i32(k)
    ws = fs.workspace(g, fs.FS_OP_PEEL)
    fs.fs_peel(g, dev(erased.astype(np.uint8)), maxit, rec, st, lp, df, dg, ws)
    st_h = host(st)
    L = int(st_h[2])
    return Decoded(None, host(rec), st_h, host(lp)[:L + 1], host(df), host(dg))


def gpu_decode(g, c_dev, erased, t, maxit=0):
    import paper_1702_07409_amd as fs
    k = g.k
    x = empty_u8(k, t)
    x.fill_(0xA5)        # every byte must be overwritten (recovered or zero-filled)
    rec, st = empty_u8(k), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_DECODE, t)
    fs.fs_decode(g, c_dev, dev(erased.astype(np.uint8)), maxit, x, rec, st, t, ws)
    return Decoded(host(x), host(rec), host(st))


def check_schedule(sched, got):
    """Library schedule == oracle schedule, element by element."""
    lp, df, dg = sched.flat()
    assert list(got.status) == list(sched.status()), (got.status, sched.status())
    assert np.array_equal(got.level_ptr, lp)
    nR = int(lp[-1])
    assert np.array_equal(got.dp_f[:nR], df)
    assert np.array_equal(got.dp_g[:nR], dg)
    assert np.array_equal(got.dp_f[nR:], sched.F)
    assert np.all(got.dp_g[nR:] == -1)
    assert np.array_equal(got.recovered, sched.recovered_mask())


def oracle_decode(G, c, erased, maxit=0):
    return codec.decode(G, c, erased.astype(np.uint8), maxit)
