"""Graphs built by kernels on the device (FS_GRAPH_ON_DEVICE) are the host
construction's, array for array, and the oracle's; stripes coded with them
equal the oracle."""

import numpy as np
import pytest

from gpu_util import dev, empty_u8, gpu_decode, host
from oracle import codec, graph
from synth import gen, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


FIN16 = workloads.finite16_weights()
SEED = graph.GraphParams(k=1, n=1).seed
CASES = {
    "tiny_rsd": dict(k=64, n=96, dist="rsd", seed=1),
    "one_input": dict(k=1, n=5, dist="rsd", seed=2),
    "degree_k": dict(k=8, n=20, dist="finite", finite_w=(0,) * 7 + (1.0,), seed=3),
    # rows of exactly 64 and 128 neighbours: a segment boundary and two full pieces
    "segment_edges": dict(k=1000, n=300, dist="finite",
                          finite_w=tuple(0.5 if d in (5, 64, 128) else 0.0 for d in range(1, 129)), seed=4),
    "large_stripe": dict(k=4096, n=4506, dist="finite", finite_w=FIN16, seed=1),
    # Robust Soliton at k = 8192: rows of degree in the thousands
    "rsd_heavy": dict(k=8192, n=8847, dist="rsd", rsd_c=0.05, rsd_delta=0.01, seed=1, stripe_key=11),
    "raptor": dict(k=10246, n=21800, dist="raptor", seed=SEED),
    "rsd_16k": dict(k=16384, n=18022, dist="rsd", seed=7, stripe_key=3),
    # rows of k - 8 of k neighbours: Floyd batches full of fallback chains
    "nearly_full_rows": dict(k=2048, n=6, dist="finite", finite_w=(0,) * 2039 + (1.0,), seed=5),
    "full_rows_16k": dict(k=16384, n=3, dist="finite", finite_w=(0,) * 15999 + (1.0,), seed=6),
    # columns of ~31 and ~62 rows: one-wave column sorts, and columns of 65 and more rows
    "columns_31": dict(k=2048, n=8000, dist="finite", finite_w=(0,) * 7 + (1.0,), seed=7),
    "columns_62": dict(k=512, n=4000, dist="finite", finite_w=(0,) * 7 + (1.0,), seed=8),
    # columns of thousands of rows, then of more rows than one LDS bitmap covers
    "long_columns": dict(k=16, n=5000, dist="finite", finite_w=(0,) * 7 + (1.0,), seed=9),
    "long_columns_two_passes": dict(k=8, n=600000, dist="finite", finite_w=(0, 0, 0, 1.0), seed=10),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_device_graph_equals_host_and_oracle(case):
    import paper_1702_07409_amd as fs
    kw = CASES[case]
    gd = fs.fs_graph_build(on_device=True, **kw)
    gh = fs.fs_graph_build(host_only=True, **kw)
    assert (gd.k, gd.n, gd.nnz, gd.max_degree, gd.max_column_degree) == \
        (gh.k, gh.n, gh.nnz, gh.max_degree, gh.max_column_degree)
    for a, b in zip(gd.export(), gh.export()):
        assert np.array_equal(a, b)
    if kw["k"] <= 4096 and kw["n"] <= 30000:
        G = graph.build(graph.GraphParams(**kw))
        rp, col, cp, ri = gd.export()
        assert np.array_equal(rp, G.row_ptr) and np.array_equal(col, G.col)
        assert np.array_equal(cp, G.col_ptr) and np.array_equal(ri, G.rowidx)


@pytest.mark.parametrize("case", ["tiny_rsd", "segment_edges", "rsd_heavy"])
def test_device_graph_codes_like_the_oracle(case):
    # encode (segments, heavy rows combined atomically) and decode with the device-built graph
    import paper_1702_07409_amd as fs
    kw = CASES[case]
    gd = fs.fs_graph_build(on_device=True, **kw)
    G = graph.build(graph.GraphParams(**kw))
    t = 1024 + 48
    x = gen.payload(5, 1, kw["k"], t)
    c = empty_u8(kw["n"], t)
    fs.fs_encode(gd, dev(x), c, t)
    c_ref = codec.encode(G, x)
    assert np.array_equal(host(c), c_ref)
    er = np.zeros(kw["n"], np.uint8)
    er[gen.erasure_ids(2, 1, kw["n"], kw["n"] // 20)] = 1
    got = gpu_decode(gd, c, er, t)
    xo, reco, sto, _ = codec.decode(G, c_ref, er)
    assert list(got.status) == list(sto)
    assert np.array_equal(got.recovered, reco) and np.array_equal(got.x, xo)
