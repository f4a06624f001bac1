"""The C-ABI library loads, exports what include/fs_api.h declares, and its
host-side graph builder agrees with the oracle (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import dist, graph
from synth import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fs_api.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_1702_07409_amd._lib as L
    lib = ctypes.CDLL(L.LIB_PATH)
    declared = header_functions()
    assert "fs_encode" in declared and "fs_decode" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) <= set(L.EXPORTED)
    assert "gfx950" in L.version()


def test_library_hides_internal_symbols():
    import subprocess
    import paper_1702_07409_amd._lib as L
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    syms = [ln.split()[-1] for ln in out.splitlines() if " T " in ln]
    assert all(s.startswith("fs_") for s in syms), [s for s in syms if not s.startswith("fs_")][:5]


def oracle_params(**kw):
    return graph.GraphParams(**kw)


CASES = [
    dict(k=64, n=96, dist="rsd", rsd_c=0.1, rsd_delta=0.05, seed=1),
    dict(k=1, n=3, dist="rsd", rsd_c=0.1, rsd_delta=0.05, seed=5),
    dict(k=1024, n=1126, dist="rsd", rsd_c=0.1, rsd_delta=0.05, seed=1, stripe_key=17),
    dict(k=4096, n=4506, dist="finite", finite_w=workloads.finite16_weights(), seed=1),
    dict(k=300, n=500, dist="raptor", seed=2**62 + 3, stripe_key=2**40),
    dict(k=40, n=70, dist="raptor", seed=9),
    dict(k=8, n=20, dist="finite", finite_w=(0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0), seed=3),
    dict(k=8041, n=8684, dist="rsd", rsd_c=0.05, rsd_delta=0.01, seed=1, stripe_key=300),
    # n >= 8192: rows and columns are built by several host threads
    dict(k=12000, n=13300, dist="rsd", rsd_c=0.1, rsd_delta=0.05, seed=1, stripe_key=0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-k%d" % (c["dist"], c["k"]))
def test_degree_table_matches_oracle(case):
    import paper_1702_07409_amd as fs
    kw = dict(case)
    G = oracle_params(**kw)
    want = dist.thresholds(graph.degree_weights(G))
    got = fs.fs_degree_table(**{k: v for k, v in kw.items()})
    assert got == want


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-k%d" % (c["dist"], c["k"]))
def test_host_graph_matches_oracle(case):
    import paper_1702_07409_amd as fs
    g = fs.fs_graph_build(host_only=True, **case)
    rp, col, cp, ri = g.export()
    G = graph.build(oracle_params(**case))
    assert g.nnz == G.nnz
    assert np.array_equal(rp, G.row_ptr)
    assert np.array_equal(col, G.col)
    assert np.array_equal(cp, G.col_ptr)
    assert np.array_equal(ri, G.rowidx)
    assert g.max_degree == int(G.degrees().max())
    assert g.max_column_degree == int(np.diff(G.col_ptr).max())


def test_invalid_parameters_are_errors():
    import paper_1702_07409_amd as fs
    from paper_1702_07409_amd._lib import FS_ERR_INVALID
    bad = [dict(k=0, n=5), dict(k=5, n=0), dict(k=10, n=5, rsd_c=0.0),
           dict(k=10, n=5, rsd_delta=1.0), dict(k=1, n=5, rsd_c=0.001, rsd_delta=0.9),
           dict(k=10, n=5, dist="finite", finite_w=()),
           dict(k=10, n=5, dist="finite", finite_w=(0.0, 0.0)),
           dict(k=10, n=5, dist="finite", finite_w=(0.5, -0.1)),
           dict(k=3, n=5, dist="finite", finite_w=(0.0, 0.0, 0.0, 1.0))]
    for kw in bad:
        with pytest.raises(fs.FsError) as e:
            fs.fs_graph_build(host_only=True, **kw)
        assert e.value.status == FS_ERR_INVALID, kw


def test_workspace_sizes_and_host_only_graph_rejects_payload_calls():
    import paper_1702_07409_amd as fs
    g = fs.fs_graph_build(64, 96, seed=1, host_only=True)
    assert fs.fs_workspace_size(g, fs.FS_OP_ENCODE) == 0
    assert fs.fs_workspace_size(g, fs.FS_OP_PEEL) > 0
    assert fs.fs_workspace_size(g, fs.FS_OP_DECODE) > fs.fs_workspace_size(g, fs.FS_OP_PEEL)
    conv = fs.fs_workspace_size(g, fs.FS_OP_REPAIR_CONVENTIONAL, 4096)
    assert conv >= 64 * 4096
    assert fs.fs_workspace_size(g, fs.FS_OP_UPDATE, 4096, 10) >= 10 * 4096
    with pytest.raises(fs.FsError):
        fs.fs_workspace_size(g, fs.FS_OP_UPDATE, 4100, 10)


def test_graph_image_size_covers_every_array():
    import paper_1702_07409_amd as fs
    g = fs.fs_graph_build(k=300, n=330, dist="rsd", rsd_c=0.05, rsd_delta=0.01, seed=1, host_only=True)
    rp, col, cp, ri = g.export()
    al = lambda b: (b + 255) // 256 * 256
    # CSR, CSC, the encode segments (at most one per 64 edges plus one per
    # row) and their edge list
    base = al(rp.nbytes) + al(col.nbytes) + al(cp.nbytes) + al(ri.nbytes) + al(col.nbytes)
    size = g.image_size()
    assert size % 256 == 0 and size >= base + 256
    segs = sum(-(-int(rp[j + 1] - rp[j]) // 64) for j in range(g.n))
    assert size <= base + al(4 * (segs + 1)) + al(4 * segs) + al(4 * g.n) + al(segs) + 256


@pytest.mark.parametrize("b,k", [(28, 49), (925, 1036), (9919, 10246), (10, 15), (110, 121)])
def test_host_precode_matches_oracle(b, k):
    import paper_1702_07409_amd as fs
    from oracle import precode
    pc = fs.fs_precode_build(b, k, host_only=True)
    p, kp, jp = precode.array_params(b, k)
    assert (pc.b, pc.k, pc.p, pc.kp, pc.jp) == (b, k, p, kp, jp)
    rp, col = pc.export()
    L = precode.check_one(b, k)
    assert rp.tolist() == [r * (kp - jp) for r in range(k - b + 1)]
    assert [sorted(row) for row in L] == [col[rp[r]:rp[r + 1]].tolist() for r in range(k - b)]


@pytest.mark.parametrize("b,k", [(27, 49), (49, 49), (0, 49), (3, 7), (5, 1)])
def test_precode_rejects_bad_parameters(b, k):
    import paper_1702_07409_amd as fs
    with pytest.raises(fs.FsError):
        fs.fs_precode_build(b, k, host_only=True)


def test_graph_build_rejects_conflicting_flags():
    # host-only and on-device builds exclude each other (checked before any HIP call)
    import paper_1702_07409_amd as fs
    with pytest.raises(fs.FsError) as e:
        fs.fs_graph_build(k=64, n=96, host_only=True, on_device=True)
    assert e.value.status == fs._lib.FS_ERR_INVALID


def test_workspace_size_knows_every_operation():
    # every FS_OP_* the header declares sizes a workspace (host-only graph, no GPU)
    import paper_1702_07409_amd as fs
    text = open(os.path.join(ROOT, "include", "fs_api.h")).read()
    ops = re.findall(r"\b(FS_OP_[A-Z_]+)\s*=\s*(\d+)", text)
    assert len(ops) >= 14
    g = fs.fs_graph_build(k=64, n=96, host_only=True)
    for name, code in ops:
        assert getattr(fs, name) == int(code), name
        # the encode needs none; every other operation some
        assert (fs.fs_workspace_size(g, int(code), 4096, 4) > 0) == (name != "FS_OP_ENCODE"), name


def test_graph_and_table_reject_out_of_range_parameters():
    # checked on the host before any HIP call
    import ctypes
    from paper_1702_07409_amd import _lib as L
    # more inputs than the builds support, a reserved field, unknown flags and distribution
    p = L.make_params(k=(1 << 20) + 1, n=5, host_only=True)
    h = L.P()
    assert L._lib.fs_graph_build(ctypes.byref(p), None, ctypes.byref(h)) == L.FS_ERR_INVALID
    p = L.make_params(k=10, n=5, host_only=True)
    p.reserved = 1
    assert L._lib.fs_graph_build(ctypes.byref(p), None, ctypes.byref(h)) == L.FS_ERR_INVALID
    p = L.make_params(k=10, n=5, host_only=True)
    p.flags |= 8
    assert L._lib.fs_graph_build(ctypes.byref(p), None, ctypes.byref(h)) == L.FS_ERR_INVALID
    p = L.make_params(k=10, n=5, host_only=True)
    p.dist = 7
    assert L._lib.fs_graph_build(ctypes.byref(p), None, ctypes.byref(h)) == L.FS_ERR_INVALID
    # the threshold table: a buffer shorter than D is refused, D is still reported
    p = L.make_params(k=100, n=1)
    D = L.U32()
    assert L._lib.fs_degree_table(ctypes.byref(p), None, 0, ctypes.byref(D)) == 0 and D.value == 100
    buf = (ctypes.c_uint64 * 10)()
    assert L._lib.fs_degree_table(ctypes.byref(p), buf, 10, ctypes.byref(D)) == L.FS_ERR_INVALID
    assert "threshold" in L._lib.fs_last_error().decode()


def test_status_strings_name_every_status():
    from paper_1702_07409_amd import _lib as L
    names = {L._lib.fs_status_string(s).decode() for s in range(7)}
    assert len(names) == 7 and "unknown status" not in names
    assert L._lib.fs_status_string(99).decode() == "unknown status"
