"""Repair and update on resident stripes at their full block size: k = 1024
inputs x 256 KiB, n = 1126 coded blocks, Robust Soliton (c = 0.1, delta =
0.05), one graph per stripe, the seeded lost rows and updated inputs of the
resident batch.  The plain calls and batched plans of two stripes are compared
with the oracle element by element (repair: re-encoding the lost rows from the
inputs; update: re-encoding every row from the updated inputs)."""

import numpy as np
import pytest

from gpu_util import dev, empty_i32, empty_u8, graphs, host
from oracle import codec
from synth import gen, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stripes():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = []
    for sp in workloads.resident256(2):
        assert sp.t == 262144 and sp.k == 1024 and sp.n == 1126
        g, G = graphs(**sp.graph_kwargs())
        x = sp.x()
        c = codec.encode(G, x)
        ids = sp.extra["update_ids"]
        new = gen.update_blocks(workloads.UPDATE_DATA_SEED, sp.stripe, ids, sp.t)
        x2, c2 = codec.update(G, x, ids, new)
        lost = sp.extra["lost"]
        out.append(dict(sp=sp, g=g, G=G, x=x, c=c, lost=lost, ids=ids, new=new, x2=x2, c2=c2,
                        rebuilt=codec.repair_from_inputs(G, x, lost)))
    return out


def _repair_args(d):
    c = dev(d["c"])
    c[d["lost"]] = 0
    return c, dev(np.array(d["lost"], np.uint32)), empty_u8(len(d["lost"])), empty_i32(3)


def _check_repair(d, c, rep, st):
    got = host(c)
    assert np.array_equal(got[d["lost"]], d["rebuilt"])
    assert np.array_equal(got, d["c"])
    assert host(rep).tolist() == [1] * len(d["lost"]) and host(st).tolist() == [1, 0, 0]


def _check_update(d, xd, cd):
    assert np.array_equal(host(xd), d["x2"])
    assert np.array_equal(host(cd), d["c2"])


def test_plain_repair_and_update_full_size(stripes):
    import paper_1702_07409_amd as fs
    for d in stripes:
        sp = d["sp"]
        print("stripe %d: lost %s, %d updated inputs" % (sp.stripe, d["lost"], len(d["ids"])), flush=True)
        c, lost, rep, st = _repair_args(d)
        ws = fs.workspace(d["g"], fs.FS_OP_REPAIR, sp.t, len(d["lost"]))
        fs.fs_repair(d["g"], dev(d["x"]), c, None, lost, len(d["lost"]), rep, st, sp.t, ws)
        _check_repair(d, c, rep, st)
        xd, cd, ust = dev(d["x"]), dev(d["c"]), empty_i32(3)
        ws = fs.workspace(d["g"], fs.FS_OP_UPDATE, sp.t, len(d["ids"]))
        fs.fs_update(d["g"], xd, cd, dev(np.array(d["ids"], np.uint32)), len(d["ids"]), dev(d["new"]), ust,
                     sp.t, ws)
        _check_update(d, xd, cd)
        aff = codec.affected_rows(d["G"], d["ids"])
        assert host(ust).tolist() == [len(aff), sum(len(d["G"].NT(i)) for i in d["ids"]), 0]


@pytest.mark.parametrize("autotune", [False, True])
def test_batched_repair_and_update_full_size(stripes, autotune):
    import paper_1702_07409_amd as fs
    import torch
    reps, upds = [], []
    for d in stripes:
        sp = d["sp"]
        c, lost, rep, st = _repair_args(d)
        reps.append((d, c, rep, st, fs.work("repair", d["g"], sp.t, x=dev(d["x"]), c=c, ids=lost,
                                              n_ids=len(d["lost"]), repaired=rep, status=st)))
        xd, cd, ust = dev(d["x"]), dev(d["c"]), empty_i32(3)
        upds.append((d, xd, cd, fs.work("update", d["g"], sp.t, x=xd, c=cd,
                                        ids=dev(np.array(d["ids"], np.uint32)), n_ids=len(d["ids"]),
                                        new_blocks=dev(d["new"]), status=ust)))
    rplan = fs.Plan([r[-1] for r in reps], autotune=autotune)
    rplan.launch()
    torch.cuda.synchronize()
    for d, c, rep, st, _ in reps:
        _check_repair(d, c, rep, st)
    uplan = fs.Plan([u[-1] for u in upds], autotune=autotune)
    uplan.launch()
    torch.cuda.synchronize()
    for d, xd, cd, _ in upds:
        _check_update(d, xd, cd)
    # a second launch carries zero deltas: nothing changes
    uplan.launch()
    torch.cuda.synchronize()
    for d, xd, cd, _ in upds:
        _check_update(d, xd, cd)
