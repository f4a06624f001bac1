"""GPU parity of check #2/#3 generation (Algorithm 4) and local-group repair:
the equations equal the oracle's exactly, and repaired blocks equal the
oracle's bit for bit.

Run on an MI355X: pytest -m gpu.
"""

import numpy as np
import pytest

from gpu_util import dev, empty_i32, empty_u8, graphs, host
from oracle import checks, codec
from synth import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("k,n,dist,seed", [(2, 3, "rsd", 1), (20, 30, "rsd", 1), (64, 96, "rsd", 1),
                                           (200, 400, "raptor", 1), (100, 130, "raptor", 4)])
def test_checks_equal_the_oracle(k, n, dist, seed):
    import paper_1702_07409_amd as fs
    g, G = graphs(k=k, n=n, dist=dist, seed=seed)
    ch = fs.fs_checks_generate(g)
    b, L, sweeps = checks.cga(G)
    want2, want3 = checks.split(b, L)
    got2, got3 = ch.export()
    assert ch.sweeps == sweeps and ch.zero_columns == sum(1 for x in b if x == 0)
    assert got3 == want3 and got2 == want2


def test_sweep_limit():
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor", seed=2)
    for m in (1, 2):
        ch = fs.fs_checks_generate(g, max_sweeps=m)
        b, L, sweeps = checks.cga(G, max_sweeps=m)
        assert ch.sweeps == sweeps == m
        assert ch.export() == tuple(checks.split(b, L))


def test_paper_example_scale_identities():
    # the paper's illustrative code size (k = 500, n = 1000): every check #3
    # group XORs to zero and every check #2 equation gives its input, on
    # encoded payloads; the groups equal the oracle's
    import paper_1702_07409_amd as fs
    g, G = graphs(k=500, n=1000, dist="raptor")
    ch = fs.fs_checks_generate(g)
    c2, c3 = ch.export()
    assert ch.n_check3 == 500 and ch.n_check2 == 500
    x = gen.payload(0, 13, 500, 32)
    c = codec.encode(G, x)
    for grp in c3:
        assert not np.bitwise_xor.reduce(c[grp], axis=0).any()
    for i, members in c2.items():
        assert np.array_equal(np.bitwise_xor.reduce(c[members], axis=0), x[i])
    b, L, _ = checks.cga(G)
    assert (c2, c3) == checks.split(b, L)


def local_case(g, G, ch, c3, lost, er, t, seed=0):
    import paper_1702_07409_amd as fs
    x = gen.payload(1, seed, G.k, t)
    c_host = codec.encode(G, x)
    want, ok, _, _, levels = checks.local_repair(c3, c_host, lost, er)
    c = dev(c_host)
    c[dev(np.array(lost, np.int64))] = 0x6D
    rep, st = empty_u8(max(len(lost), 1)), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_REPAIR_LOCAL, t, len(lost))
    fs.fs_repair_local(g, ch, c, dev(er) if er is not None else None, dev(np.array(lost, np.uint32)), len(lost),
                       rep, st, t, ws)
    got = host(c)
    assert np.array_equal(host(rep)[:len(lost)], ok)
    assert np.array_equal(got[lost], want)
    others = [j for j in range(G.n) if j not in set(lost)]
    assert np.array_equal(got[others], c_host[others])
    assert host(st).tolist() == [int(ok.all()), int(len(lost) - ok.sum()), levels]
    return ok, levels


def test_local_repair_random_losses():
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    ch = fs.fs_checks_generate(g)
    _, c3 = ch.export()
    rng = np.random.default_rng(7)
    some = 0
    for trial in range(12):
        lost = sorted(rng.choice(400, size=int(rng.integers(1, 9)), replace=False).tolist())
        er = (rng.random(400) < 0.05).astype(np.uint8)
        er[lost] = 0
        ok, _ = local_case(g, G, ch, c3, lost, er if trial % 2 else None, 512 * 3 + 16, trial)
        some += int(ok.sum())
    assert some > 0


@pytest.mark.parametrize("disk", [0, 3])
def test_local_repair_of_a_whole_disk_takes_several_levels(disk):
    # a tenth of the rows lost at once: blocks rebuilt at one level complete
    # the groups of others at the next
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    ch = fs.fs_checks_generate(g)
    _, c3 = ch.export()
    lost = list(range(disk * 40, disk * 40 + 40))
    ok, levels = local_case(g, G, ch, c3, lost, None, 256 + 48, disk)
    assert levels >= 2 and ok.sum() > 0


@pytest.mark.parametrize("t", [304, 32768, 65536])
def test_local_repair_of_a_long_chain(t):
    # groups {i, i+1} with blocks 0..39 lost: one block per level, 40 levels
    # and the level of blocks no group rebuilds.  Short blocks run the first
    # levels as launches of their own and the rest as a slice walk; 64 KiB
    # blocks take the slice walk throughout.
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    arr = []
    for i in range(40):
        arr += [0, 2, i, i + 1]
    ch = fs.fs_checks_load(g, arr)
    _, c3 = ch.export()
    assert c3 == [[i, i + 1] for i in range(40)]
    ok, levels = local_case(g, G, ch, c3, list(range(40)), None, t, 5)
    assert levels == 40 and ok.all()
    # a block of the chain that stays unknown: the blocks below it are not rebuilt
    er = np.zeros(400, np.uint8)
    er[25] = 1
    ok, levels = local_case(g, G, ch, c3, [i for i in range(40) if i != 25], er, t, 6)
    assert levels == 14 and ok.sum() == 14


def test_local_repair_with_group_counters_in_global_memory():
    # 20000 groups: 8 bytes each no longer fit LDS beside the two bitsets, so
    # the level loop lowers the counters in the workspace
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=25000, dist="raptor")
    arr = []
    for i in range(20000):
        arr += [0, 2, i, i + 1]
    ch = fs.fs_checks_load(g, arr)
    _, c3 = ch.export()
    assert len(c3) == 20000
    ok, levels = local_case(g, G, ch, c3, list(range(40)), None, 304, 7)
    assert levels == 40 and ok.all()


@pytest.mark.parametrize("lost", [[0], [0, 1], [1, 0, 7]])
def test_local_repair_of_a_block_in_many_groups(lost):
    # block 0 sits in 300 groups {0, j}: removing it from them takes the
    # lanes of a wave several passes; with block 1 lost too, group {0, 1}
    # waits a level for block 0
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    arr = []
    for j in range(1, 301):
        arr += [0, 2, 0, j]
    ch = fs.fs_checks_load(g, arr)
    _, c3 = ch.export()
    ok, levels = local_case(g, G, ch, c3, lost, None, 304, 8)
    assert ok.all() and levels == (1 if lost == [0] else 2)


def test_local_repair_nothing_lost():
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    ch = fs.fs_checks_generate(g)
    _, c3 = ch.export()
    local_case(g, G, ch, c3, [], None, 64)


def test_local_repair_rejects_bad_ids_without_writing():
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    ch = fs.fs_checks_generate(g)
    x = gen.payload(1, 2, 200, 64)
    c_host = codec.encode(G, x)
    for lost in ([3, 400], [5, 9, 5]):
        c = dev(c_host)
        rep, st = empty_u8(len(lost)), empty_i32(3)
        ws = fs.workspace(g, fs.FS_OP_REPAIR_LOCAL, 64, len(lost))
        fs.fs_repair_local(g, ch, c, None, dev(np.array(lost, np.uint32)), len(lost), rep, st, 64, ws)
        assert np.array_equal(host(c), c_host)
        assert host(st).tolist() == [0, len(lost), -fs._lib.FS_ERR_INVALID] and not host(rep).any()


@pytest.mark.parametrize("k,n,dist", [(64, 96, "rsd"), (200, 400, "raptor")])
def test_check_data_equals_the_oracle_and_loads_back(k, n, dist):
    # the library's check data array equals the oracle's (§2.7 records), and
    # loading it back gives the same equations
    import paper_1702_07409_amd as fs
    g, G = graphs(k=k, n=n, dist=dist)
    ch = fs.fs_checks_generate(g)
    arr = ch.serialize()
    want2, want3 = checks.split(*checks.cga(G)[:2])
    assert arr.tolist() == checks.check_data(want2, want3)
    back = fs.fs_checks_load(g, arr)
    assert back.export() == (want2, want3)
    assert back.serialize().tolist() == arr.tolist()


def test_check_data_of_the_paper_example_loads():
    # §2.7's example array on a code with at least 89 coded and 20 data blocks
    import json
    import os
    import paper_1702_07409_amd as fs
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_check_data.json")) as fh:
        ex = json.load(fh)
    g, G = graphs(k=64, n=96)
    ch = fs.fs_checks_load(g, ex["array"])
    assert ch.export() == checks.from_check_data(ex["array"])
    assert ch.n_check2 == 1 and ch.n_check3 == 2


def test_local_repair_with_loaded_checks_equals_generated():
    import paper_1702_07409_amd as fs
    g, G = graphs(k=200, n=400, dist="raptor")
    ch = fs.fs_checks_generate(g)
    loaded = fs.fs_checks_load(g, ch.serialize())
    _, c3 = ch.export()
    rng = np.random.default_rng(21)
    for trial in range(3):
        lost = sorted(rng.choice(400, size=30, replace=False).tolist())
        for which in (ch, loaded):
            local_case(g, G, which, c3, lost, None, 256 + 32, trial)


@pytest.mark.parametrize("arr", [[2, 1, 5], [0, 3, 1, 2], [1, 4, 2, 7], [1, 64, 1, 0], [0, 1, 96], [0, -1]])
def test_check_data_load_rejects_malformed_arrays(arr):
    # unknown flag, records past the end, input >= k, coded block >= n, a negative size
    import paper_1702_07409_amd as fs
    g, _ = graphs(k=64, n=96)
    with pytest.raises(fs.FsError):
        fs.fs_checks_load(g, arr)


@pytest.mark.parametrize("with_precode", [False, True])
def test_added_groups_equal_the_oracle(with_precode):
    # §2.5's extra check #3 groups (degree-one blocks; check #1 sets combined
    # through check #2, Eqs. (1)-(4)) equal the oracle's, in order, and serve
    # the local repair
    import paper_1702_07409_amd as fs
    from oracle import precode
    b, k, n = 85, 100, 170
    g, G = graphs(k=k, n=n, dist="raptor", seed=3)
    ch = fs.fs_checks_generate(g)
    pc = fs.fs_precode_build(b, k) if with_precode else None
    added = ch.add_groups(g, pc)
    check2, check3 = checks.split(*checks.cga(G)[:2])
    extra = checks.extra_groups(G, check2, precode.checks(b, k) if with_precode else None)
    want = checks.with_extra_groups(check3, extra)
    got2, got3 = ch.export()
    assert got2 == check2 and got3 == want
    assert added == len(want) - len(check3) and (added > 0 or not with_precode)
    rng = np.random.default_rng(5)
    for trial in range(3):
        lost = sorted(rng.choice(n, size=25, replace=False).tolist())
        local_case(g, G, ch, want, lost, None, 128 + 16, trial)


def test_added_groups_reject_a_precode_of_another_size():
    import paper_1702_07409_amd as fs
    g, _ = graphs(k=100, n=170, dist="raptor", seed=3)
    ch = fs.fs_checks_generate(g)
    before = ch.export()
    with pytest.raises(fs.FsError):
        ch.add_groups(g, fs.fs_precode_build(75, 90))
    assert ch.export() == before
