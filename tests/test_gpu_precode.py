"""GPU parity of the array-LDPC precode: the parity encode and the two-stage
decode equal the oracle's, bit for bit.

Run on an MI355X: pytest -m gpu.
"""

import numpy as np
import pytest

from gpu_util import dev, empty_i32, empty_u8, graphs, host
from oracle import codec, precode, simdisk
from synth import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_precode_encode(pc, data, t):
    import paper_1702_07409_amd as fs
    x = empty_u8(pc.k, t)
    x.fill_(0x3C)
    x[:pc.b] = dev(data)
    fs.fs_precode_encode(pc, x, t)
    return x


@pytest.mark.parametrize("b,k,t", [(925, 1036, 1024), (28, 49, 512 * 3 + 16), (9919, 10246, 512), (10, 15, 16)])
def test_precode_encode(b, k, t):
    import paper_1702_07409_amd as fs
    pc = fs.fs_precode_build(b, k)
    data = gen.payload(0, 11, b, t)
    assert np.array_equal(host(gpu_precode_encode(pc, data, t)), precode.encode(b, k, data))


def oracle_two_stage(G, b, c, er):
    """All k blocks, the known mask and the status, as decode_two_stage
    computes them."""
    x, rec, st, _ = codec.decode(G, c, er)
    known = rec.astype(bool)
    L2 = 0
    if not known[:b].all():
        x, known, L2 = precode.precode_bp(b, G.k, x, known)
        x[~known] = 0
    ok = known[:b]
    return x, known, [int(ok.all()), int(b - ok.sum()), int(st[2]), int(L2)]


def two_stage_case(b, k, n, t, er_fn, dist="raptor", seed=3):
    import paper_1702_07409_amd as fs
    g, G = graphs(k=k, n=n, dist=dist, seed=seed)
    pc = fs.fs_precode_build(b, k)
    data = gen.payload(0, 12, b, t)
    xfull = precode.encode(b, k, data)
    c = codec.encode(G, xfull)
    er = er_fn(G)
    want_x, want_known, want_st = oracle_two_stage(G, b, c, er)
    x = empty_u8(k, t)
    x.fill_(0xA5)
    rec, st = empty_u8(k), empty_i32(4)
    ws = fs.workspace(g, fs.FS_OP_DECODE_PRECODED, t)
    fs.fs_decode_precoded(g, pc, dev(c), dev(er), 0, x, rec, st, t, ws)
    got = host(x)
    assert host(st).tolist() == want_st
    assert np.array_equal(host(rec).astype(bool), want_known)
    assert np.array_equal(got, want_x)
    okb = want_known[:b]
    assert np.array_equal(got[:b][okb], data[okb])
    return want_st


def test_precode_recovers_blocks_the_ldgm_pass_cannot():
    def er_fn(G):
        er = np.zeros(G.n, np.uint8)
        for i in (5, 400, 900):
            er[G.NT(i)] = 1
        return er
    st = two_stage_case(925, 1036, 1500, 1024, er_fn)
    assert st[0] == 1 and st[3] >= 1


def test_no_erasures_skips_the_second_pass():
    st = two_stage_case(925, 1036, 2180, 512, lambda G: np.zeros(G.n, np.uint8))
    assert st[0] == 1 and st[3] == 0


@pytest.mark.parametrize("failed", [(0, 1), (2, 5, 7), (1, 3, 6, 8), (0, 1, 2, 3, 4, 5)])
def test_paper_table2_codes_with_failed_disks(failed):
    # the smaller code of the paper's measurements: k = 1036 over n = 2180
    # coded blocks on 10 disks, 2-4 disks lost (and 6, where decoding fails)
    two_stage_case(925, 1036, 2180, 512, lambda G: simdisk.erased_mask(G.n, 10, failed))


def test_large_code_three_disks_lost():
    # the larger code (k = 10246, n = 21800, t = 512), 3 of 10 disks lost
    st = two_stage_case(9919, 10246, 21800, 512, lambda G: simdisk.erased_mask(G.n, 10, (1, 4, 8)))
    assert st[1] < 50


def test_random_erasures_small_code():
    rng = np.random.default_rng(5)
    for trial in range(6):
        frac = rng.uniform(0.1, 0.5)
        two_stage_case(28, 49, 70, 48, lambda G: (rng.random(G.n) < frac).astype(np.uint8), dist="rsd",
                       seed=trial + 1)


def test_precode_arguments_are_checked():
    import paper_1702_07409_amd as fs
    g, _ = graphs(k=1036, n=1200, dist="raptor")
    pc = fs.fs_precode_build(28, 49)
    ws = fs.workspace(g, fs.FS_OP_DECODE_PRECODED, 16)
    with pytest.raises(fs.FsError):
        fs.fs_decode_precoded(g, pc, empty_u8(1200, 16), empty_u8(1200), 0, empty_u8(1036, 16), empty_u8(1036),
                              empty_i32(4), 16, ws)
    hpc = fs.fs_precode_build(28, 49, host_only=True)
    with pytest.raises(fs.FsError):
        fs.fs_precode_encode(hpc, empty_u8(49, 16), 16)


@pytest.mark.parametrize("disks,erase", [(2, False), (3, False), (3, True), (6, False)])
def test_precoded_repair_equals_the_oracle(disks, erase):
    # the conventional repair of Table 2's smaller code: two-stage decode,
    # parity encoded again when the data is complete, lost rows re-encoded;
    # with six of ten disks lost the data stays incomplete
    import paper_1702_07409_amd as fs
    b, k, n, t = 925, 1036, 2180, 256 + 48
    g, G = graphs(k=k, n=n, dist="raptor", seed=1)
    pc = fs.fs_precode_build(b, k)
    x = precode.encode(b, k, gen.payload(0, 7, b, t))
    c_host = codec.encode(G, x)
    # disks 0 .. disks-1 lost, or with disk 0 erased the next ones
    first = n // 10 if erase else 0
    lost = list(range(first, first + disks * n // 10))
    er = np.zeros(n, np.uint8)
    if erase:
        er[:n // 10] = 1
    want, ok = precode.repair_two_stage(G, b, c_host, er, lost)
    c = dev(c_host)
    c[dev(np.array(lost, np.int64))] = 0x5A
    rep, st = empty_u8(len(lost)), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_REPAIR_PRECODED, t, len(lost))
    fs.fs_repair_precoded(g, pc, c, dev(er), dev(np.array(lost, np.uint32)), len(lost), rep, st, t, ws)
    got = host(c)
    assert np.array_equal(host(rep), ok)
    assert np.array_equal(got[lost], want)
    others = [j for j in range(n) if j not in set(lost)]
    assert np.array_equal(got[others], c_host[others])
    assert host(st).tolist()[:2] == [int(ok.all()), int(len(lost) - ok.sum())]
    if disks == 3 and not erase:
        _, ok1 = codec.repair_conventional(G, c_host, er, lost)
        assert ok.all() and ok1.sum() < ok.sum()


def test_precoded_repair_rejects_bad_ids_without_writing():
    import paper_1702_07409_amd as fs
    b, k, n, t = 925, 1036, 2180, 64
    g, G = graphs(k=k, n=n, dist="raptor", seed=1)
    pc = fs.fs_precode_build(b, k)
    c_host = codec.encode(G, precode.encode(b, k, gen.payload(0, 8, b, t)))
    for lost in ([3, n], [5, 9, 5]):
        c = dev(c_host)
        rep, st = empty_u8(len(lost)), empty_i32(3)
        ws = fs.workspace(g, fs.FS_OP_REPAIR_PRECODED, t, len(lost))
        fs.fs_repair_precoded(g, pc, c, None, dev(np.array(lost, np.uint32)), len(lost), rep, st, t, ws)
        assert np.array_equal(host(c), c_host) and not host(rep).any()
        assert host(st).tolist()[:2] == [0, len(lost)]
