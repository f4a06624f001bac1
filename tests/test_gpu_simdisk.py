"""GPU parity of the disk-failure sweep (fs_sim_disks): every combination's
status triple equals the oracle's, element by element.

Run on an MI355X: pytest -m gpu.
"""

import math

import numpy as np
import pytest

from gpu_util import empty_i32, graphs, host
from oracle import simdisk
from synth import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_sweep(g, s, f, first=0, count=None, maxit=0):
    import paper_1702_07409_amd as fs
    count = math.comb(s, f) - first if count is None else count
    res = empty_i32(max(count, 1), 3)
    res.fill_(-7)
    ws = fs.workspace(g, fs.FS_OP_SIM_DISKS)
    fs.fs_sim_disks(g, s, f, first, count, maxit, res, ws)
    return host(res)[:count]


def check_sweep(kw, s, fs_, maxit=0):
    g, G = graphs(**kw)
    for f in fs_:
        got = gpu_sweep(g, s, f, maxit=maxit)
        want = simdisk.sim_disks(G, s, f, maxit=maxit)
        assert np.array_equal(got, want), (kw, s, f, np.flatnonzero((got != want).any(axis=1))[:5])
    return g, G


def test_sweep_paper_code_ten_disks():
    # the smaller code of the paper's measurements (k = 1036, n = 2180, 10 disks)
    # with the finite (Raptor) degree table: every combination of 0..4 failures
    check_sweep(dict(k=1036, n=2180, dist="raptor"), 10, range(0, 5))


def test_sweep_every_failure_count_small():
    # index-sum state (small degrees), disks of unequal size (97 rows on 7 disks)
    check_sweep(dict(k=64, n=97, dist="rsd", seed=3), 7, range(0, 8))


def test_sweep_heavy_rows_use_the_index_xor_state():
    # Robust Soliton rows of degree > 255 rule out the packed index sum
    kw = dict(k=3000, n=3600, dist="rsd", rsd_c=0.1, rsd_delta=0.05, seed=2)
    g, G = graphs(**kw)
    assert G.degrees().max() > 255
    check_sweep(kw, 12, (1, 2))


def test_sweep_beyond_lds_uses_workgroup_slots():
    # 6 n bytes of per-row state exceed one workgroup's LDS at n = 28000
    kw = dict(k=22000, n=28000, dist="finite", finite_w=workloads.finite16_weights())
    check_sweep(kw, 20, (0, 1))


def test_sweep_sub_ranges_and_level_limit():
    kw = dict(k=1036, n=2180, dist="raptor")
    g, G = graphs(**kw)
    full = gpu_sweep(g, 10, 3)
    for first, count in ((0, 1), (17, 40), (119, 1), (60, 60)):
        assert np.array_equal(gpu_sweep(g, 10, 3, first, count), full[first:first + count])
    for maxit in (1, 5):
        assert np.array_equal(gpu_sweep(g, 10, 3, maxit=maxit), simdisk.sim_disks(G, 10, 3, maxit=maxit))


def test_sweep_one_row_per_disk_and_one_disk():
    # s = n: every disk is a single coded row; s = 1: all or nothing
    kw = dict(k=20, n=30, dist="rsd", seed=4)
    check_sweep(kw, 30, (0, 1, 2, 28, 29, 30))
    check_sweep(kw, 1, (0, 1))


def test_sweep_rejects_bad_arguments():
    import paper_1702_07409_amd as fs
    g, _ = graphs(k=64, n=96, dist="rsd")
    res = empty_i32(8, 3)
    ws = fs.workspace(g, fs.FS_OP_SIM_DISKS)
    for s, f, first, count in ((0, 0, 0, 1), (65, 1, 0, 1), (97, 1, 0, 1), (10, 11, 0, 1),
                               (10, 2, 40, 6), (10, 2, 46, 0)):
        with pytest.raises(fs.FsError):
            fs.fs_sim_disks(g, s, f, first, count, 0, res, ws)
    fs.fs_sim_disks(g, 10, 2, 45, 0, 0, res, ws)   # an empty range at the end is fine


def test_sweep_large_code_sampled():
    # the larger code of the paper's measurements (k = 10246, n = 21800) on 24
    # disks, 4 failed: sampled ranks against the oracle, and the tolerable
    # fraction is between 0 and 1
    kw = dict(k=10246, n=21800, dist="raptor")
    g, G = graphs(**kw)
    s, f = 24, 4
    total = math.comb(s, f)
    got = gpu_sweep(g, s, f)
    assert got.shape == (total, 3) and (got[:, 1] >= 0).all()
    assert ((got[:, 0] == 1) == (got[:, 1] == 0)).all()
    for r in (0, 1, total // 3, total // 2, total - 2, total - 1):
        assert np.array_equal(got[r], simdisk.sim_disks(G, s, f, first=r, count=1)[0]), r


def gpu_sweep_precoded(g, pc, s, f, first=0, count=None, maxit=0):
    import paper_1702_07409_amd as fs
    count = math.comb(s, f) - first if count is None else count
    res = empty_i32(max(count, 1), 4)
    res.fill_(-7)
    ws = fs.workspace(g, fs.FS_OP_SIM_DISKS, 16, pc.k - pc.b)
    fs.fs_sim_disks_precoded(g, pc, s, f, first, count, maxit, res, ws)
    return host(res)[:count]


@pytest.mark.parametrize("b,k,n,dist,s,fs_", [(925, 1036, 2180, "raptor", 10, (0, 2, 3, 4, 5)),
                                             (28, 49, 84, "rsd", 7, range(0, 8))])
def test_precoded_sweep(b, k, n, dist, s, fs_):
    import paper_1702_07409_amd as fs
    g, G = graphs(k=k, n=n, dist=dist)
    pc = fs.fs_precode_build(b, k)
    for f in fs_:
        got = gpu_sweep_precoded(g, pc, s, f)
        want = simdisk.sim_disks_precoded(G, b, s, f)
        assert np.array_equal(got, want), (s, f, np.flatnonzero((got != want).any(axis=1))[:5])


def test_precoded_sweep_large_code_sampled_and_slots():
    # the k = 10246 code on 24 disks: sampled ranks; and a code whose state
    # lives in workgroup slots (3 bytes a row for n = 56000 exceed LDS)
    import paper_1702_07409_amd as fs
    for b, k, n, s, f in ((9919, 10246, 21800, 24, 4), (21854, 22523, 56000, 20, 1)):
        g, G = graphs(k=k, n=n, dist="raptor")
        pc = fs.fs_precode_build(b, k)
        total = math.comb(s, f)
        got = gpu_sweep_precoded(g, pc, s, f)
        assert got.shape == (total, 4)
        for r in sorted({0, 1, total // 2, total - 1}):
            assert np.array_equal(got[r], simdisk.sim_disks_precoded(G, b, s, f, first=r, count=1)[0]), r
