"""GPU parity of the code extension (fs_extend): the new coded rows equal the
oracle's, bit for bit, and the existing rows are left as they were.

Run on an MI355X: pytest -m gpu.
"""

from dataclasses import replace

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


def extend_case(sp, n_old, from_inputs, n_erased=0, fill=0x5A):
    """Run fs_extend on the code of sp (sp.n rows) grown from n_old rows and
    compare with the oracle.  Returns (made, status) as host arrays."""
    import paper_1702_07409_amd as fs
    g, G = graphs(**sp.graph_kwargs())
    x = sp.x()
    c_full = codec.encode(G, x)
    er = gen.erasure_mask(sp.erase_seed, sp.stripe, n_old, n_erased) if n_old else np.zeros(0, np.uint8)
    if from_inputs:
        want, ok = codec.extend(G, n_old, x=x)
    else:
        want, ok = codec.extend(G, n_old, c_old=c_full[:n_old], erased=er)
    c = dev(c_full)
    c[n_old:] = fill
    # erased old rows hold garbage: the extension must not read them
    er_ids = np.flatnonzero(er)
    if len(er_ids):
        c[dev(er_ids.astype(np.int64))] = 0xC3
    made, st = empty_u8(max(sp.n - n_old, 1)), empty_i32(3)
    op = fs.FS_OP_EXTEND if from_inputs else fs.FS_OP_EXTEND_CONVENTIONAL
    ws = fs.workspace(g, op, sp.t)
    fs.fs_extend(g, n_old, dev(x) if from_inputs else None, c, dev(er) if len(er) else None, made, st,
                 sp.t, ws)
    got = host(c)
    old = c_full[:n_old].copy()
    old[er_ids] = 0xC3
    assert np.array_equal(got[:n_old], old)
    assert np.array_equal(got[n_old:], want)
    made_h = host(made)[:sp.n - n_old]
    assert np.array_equal(made_h, ok)
    st_h = host(st).tolist()
    assert st_h == [int(ok.all()), int(len(ok) - ok.sum()), 0]
    return made_h, st_h


SMALL = workloads.StripeSpec(stripe=4, k=150, n=320, t=512 * 3 + 16, dist="rsd", stripe_key=5)


@pytest.mark.parametrize("from_inputs", [True, False])
@pytest.mark.parametrize("n_erased", [0, 30])
def test_extend_small(from_inputs, n_erased):
    made, _ = extend_case(SMALL, 260, from_inputs, n_erased)
    if not from_inputs and n_erased:
        assert 0 < made.sum() < len(made)


def test_extend_degenerate_sizes():
    # nothing to add; nothing existing (every new row is then unknown);
    # a single new row
    for n_old, from_inputs in ((SMALL.n, True), (SMALL.n, False), (0, True), (0, False),
                               (SMALL.n - 1, False)):
        made, st = extend_case(SMALL, n_old, from_inputs)
        if n_old == 0 and not from_inputs:
            assert not made.any()


def test_extend_rejects_more_old_rows_than_the_graph():
    import paper_1702_07409_amd as fs
    g, _ = graphs(**SMALL.graph_kwargs())
    made, st = empty_u8(1), empty_i32(3)
    c = empty_u8(SMALL.n, SMALL.t)
    ws = fs.workspace(g, fs.FS_OP_EXTEND_CONVENTIONAL, SMALL.t)
    with pytest.raises(fs.FsError):
        fs.fs_extend(g, SMALL.n + 1, None, c, None, made, st, SMALL.t, ws)


def test_extend_ragged_finite_graph():
    sp = workloads.StripeSpec(stripe=7, k=700, n=900, t=256 * 5 + 48, dist="finite",
                              finite_w=workloads.finite16_weights())
    extend_case(sp, gen.overhead_n(700, 0.10), True)
    extend_case(sp, gen.overhead_n(700, 0.10), False, 20)


def test_extend_large_stripe_full_size():
    # the large stripe (k = 4096, 64 KiB blocks, n = 1.1 k) grown to 1.2 k rows
    # from its own blocks with 5 % of them erased
    base = workloads.large_stripe()
    sp = replace(base, n=gen.overhead_n(4096, 0.20))
    made, st = extend_case(sp, base.n, False, base.n_erased)
    assert made.sum() > 0


@pytest.mark.parametrize("n_erased", [0, 12])
def test_extend_through_local_groups(n_erased):
    # §2.9: the new rows of a code grown from 360 to 400 rows, made from the
    # existing rows through the longer code's check #3 groups; the same rows,
    # made flags and status as the oracle, old rows untouched
    import paper_1702_07409_amd as fs
    from oracle import checks
    g, G = graphs(k=200, n=400, dist="raptor", seed=2)
    ch = fs.fs_checks_generate(g)
    _, c3 = ch.export()
    t, n_old = 1024 + 16, 360
    x = gen.payload(4, 0, 200, t)
    c_full = codec.encode(G, x)
    er = gen.erasure_mask(2, 0, n_old, n_erased) if n_erased else None
    rows, made_w, levels = checks.extend_local(c3, c_full[:n_old], 400, er)
    c = dev(c_full)
    c[n_old:] = 0x5A
    old = c_full[:n_old].copy()
    if er is not None:
        # unavailable old rows hold garbage: the extension must not read them
        ids = np.flatnonzero(er)
        c[dev(ids.astype(np.int64))] = 0xC3
        old[ids] = 0xC3
    made, st = empty_u8(40), empty_i32(3)
    ws = fs.workspace(g, fs.FS_OP_EXTEND_LOCAL, t, 40)
    fs.fs_extend_local(g, ch, n_old, c, dev(er) if er is not None else None, made, st, t, ws)
    got = host(c)
    assert np.array_equal(got[:n_old], old)
    assert np.array_equal(host(made), made_w)
    assert np.array_equal(got[n_old:][made_w == 1], rows[made_w == 1])
    assert np.array_equal(got[n_old:][made_w == 1], c_full[n_old:][made_w == 1])
    assert host(st).tolist() == [int(made_w.all()), int(40 - made_w.sum()), levels]
    assert made_w.sum() > 0
