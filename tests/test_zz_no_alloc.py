"""fs_decode_noalloc (the decode with its workspace in the library's fixed
device array) gives what fs_decode with a caller workspace gives, on two
calls in a row, the second on a smaller stripe, so the second runs over what
the first left in the array; and it refuses a graph whose decode needs more
than the array holds."""

import numpy as np
import pytest

from gpu_util import dev, empty_i32, empty_u8, graphs, host
from oracle import codec
from synth import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _both(sp):
    import paper_1702_07409_amd as fs
    g, G = graphs(**sp.graph_kwargs())
    x = sp.x()
    c_host = codec.encode(G, x)
    c, er = dev(c_host), dev(sp.erased_mask())
    outs = []
    for noalloc in (False, True):
        xo = empty_u8(sp.k, sp.t)
        xo.fill_(0x5A if noalloc else 0xA5)
        rec, st = empty_u8(sp.k), empty_i32(3)
        rec.fill_(7)
        st.fill_(-9)
        if noalloc:
            fs.fs_decode_noalloc(g, c, er, 0, xo, rec, st, sp.t)
        else:
            ws = fs.workspace(g, fs.FS_OP_DECODE, sp.t)
            fs.fs_decode(g, c, er, 0, xo, rec, st, sp.t, ws)
        outs.append((host(xo), host(rec), host(st)))
    (xa, ra, sa), (xb, rb, sb) = outs
    assert np.array_equal(xa, xb) and np.array_equal(ra, rb) and sa.tolist() == sb.tolist()
    xw, recw, stw, _ = codec.decode(G, c_host, sp.erased_mask())
    assert np.array_equal(xb, xw) and np.array_equal(rb, recw) and sb.tolist() == list(stw)
    return sb


def test_noalloc_decode_equals_decode_twice_second_smaller():
    big = workloads.scaled(workloads.large_stripe(), 4096)       # k = 4096, n = 4506, 225 erased
    small = workloads.tiny()                                      # k = 64, n = 96, 16 erased
    print("noalloc decode: k=%d n=%d t=%d" % (big.k, big.n, big.t), flush=True)
    s1 = _both(big)
    print("noalloc decode: k=%d n=%d t=%d" % (small.k, small.n, small.t), flush=True)
    s2 = _both(small)
    assert s1[2] > 0 and s2[2] > 0


def test_noalloc_decode_rejects_a_graph_above_the_limit():
    import paper_1702_07409_amd as fs
    g = fs.fs_graph_build(k=400000, n=420000, dist="rsd")
    assert fs.fs_workspace_size(g, fs.FS_OP_DECODE, 16, 0) > 16 << 20
    c, x = empty_u8(420000, 16), empty_u8(400000, 16)
    er, rec, st = empty_u8(420000), empty_u8(400000), empty_i32(3)
    st.fill_(-9)
    with pytest.raises(fs.FsError) as e:
        fs.fs_decode_noalloc(g, c, er, 0, x, rec, st, 16)
    assert "16777216" in str(e.value)
    assert host(st).tolist() == [-9, -9, -9]
