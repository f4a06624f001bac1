"""The GPU payload generator writes the same bytes as the numpy one."""

import numpy as np
import pytest

from synth import gen

pytestmark = pytest.mark.gpu


def test_gpu_fill_matches_numpy():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth.gpu as sg
    for seed, stripe, k, t, purpose in [(0, 0, 64, 4096, sg.DATA), (3, 17, 9, 4096 + 48, sg.DATA),
                                        (6, 5, 4, 65536, sg.UPDATE_DATA)]:
        x = torch.empty((k, t), dtype=torch.uint8, device="cuda")
        sg.fill(x, seed, stripe, t, purpose=purpose)
        want = gen.payload_slice(seed, stripe, range(k), 0, t, purpose=purpose)
        assert np.array_equal(x.cpu().numpy(), want)
    # a block range starting past 0
    x = torch.empty((3, 1024), dtype=torch.uint8, device="cuda")
    sg.fill(x, 1, 2, 1024, first_block=40)
    assert np.array_equal(x.cpu().numpy(), gen.payload_slice(1, 2, [40, 41, 42], 0, 1024))
