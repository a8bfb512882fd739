"""nnc_fill_uniform / nnc_fill_uniform_f64 against the host generator synth.uniform: the same
counter-based SplitMix64 stream, so every value must match bit for bit (FP32 values are the
round-to-nearest-even of the same doubles)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

CASES = [(0, 0, 1), (1, 48, 1000), (2, 64, 65536 + 7), (5, 32, 1000003), (2**63 + 12345, 1024 + 16 * 63 + 4, 4097),
         (7, (1 << 24) + 5, 333)]


@pytest.mark.parametrize("seed,stream,n", CASES)
def test_fill_uniform_f32_bit_exact(seed, stream, n):
    nnc = need_gpu()
    got = nnc.nnc_fill_uniform(seed, stream, n).cpu().numpy()
    ref = synth.uniform(seed, stream, n).astype(np.float32)
    assert got.dtype == np.float32 and got.shape == (n,)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (seed, stream, n)


@pytest.mark.parametrize("seed,stream,n", CASES)
@pytest.mark.parametrize("offset", [0, 1, 123456789])
def test_fill_uniform_f64_bit_exact(seed, stream, n, offset):
    nnc = need_gpu()
    got = nnc.nnc_fill_uniform_f64(seed, stream, n, offset=offset).cpu().numpy()
    ref = synth.uniform(seed, stream, n, offset)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (seed, stream, n, offset)


def test_fill_uniform_empty_and_slices_compose():
    nnc = need_gpu()
    import torch
    assert nnc.nnc_fill_uniform(3, 4, 0).numel() == 0
    whole = nnc.nnc_fill_uniform_f64(3, 4, 10000)
    parts = torch.cat([nnc.nnc_fill_uniform_f64(3, 4, 3333, offset=0),
                       nnc.nnc_fill_uniform_f64(3, 4, 6667, offset=3333)])
    assert torch.equal(whole, parts)
