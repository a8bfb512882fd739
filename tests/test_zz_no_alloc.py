"""nncp_fit_noalloc (static device scratch, no allocation) against nncp_fit (caller
workspace) through the C ABI: the same kernels on the same inputs, so factors and residuals
must agree bit for bit.  Two calls in a row, the second with a smaller core and rank, so the
static scratch holds the first call's contents when the second starts."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, need_gpu

pytestmark = pytest.mark.gpu


def _fit_both(nnc, core_dims, rank, iters, seed):
    G = dev(synth.uniform(seed, synth.STREAM_CORE0, int(np.prod(core_dims))).reshape(core_dims))
    B0 = synth.init_cp_factors(seed, core_dims, rank)
    Bw = [dev(b) for b in B0]
    Bs = [dev(b) for b in B0]
    rw = nnc.nncp_fit(G, rank, iters, Bw)
    rs = nnc.nncp_fit_noalloc(G, rank, iters, Bs)
    return rw, rs, [host(b) for b in Bw], [host(b) for b in Bs]


@pytest.mark.parametrize("first,second", [
    (((20, 20, 20), 10, 60), ((12, 9, 7), 4, 40)),
    (((16, 12, 10, 8), 16, 30), ((6, 5, 4), 3, 25)),
])
def test_noalloc_matches_workspace_two_calls(first, second):
    nnc = need_gpu()
    for seed, (dims, rank, iters) in enumerate((first, second), start=71):
        rw, rs, Bw, Bs = _fit_both(nnc, dims, rank, iters, seed)
        print("case", dims, rank, iters, rw, rs, flush=True)
        assert rw == rs, (dims, rw, rs)
        for a, b in zip(Bw, Bs):
            assert np.array_equal(a, b), dims


def test_noalloc_refuses_scratch_above_maximum():
    nnc = need_gpu()
    import ctypes
    # a 64 x 64 x 64 x 16 core at rank 32 needs 8 MiB of contraction scratch plus the tables
    shape = (64, 64, 64, 16)
    dims = (ctypes.c_int64 * 4)(*shape)
    need = nnc.lib().nncp_workspace_bytes(4, dims, 32)
    assert need > nnc.lib().nncp_noalloc_max_scratch_bytes()
    G = dev(np.ones(shape, dtype=np.float32))
    B = [dev(np.ones((m, 32), dtype=np.float32)) for m in shape]
    with pytest.raises(nnc.NncError) as e:
        nnc.nncp_fit_noalloc(G, 32, 1, B)
    assert e.value.status == nnc.NNC_EUNSUPPORTED
