"""X passes over modes longer than the factor the matrix-core kernels can hold in LDS.

The contracted index is then split into chunks, each a launch on its slab of X whose output
is added to the earlier chunks' in chunk order (eq. nnCANDELINC allows any N_i).  Every case
asserts through nnc_last_ttm_kernel that a matrix-core pass ran (never the general kernel)
and checks the result against the FP64 oracle, per output fibre as well as in total."""
import zlib

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import bf16_dev, dev, host, need_gpu, problem, rel_fro

pytestmark = pytest.mark.gpu


def _fibre_err(out, ref, n):
    """Largest relative error over the mode-n fibres of the output (a wrong chunk or tile
    shows up even when the total is close)."""
    o = np.moveaxis(out, n, -1).reshape(-1, out.shape[n])
    r = np.moveaxis(ref, n, -1).reshape(-1, ref.shape[n])
    return float((np.linalg.norm(o - r, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-30)).max())


CASES = [((1024, 512, 512), 0, 20), ((512, 512, 1024), 2, 20), ((64, 1024, 256), 1, 20),
         ((256, 256, 256), 0, 32), ((256, 256, 256), 2, 32), ((800, 64, 800), 0, 20), ((800, 64, 800), 2, 20),
         # earlier-mode bf16 pass with its output staged by halves of the tile (R above 20)
         ((512, 512, 512), 0, 24), ((512, 384, 512), 1, 32)]


@pytest.mark.parametrize("shape,mode,R", CASES)
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_long_mode_pass_matches_oracle(shape, mode, R, dt):
    nnc = need_gpu()
    rng = np.random.default_rng(zlib.crc32(repr((shape, mode, R, dt)).encode()))
    X64 = rng.random(shape)
    if dt == "bf16":
        X64 = synth.round_bf16(X64)
        Xd, tol = bf16_dev(X64), 1e-4
    else:
        X64 = X64.astype(np.float32).astype(np.float64)
        Xd, tol = dev(X64.astype(np.float32)), 1e-5
    A = rng.random((shape[mode], R)).astype(np.float32)
    print("case", shape, mode, R, dt, flush=True)
    out = host(nnc.nnc_ttm(Xd, mode, dev(A)))
    name = nnc.last_ttm_kernel()
    assert name.startswith("ttm_") and "generic" not in name, name
    ref = oracle.ttm_t(X64, mode, A.astype(np.float64))
    assert rel_fro(out, ref) <= tol, (name, rel_fro(out, ref))
    assert _fibre_err(out, ref, mode) <= 10 * tol, name


def test_chunked_passes_report_chunks():
    """The shapes that exceed one launch's LDS are the chunked ones."""
    nnc = need_gpu()
    X = dev(np.ones((64, 1024, 256), dtype=np.float32))
    nnc.nnc_ttm(X, 1, dev(np.ones((1024, 20), dtype=np.float32)))
    assert nnc.last_ttm_kernel() == "ttm_mid_f32 (chunked)"
    Xb = bf16_dev(np.ones((512, 512, 1024)))
    # the last-mode pass holds R + 1 factor rows: N_d = 1024 fits at R = 20, not at R = 32
    nnc.nnc_ttm(Xb, 2, dev(np.ones((1024, 20), dtype=np.float32)))
    assert nnc.last_ttm_kernel() == "ttm_last_lds_bf16"
    nnc.nnc_ttm(Xb, 2, dev(np.ones((1024, 32), dtype=np.float32)))
    assert nnc.last_ttm_kernel() == "ttm_last_lds_bf16 (chunked)"
    nnc.nnc_ttm(Xb, 0, dev(np.ones((512, 20), dtype=np.float32)))
    assert nnc.last_ttm_kernel() == "ttm_mid_bf16"
    # R = 32 at N = 512: the tile's output staged by halves, one launch (no chunks)
    nnc.nnc_ttm(Xb, 0, dev(np.ones((512, 32), dtype=np.float32)))
    assert nnc.last_ttm_kernel() == "ttm_mid_bf16"


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_fit_with_long_first_and_last_modes(dt):
    """A few nnTucker sweeps on 800 x 64 x 800 (both X passes chunked in the BF16 form, the
    last-mode pass in both forms) against the oracle."""
    nnc = need_gpu()
    X, _, G0, A0 = problem(91, (800, 64, 800), 5, (20, 20, 20))
    X64 = X.astype(np.float64)
    if dt == "bf16":
        X64 = synth.round_bf16(X64)
        Xd = bf16_dev(X64)
    else:
        Xd = dev(X)
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.nntucker_fit(Xd, G0.shape, 3, G, A)
    Go, Ao, _, _ = oracle.nntucker(X64, G0, A0, 3)
    assert rel_fro(oracle.tucker_full(host(G), [host(a) for a in A]), oracle.tucker_full(Go, Ao)) <= 1e-4
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X64, Go, Ao)) <= 1e-5
