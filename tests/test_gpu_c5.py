"""The 64^5 workload (planted rank 6, U[0,1) factors, U[0,1e-3) noise, stored FP32, 4.3 GB)
at its full sweep counts against the FP64 oracle's results stored in
tests/golden/c5_reference.json by tests/golden/make_c5_reference.py (oracle only):

- nnTucker multirank 8^5, 300 sweeps from the seeded initial values: final relative residual
  within 1e-3 of the oracle's (X is built on the GPU from the same seeded draws);
- 64 random-restart nnCP fits of the oracle's fitted core (rounded to float32,
  c5_core.npy), ranks 2 + (j mod 15), 300 sweeps each, in one batched launch: every
  restart's relative residual within 1e-3 of the oracle's on the identical input.
"""
import json
import os

import numpy as np
import pytest

import synth
from tests.gpu_util import dev, need_gpu, planted_tensor_dev

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = os.path.join(HERE, "c5_reference.json")
SEED, N, D, PLANTED, R = 5, 64, 5, 6, 8


def _ref():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/c5_reference.json not generated")
    return json.load(open(GOLDEN))


def test_c5_full_sweeps_match_stored_oracle():
    ref = _ref()
    nnc = need_gpu()
    import torch
    dims, ranks = (N,) * D, (R,) * D
    X = planted_tensor_dev(SEED, dims, PLANTED, noise=1e-3)
    # the device build against the host generator on its first chunk of rows
    X0, _ = synth.planted_tensor(SEED, (2,) + dims[1:], PLANTED, noise=1e-3, dtype="f32")
    head = X[:2].cpu().numpy()
    assert (np.abs(head - X0) <= np.spacing(np.abs(X0))).all()  # at most one float32 ulp
    G = dev(synth.init_core(SEED, ranks))
    A = [dev(a) for a in synth.init_factors(SEED, dims, ranks)]
    rep = nnc.nntucker_fit(X, ranks, ref["sweeps"], G, A)
    print("c5 tucker", rep.rel_residual, "oracle", ref["tucker_rel"], flush=True)
    assert abs(rep.rel_residual - ref["tucker_rel"]) <= 1e-3
    assert rep.eps_clips == ref["clips"] == 0
    assert float(G.min()) >= 0 and all(float(a.min()) >= 0 for a in A)
    del X
    torch.cuda.empty_cache()


def test_c5_batched_restarts_match_stored_oracle():
    ref = _ref()
    nnc = need_gpu()
    ranks = (R,) * D
    core = np.load(os.path.join(HERE, ref["core_npy"]))
    assert core.shape == ranks and core.dtype == np.float32
    cp_ranks = ref["restart_ranks"]
    facs = [[dev(b) for b in synth.init_cp_factors(SEED, ranks, r, restart=j)] for j, r in enumerate(cp_ranks)]
    res = nnc.nncp_fit_batched(dev(core), cp_ranks, ref["cp_sweeps"], facs)
    err = np.abs(np.array(res) - np.array(ref["restart_core_rel"]))
    print("c5 restarts max |diff|", err.max(), "at", int(err.argmax()), flush=True)
    assert err.max() <= 1e-3, (int(err.argmax()), res[int(err.argmax())])
