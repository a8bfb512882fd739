"""The 128^4 workload stored as bfloat16 (planted rank 8, U[0,1) factors, U[0,1e-3) noise),
multirank 16^4, at its full sweep count against the FP64 oracle's results stored in
tests/golden/c3_reference.json by tests/golden/make_c3_reference.py (oracle only):

- the BF16 form (bf16 MFMA on the stored values, the last 20 sweeps in FP32 on their exact
  FP32 widening) and the FP32 form (FP32 MFMA on that widening), 500 sweeps each from the
  seeded initial values: final relative residual within 1e-3 of the oracle's; then nnCP
  rank 8 of the fitted core (300 sweeps) and the lift: lifted residual within 1e-3;
- nnCP rank 8 (300 sweeps) of the oracle's own fitted core (rounded to float32, c3_core.npy),
  the identical input on both sides: core residual within 1e-3.
"""
import json
import os

import numpy as np
import pytest

import synth
from tests.gpu_util import dev, need_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = os.path.join(HERE, "c3_reference.json")
SEED, N, D, PLANTED, R, RANK, SWEEPS, CP_SWEEPS, FP32_FINAL = 3, 128, 4, 8, 16, 8, 500, 300, 20


@pytest.fixture(scope="module")
def c3():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/c3_reference.json not generated")
    nnc = need_gpu()
    import torch
    dims, ranks = (N,) * D, (R,) * D
    bits, _ = synth.planted_tensor(SEED, dims, PLANTED, noise=1e-3, dtype="bf16")
    Xb = torch.from_numpy(bits.view(np.int16)).to("cuda").view(torch.bfloat16)
    del bits
    X32 = Xb.float()  # exact widening of the stored values
    return nnc, json.load(open(GOLDEN)), Xb, X32, dims, ranks


@pytest.mark.parametrize("form", ["bf16", "fp32"])
def test_c3_full_sweeps_match_stored_oracle(c3, form):
    nnc, ref, Xb, X32, dims, ranks = c3
    G = dev(synth.init_core(SEED, ranks))
    A = [dev(a) for a in synth.init_factors(SEED, dims, ranks)]
    if form == "bf16":
        rep = nnc.nntucker_fit(Xb, ranks, SWEEPS, G, A, x_fp32=X32, fp32_final_sweeps=FP32_FINAL)
    else:
        rep = nnc.nntucker_fit(X32, ranks, SWEEPS, G, A)
    print("c3", form, "tucker", rep.rel_residual, "oracle", ref["tucker_rel"], flush=True)
    assert abs(rep.rel_residual - ref["tucker_rel"]) <= 1e-3, (form, rep.rel_residual, ref["tucker_rel"])
    assert rep.eps_clips == ref["clips"] == 0
    assert float(G.min()) >= 0 and all(float(a.min()) >= 0 for a in A)
    B = [dev(b) for b in synth.init_cp_factors(SEED, ranks, RANK)]
    nnc.nncp_fit(G, RANK, CP_SWEEPS, B)
    cp_rel = nnc.reconstruct_residual(X32, nnc.nncandelinc_lift(A, B))
    print("c3", form, "lifted", cp_rel, "oracle", ref["cp_rel"], flush=True)
    assert abs(cp_rel - ref["cp_rel"]) <= 1e-3, (form, cp_rel, ref["cp_rel"])


def test_c3_nncp_of_the_oracle_core(c3):
    nnc, ref, _, _, _, ranks = c3
    core = np.load(os.path.join(HERE, ref["core_npy"]))
    assert core.shape == ranks and core.dtype == np.float32
    B = [dev(b) for b in synth.init_cp_factors(SEED, ranks, RANK)]
    rep = nnc.nncp_fit(dev(core), RANK, CP_SWEEPS, B, report=True)
    assert abs(rep.rel_residual - ref["core_cp_rel"]) <= 1e-3, (rep.rel_residual, ref["core_cp_rel"])
    assert rep.eps_clips == ref["core_cp_clips"]
