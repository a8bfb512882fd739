"""Real-valued CANDELINC at full size (512^3 real tensor, Tucker multirank 20^3, 25 sweeps;
CP rank 20 of the core, 300 sweeps) against the FP64 oracle's stored results
(tests/golden/real512_reference.json, written by tests/golden/make_real512_reference.py from
the oracle and the seeded generator only).

- The Tucker fit: the final relative residual and the per-sweep residuals, and the factor
  subspaces through their projectors A_n A_n^T (the bases themselves can rotate).
- The CP fit of the oracle's own core (rounded to float32, real512_core.npy) from the same
  initial values: its residual, and the lifted model's residual against X through the
  oracle's factors.
X is built on the GPU from the same seeded draws (tests.gpu_util.signed_planted_dev)."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import dev, host, need_gpu, rel_fro, signed_planted_dev

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = os.path.join(HERE, "real512_reference.json")


@pytest.fixture(scope="module")
def ref():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/real512_reference.json not generated")
    with open(GOLDEN) as f:
        r = json.load(f)
    nnc = need_gpu()
    X = signed_planted_dev(r["seed"], r["dims"], r["planted_rank"], noise=r["noise"])
    return nnc, r, X


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_real512_tucker_matches_stored_oracle(ref, form):
    nnc, r, X = ref
    dims, ranks = r["dims"], r["multirank"]
    G = dev(synth.init_core(r["seed"], ranks))
    A = [dev(a) for a in synth.init_factors(r["seed"], dims, ranks)]
    if form == "bf16":
        Xb = nnc.nnc_convert_f32_bf16(X)
        rep = nnc.tucker_ls_fit(Xb, ranks, r["sweeps"], G, A, x_fp32=X, fp32_final_sweeps=5,
                                objective_every=1)
        tol = 1e-3
    else:
        rep = nnc.tucker_ls_fit(X, ranks, r["sweeps"], G, A, objective_every=1)
        tol = 1e-5
    print("real512", form, rep.rel_residual, "oracle", r["tucker_rel"], flush=True)
    assert abs(rep.rel_residual - r["tucker_rel"]) <= tol * max(1.0, r["tucker_rel"])
    hist = np.array(rep.history)
    ho = np.array(r["tucker_rel_history"])
    assert len(hist) == len(ho)
    # The first sweep starts from random factors: its first systems K_n are ill-conditioned
    # (condition numbers near 1e7 here), so FP32 rounding moves that sweep's model; in the
    # oracle, relative perturbations of 1e-7..1e-6 in num_n and K_n move the first sweep's
    # residual by 0.4-2 % on a 64^3 instance of this workload and the later ones by < 1e-8.
    # From the second sweep on the fit sits on the dominant subspaces and agrees closely.  The
    # BF16 form's first sweep reads X rounded to 8 bits of mantissa, a far larger perturbation
    # of those systems, so only the FP32 form's first residual is held to the oracle's.
    if form == "f32":
        assert abs(hist[0] - ho[0]) <= 0.5 * ho[0]
    assert np.abs(hist[1:] - ho[1:]).max() <= tol * max(1.0, ho.max())
    with np.load(os.path.join(HERE, r["factors_npz"])) as z:
        Ao = [z["arr_%d" % k].astype(np.float64) for k in range(3)]
    for a, ao in zip(A, Ao):
        a = host(a)
        assert np.abs(a.T @ a - np.eye(a.shape[1])).max() <= 1e-5
        assert rel_fro(a @ a.T, ao @ ao.T) <= (1e-4 if form == "f32" else 1e-2)


def test_real512_cp_of_the_oracle_core(ref):
    nnc, r, X = ref
    core = dev(np.load(os.path.join(HERE, r["core_npy"])))
    B = [dev(2.0 * b - 1.0) for b in synth.init_cp_factors(r["seed"], r["multirank"], r["cp_rank"])]
    rep = nnc.cp_ls_fit(core, r["cp_rank"], r["cp_sweeps"], B, report=True)
    print("real512 core cp", rep.rel_residual, "oracle", r["core_cp_rel"], flush=True)
    assert abs(rep.rel_residual - r["core_cp_rel"]) <= 1e-4 * max(1.0, r["core_cp_rel"]) + 1e-5
    with np.load(os.path.join(HERE, r["factors_npz"])) as z:
        Ao = [dev(z["arr_%d" % k]) for k in range(3)]
    C = nnc.nncandelinc_lift(Ao, B)
    cp_rel = nnc.reconstruct_residual(X, C)
    print("real512 lifted", cp_rel, "oracle", r["cp_rel"], flush=True)
    assert abs(cp_rel - r["cp_rel"]) <= 1e-4 * max(1.0, r["cp_rel"]) + 1e-5
