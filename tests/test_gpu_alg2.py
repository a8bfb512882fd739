"""GPU parity of Algorithm 2 (nnCP of X, then an NMF of each CP factor) through the C ABI
against the FP64 oracle.

- nncpx_fit: a few sweeps from identical initial values on ragged 2- to 5-way shapes, FP32
  and BF16 X (the oracle reads the bf16 values), every rank class of the kernels (<= 8, <= 16,
  <= 32): factors within 1e-4 relative Frobenius.  Long runs: final relative residual within
  1e-3 of the oracle's.
- nmf_fit: a few sweeps, factors within 1e-4; residual after many sweeps within 1e-3.
- Algorithm 2 end to end on the 40^3 workload: lifted residual within 1e-3 of the oracle.
- 512^3, rank 10: one sweep of both forms against one oracle sweep.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import bf16_dev, dev, host, need_gpu, rel_fro

pytestmark = pytest.mark.gpu

CPX_CASES = [
    ((40, 40, 40), 3),
    ((30, 37, 41), 5),        # ragged
    ((33, 70, 29), 12),
    ((24, 20, 36), 20),
    ((17, 23, 19), 32),
    ((12, 13, 14, 15), 4),    # 4-way: Khatri-Rao weights on both sides of a mode
    ((6, 7, 5, 6, 4), 3),     # 5-way
    ((50, 70), 6),            # 2-way: plain NMF of X
    ((300, 40, 260), 10),     # several diagonal slices
    ((600, 12, 10), 32),      # the one-workgroup Gram in three LDS chunks of 256 rows (ragged)
    ((2000, 9, 7), 10),       # ... and of 810 rows
]


def _cp_problem(seed, dims, r):
    X, _ = synth.planted_tensor(seed, dims, max(2, r // 2), noise=1e-3, dtype="f32")
    B0 = synth.init_cp_factors(seed, dims, r)
    return X, B0


@pytest.mark.parametrize("dims,r", CPX_CASES)
def test_nncpx_few_sweeps_fp32(dims, r):
    nnc = need_gpu()
    X, B0 = _cp_problem(31, dims, r)
    B = [dev(b) for b in B0]
    rep = nnc.nncpx_fit(dev(X), r, 3, B)
    Bo, clips, _ = oracle.nncp(X.astype(np.float64), B0, 3)
    for b, bo in zip(B, Bo):
        assert rel_fro(host(b), bo) <= 1e-4, (dims, r, rel_fro(host(b), bo))
    assert rep.eps_clips == clips == 0
    C = [host(b) for b in B]
    assert abs(rep.rel_residual - oracle.cp_rel_residual(X.astype(np.float64), C)) <= 1e-6


@pytest.mark.parametrize("dims,r", [((40, 40, 40), 3), ((30, 37, 41), 20), ((12, 13, 14, 15), 4)])
def test_nncpx_few_sweeps_bf16(dims, r):
    nnc = need_gpu()
    X, B0 = _cp_problem(32, dims, r)
    Xb64 = synth.round_bf16(X.astype(np.float64))
    B = [dev(b) for b in B0]
    nnc.nncpx_fit(bf16_dev(Xb64), r, 3, B)
    Bo, _, _ = oracle.nncp(Xb64, B0, 3)
    for b, bo in zip(B, Bo):
        assert rel_fro(host(b), bo) <= 1e-4, (dims, r, rel_fro(host(b), bo))


def test_nncpx_zero_sweeps_and_resume():
    """iters = 0 leaves the factors; 4 sweeps in one call equal 2 + 2 (graph and eager paths)."""
    nnc = need_gpu()
    dims, r = (30, 37, 41), 5
    X, B0 = _cp_problem(33, dims, r)
    Xd = dev(X)
    B = [dev(b) for b in B0]
    nnc.nncpx_fit(Xd, r, 0, B)
    assert all(np.array_equal(host(b), b0.astype(np.float64)) for b, b0 in zip(B, B0))
    one = [dev(b) for b in B0]
    nnc.nncpx_fit(Xd, r, 4, one, use_graph=True)
    two = [dev(b) for b in B0]
    nnc.nncpx_fit(Xd, r, 2, two, use_graph=False)
    nnc.nncpx_fit(Xd, r, 2, two, use_graph=False)
    for a, b in zip(one, two):
        assert torch.equal(a, b)


def test_nncpx_objective_history_non_increasing():
    nnc = need_gpu()
    dims, r = (40, 40, 40), 3
    X, B0 = _cp_problem(34, dims, r)
    B = [dev(b) for b in B0]
    rep = nnc.nncpx_fit(dev(X), r, 30, B, objective_every=5)
    h = rep.history
    assert len(h) == 6 and all(np.isfinite(h))
    assert all(h[i + 1] <= h[i] * (1 + 1e-6) for i in range(len(h) - 1)), h


@pytest.mark.parametrize("dims,r", [((40, 40, 40), 3), ((30, 37, 41), 5)])
def test_nncpx_long_run_residual(dims, r):
    nnc = need_gpu()
    X, B0 = _cp_problem(35, dims, r)
    B = [dev(b) for b in B0]
    rep = nnc.nncpx_fit(dev(X), r, 300, B)
    Bo, _, _ = oracle.nncp(X.astype(np.float64), B0, 300)
    ref = oracle.cp_rel_residual(X.astype(np.float64), Bo)
    assert abs(rep.rel_residual - ref) <= 1e-3, (rep.rel_residual, ref)
    assert all(float(b.min()) >= 0 for b in B)


@pytest.mark.parametrize("rows,cols,m", [(40, 3, 5), (512, 10, 20), (37, 9, 4), (200, 32, 32),
                                          (60, 40, 32)])  # the last one runs as a two-way nnCP
def test_nmf_matches_oracle(rows, cols, m):
    nnc = need_gpu()
    rng = np.random.default_rng(rows * 100 + m)
    A = rng.random((rows, cols)).astype(np.float32)
    W0 = rng.random((rows, m)).astype(np.float32)
    H0 = rng.random((m, cols)).astype(np.float32)
    W, H = dev(W0), dev(H0)
    res = nnc.nmf_fit(dev(A), m, 4, W, H)
    Wo, Ho, _ = oracle.nmf(A.astype(np.float64), W0, H0, 4)
    assert rel_fro(host(W), Wo) <= 1e-4 and rel_fro(host(H), Ho) <= 1e-4
    ref = np.linalg.norm(A - Wo @ Ho) / np.linalg.norm(A)
    assert abs(res - ref) <= 1e-5
    W, H = dev(W0), dev(H0)
    res = nnc.nmf_fit(dev(A), m, 300, W, H)
    Wo, Ho, _ = oracle.nmf(A.astype(np.float64), W0, H0, 300)
    assert abs(res - np.linalg.norm(A - Wo @ Ho) / np.linalg.norm(A)) <= 1e-3


def test_nmf_too_large_for_one_workgroup_is_unsupported():
    """5000 x 10 at rank 8 fits neither the one-workgroup NMF kernel nor the nnCP kernel's LDS:
    a clean NNC_EUNSUPPORTED, inputs untouched."""
    nnc = need_gpu()
    rng = np.random.default_rng(8)
    A = dev(rng.random((5000, 10)).astype(np.float32))
    W0 = rng.random((5000, 8)).astype(np.float32)
    W, H = dev(W0), dev(rng.random((8, 10)).astype(np.float32))
    with pytest.raises(nnc.NncError) as e:
        nnc.nmf_fit(A, 8, 5, W, H)
    assert e.value.status == nnc.NNC_EUNSUPPORTED
    assert np.array_equal(host(W), W0.astype(np.float64))


def test_nmf_batched_matches_single():
    """Uneven problems in one call equal the single calls bit for bit, residuals included."""
    nnc = need_gpu()
    rng = np.random.default_rng(7)
    shapes = [(40, 5), (512, 20), (1000, 12), (33, 3)]
    A = [dev(rng.random((n, 10)).astype(np.float32)) for n, _ in shapes]
    W0 = [rng.random((n, m)).astype(np.float32) for n, m in shapes]
    H0 = [rng.random((m, 10)).astype(np.float32) for _, m in shapes]
    W, H = [dev(w) for w in W0], [dev(h) for h in H0]
    res = nnc.nmf_fit_batched(A, [m for _, m in shapes], 20, W, H)
    for j, (n, m) in enumerate(shapes):
        w, h = dev(W0[j]), dev(H0[j])
        r1 = nnc.nmf_fit(A[j], m, 20, w, h)
        assert torch.equal(w, W[j]) and torch.equal(h, H[j]), j
        assert res[j] == r1, (j, res[j], r1)


def test_alg2_end_to_end_40cubed():
    """The 40^3 workload (planted rank 3): nnCP rank 3 x 300 sweeps, NMF with m = (5, 5, 5)
    x 300 sweeps, lift, residual of the lifted model."""
    nnc = need_gpu()
    dims, r, m = (40, 40, 40), 3, (5, 5, 5)
    X, _ = synth.planted_tensor(1, dims, 3, noise=1e-3, dtype="f32")
    B0 = synth.init_cp_factors(1, dims, r)
    F0, H0 = synth.init_nmf(1, dims, m, r)
    Xd = dev(X)
    Acp = [dev(b) for b in B0]
    F = [dev(f) for f in F0]
    H = [dev(h) for h in H0]
    nnc.nncandelinc_alg2(Xd, r, m, 300, 300, Acp, F, H)
    C = nnc.nncandelinc_lift(F, H)
    rel = nnc.reconstruct_residual(Xd, C)
    ref = oracle.nncandelinc_alg2(X.astype(np.float64), B0, F0, H0, 300, 300)
    assert abs(rel - ref["cp_rel"]) <= 1e-3, (rel, ref["cp_rel"])
    assert abs(nnc.reconstruct_residual(Xd, Acp) - ref["cp_x_rel"]) <= 1e-3


def test_nncpx_512cubed_one_sweep_both_forms():
    nnc = need_gpu()
    N, r = 512, 10
    X32, _ = synth.planted_tensor(2, (N, N, N), 10, zero_prob=0.5, noise=1e-3, dtype="f32")
    B0 = synth.init_cp_factors(2, (N, N, N), r)
    Xd = dev(X32)
    Xb = nnc.nnc_convert_f32_bf16(Xd)
    Bo, _, _ = oracle.nncp(X32.astype(np.float64), B0, 1)
    for bf, tol in ((False, 1e-4), (True, 2e-3)):
        B = [dev(b) for b in B0]
        nnc.nncpx_fit(Xb if bf else Xd, r, 1, B)
        for b, bo in zip(B, Bo):
            assert rel_fro(host(b), bo) <= tol, (bf, rel_fro(host(b), bo))
