"""The eps-guarded division of the multiplicative updates, A <- A * num / max(den, eps)
(reading R3: the paper is silent on the guard, Section 4.1), on the GPU against the FP64
oracle.  A factor column that starts at zero makes its Gram row and column zero, so later
denominators are exactly zero on both sides and take the guard: the clip counts must match
the oracle's exactly (integer), the zero column must stay zero, and the iterates must match
at the usual tolerance."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import bf16_dev, dev, host, need_gpu, rel_fro

pytestmark = pytest.mark.gpu

SWEEPS = 5


@pytest.mark.parametrize("dims,ranks,zero_mode,form", [
    ((40, 40, 40), (5, 5, 5), 1, "f32"),
    ((40, 40, 40), (5, 5, 5), 1, "bf16"),
    ((40, 36, 24), (6, 4, 5), 0, "f32"),
    ((24, 20, 16, 12), (4, 3, 5, 2), 2, "f32"),
    ((40, 40, 40), (34, 3, 3), 1, "f32"),   # multirank above 32: the general (unfused) sweep
])
def test_nntucker_zero_column_clips_match_oracle(dims, ranks, zero_mode, form):
    nnc = need_gpu()
    seed = 140 + zero_mode
    X32, _ = synth.planted_tensor(seed, dims, 3, dtype="f32")
    X64 = X32.astype(np.float64)
    G0 = synth.init_core(seed, ranks)
    A0 = synth.init_factors(seed, dims, ranks)
    A0[zero_mode][:, 1] = 0.0
    if form == "bf16":
        X64 = synth.round_bf16(X64)
        Xd = bf16_dev(X64)
    else:
        Xd = dev(X32)
    Go, Ao, clips_o, _ = oracle.nntucker(X64, G0, A0, SWEEPS)
    assert clips_o > 0
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.nntucker_fit(Xd, ranks, SWEEPS, G, A)
    print("case", dims, ranks, zero_mode, form, rep.eps_clips, clips_o, flush=True)
    assert rep.eps_clips == clips_o
    assert (host(A[zero_mode])[:, 1] == 0).all()
    assert rel_fro(host(G), Go) <= 1e-4
    for a, ao in zip(A, Ao):
        assert rel_fro(host(a), ao) <= 1e-4
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X64, Go, Ao)) <= 1e-5


@pytest.mark.parametrize("core_dims,rank", [((20, 20, 20), 10), ((8, 7, 6, 5), 4), ((12, 9), 3)])
def test_nncp_zero_column_clips_match_oracle(core_dims, rank):
    nnc = need_gpu()
    seed = 150 + rank
    T = synth.uniform(seed, synth.STREAM_CORE0, int(np.prod(core_dims))).reshape(core_dims).astype(np.float32)
    B0 = synth.init_cp_factors(seed, core_dims, rank)
    B0[1][:, 1] = 0.0
    Bo, clips_o, _ = oracle.nncp(T, B0, 20)
    assert clips_o > 0
    for fit in (nnc.nncp_fit, nnc.nncp_fit_noalloc):
        B = [dev(b) for b in B0]
        rep = fit(dev(T), rank, 20, B, report=True)
        assert rep.eps_clips == clips_o, (fit.__name__, rep.eps_clips, clips_o)
        for k in range(len(core_dims)):
            assert (host(B[k])[:, 1] == 0).all()
        for b, bo in zip(B, Bo):
            assert rel_fro(host(b), bo) <= 1e-4
        assert abs(rep.rel_residual - oracle.cp_rel_residual(T, Bo)) <= 1e-5


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_nncpx_zero_column_clips_match_oracle(form):
    nnc = need_gpu()
    dims, r = (40, 36, 32), 6
    X32, _ = synth.planted_tensor(160, dims, 3, dtype="f32")
    X64 = X32.astype(np.float64)
    if form == "bf16":
        X64 = synth.round_bf16(X64)
        Xd = bf16_dev(X64)
    else:
        Xd = dev(X32)
    B0 = synth.init_cp_factors(160, dims, r)
    B0[2][:, 1] = 0.0
    Bo, clips_o, _ = oracle.nncp(X64, B0, SWEEPS)
    assert clips_o > 0
    B = [dev(b) for b in B0]
    rep = nnc.nncpx_fit(Xd, r, SWEEPS, B)
    assert rep.eps_clips == clips_o, (rep.eps_clips, clips_o)
    for k in range(3):
        assert (host(B[k])[:, 1] == 0).all()
    for b, bo in zip(B, Bo):
        assert rel_fro(host(b), bo) <= 1e-4


@pytest.mark.parametrize("rows,cols,rank", [(60, 10, 4), (500, 40, 4)])  # one-workgroup NMF; two-way nnCP (cols > 32)
def test_nmf_zero_column_matches_oracle(rows, cols, rank):
    """W's column 1 starts at zero: H's row 1 becomes zero in the first sweep and both stay
    zero (the guard keeps 0 * 0 / eps = 0); the iterates match the oracle."""
    nnc = need_gpu()
    A = synth.uniform(170, 0, rows * cols).reshape(rows, cols).astype(np.float32)
    W0 = synth.uniform_matrix(170, synth.STREAM_NMF_W, rows, rank).astype(np.float32)
    H0 = synth.uniform_matrix(170, synth.STREAM_NMF_H, rank, cols).astype(np.float32)
    W0[:, 1] = 0.0
    Wo, Ho, clips_o = oracle.nmf(A, W0, H0, 10)
    assert clips_o > 0
    W, H = dev(W0), dev(H0)
    nnc.nmf_fit(dev(A), rank, 10, W, H)
    assert (host(W)[:, 1] == 0).all() and (host(H)[1, :] == 0).all()
    assert rel_fro(host(W), Wo) <= 1e-4
    assert rel_fro(host(H), Ho) <= 1e-4
