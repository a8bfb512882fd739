"""The fused three-way sweep (both X passes carrying the next small contraction, the R x R
matrices of modes 0 and 1 formed by side jobs of the passes, in the first blocks to finish
their share of the stream; bf16 X) against the FP64
oracle and against the general fused schedule (selected by NNC_NO_FUSED3), on shapes that
span the pass kernels' cases: several slabs per block and fewer slabs than side rows,
ragged and padded multiranks, multiranks above the dimensions, one or two 16-column tiles,
pass-2 units of one tile per wave and of several.  FP32 X takes the general schedule; the
same cases run in that form too."""
import os

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import bf16_dev, dev, host, need_gpu, problem, rel_fro

pytestmark = pytest.mark.gpu

SHAPES = [((48, 32, 256), (5, 7, 9)),
          ((40, 48, 512), (20, 20, 20)),
          ((24, 32, 128), (3, 32, 8)),       # pass 2: one tile per i1 row, 8 groups per unit
          ((8, 32, 256), (20, 4, 20)),       # fewer slabs and units than side rows
          ((16, 16, 256), (20, 20, 20)),     # multirank above the first two dimensions
          ((300, 64, 256), (17, 1, 32)),     # several slabs per block, rank 1
          ((1, 16, 256), (1, 1, 1))]


def _fit(nnc, Xd, G0, A0, iters, **kw):
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.nntucker_fit(Xd, G0.shape, iters, G, A, **kw)
    return host(G), [host(a) for a in A], rep


def _general(nnc, Xd, G0, A0, iters, **kw):
    os.environ["NNC_NO_FUSED3"] = "1"
    try:
        return _fit(nnc, Xd, G0, A0, iters, **kw)
    finally:
        del os.environ["NNC_NO_FUSED3"]


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_fused3_few_sweeps_match_oracle(dims, ranks, dt):
    nnc = need_gpu()
    X, _, G0, A0 = problem(61, dims, 3, ranks)
    X64 = X.astype(np.float64)
    if dt == "bf16":
        import synth
        X64 = synth.round_bf16(X64)
        Xd = bf16_dev(X64)
    else:
        Xd = dev(X)
    print("case", dims, ranks, dt, flush=True)
    G, A, rep = _fit(nnc, Xd, G0, A0, 3)
    Go, Ao, _, _ = oracle.nntucker(X64, G0, A0, 3)
    assert rel_fro(oracle.tucker_full(G, A), oracle.tucker_full(Go, Ao)) <= 1e-4
    assert rel_fro(G, Go) <= 1e-3
    for a, ao in zip(A, Ao):
        assert rel_fro(a, ao) <= 1e-3
    assert (G >= 0).all() and all((a >= 0).all() for a in A)
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X64, Go, Ao)) <= 1e-5
    assert rep.eps_clips == 0
    # the general schedule computes the same sweep with other summation orders
    Gg, Ag, _ = _general(nnc, Xd, G0, A0, 3)
    assert rel_fro(G, Gg) <= 1e-5
    for a, ag in zip(A, Ag):
        assert rel_fro(a, ag) <= 1e-5


@pytest.mark.parametrize("use_graph", [False, True])
def test_fused3_many_sweeps_deterministic_and_resumable(use_graph):
    nnc = need_gpu()
    X, _, G0, A0 = problem(62, (64, 48, 256), 4, (6, 5, 7))
    import synth
    X = synth.round_bf16(X.astype(np.float64))
    Xd = bf16_dev(X)
    G1, A1, r1 = _fit(nnc, Xd, G0, A0, 30, use_graph=use_graph)
    G2, A2, r2 = _fit(nnc, Xd, G0, A0, 30, use_graph=use_graph)
    assert np.array_equal(G1, G2) and all(np.array_equal(a, b) for a, b in zip(A1, A2))
    assert r1.rel_residual == r2.rel_residual
    G = dev(G0)
    A = [dev(a) for a in A0]
    nnc.nntucker_fit(Xd, G0.shape, 17, G, A, use_graph=use_graph)
    nnc.nntucker_fit(Xd, G0.shape, 13, G, A, use_graph=use_graph)
    assert np.array_equal(host(G), G1) and all(np.array_equal(host(a), b) for a, b in zip(A, A1))
    Go, Ao, _, _ = oracle.nntucker(X.astype(np.float64), G0, A0, 30)
    assert abs(r1.rel_residual - oracle.tucker_rel_residual(X.astype(np.float64), Go, Ao)) <= 1e-4


def test_fused3_graph_replays_match_eager_sweeps():
    """Sweeps replayed from captured graphs (several sweeps per graph, a remainder graph) give
    the eager sweeps' results bit for bit, with the workspace reused across the fits, also
    after new contents are written into the same X buffer (the cached graphs read them)."""
    nnc = need_gpu()
    import synth
    X, _, G0, A0 = problem(67, (40, 48, 512), 4, (20, 20, 20))
    Xd = bf16_dev(synth.round_bf16(X.astype(np.float64)))
    dims, ranks = X.shape, G0.shape
    ws = torch.empty(nnc.nntucker_workspace_bytes(dims, ranks), dtype=torch.uint8, device="cuda")
    out = []
    for use_graph in (False, True, True):
        G = dev(G0)
        A = [dev(a) for a in A0]
        nnc.nntucker_fit(Xd, ranks, 19, G, A, use_graph=use_graph, workspace=ws, report=False)
        out.append((host(G), [host(a) for a in A]))
    for G, A in out[1:]:
        assert np.array_equal(G, out[0][0]) and all(np.array_equal(a, b) for a, b in zip(A, out[0][1]))
    # new contents in the same X buffer: the replayed graphs read them
    X2, _, _, _ = problem(68, (40, 48, 512), 4, (20, 20, 20))
    Xd.copy_(bf16_dev(synth.round_bf16(X2.astype(np.float64))))
    out2 = []
    for use_graph in (True, False):
        G = dev(G0)
        A = [dev(a) for a in A0]
        nnc.nntucker_fit(Xd, ranks, 19, G, A, use_graph=use_graph, workspace=ws, report=False)
        out2.append((host(G), [host(a) for a in A]))
    assert np.array_equal(out2[0][0], out2[1][0]) and all(np.array_equal(a, b) for a, b in zip(out2[0][1], out2[1][1]))
    assert not np.array_equal(out2[0][0], out[0][0])


def test_fused3_objective_history_monotone():
    nnc = need_gpu()
    X, _, G0, A0 = problem(63, (32, 32, 512), 4, (4, 4, 4))
    _, _, rep = _fit(nnc, bf16_dev(X.astype(np.float64)), G0, A0, 40, objective_every=1)
    f = 0.5 * np.array(rep.history) ** 2
    assert len(f) == 40 and (np.diff(f) <= 1e-6 * f[0]).all()


def test_fused3_bf16_with_fp32_refinement():
    nnc = need_gpu()
    X, _, G0, A0 = problem(64, (48, 32, 512), 3, (8, 8, 8))
    Xb = bf16_dev(X.astype(np.float64))
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.nntucker_fit(Xb, G0.shape, 40, G, A, x_fp32=dev(X), fp32_final_sweeps=10)
    Go, Ao, _, _ = oracle.nntucker(X.astype(np.float64), G0, A0, 40)
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X.astype(np.float64), Go, Ao)) <= 1e-3
    assert rep.eps_clips == 0


def test_fused3_zero_column_clips_match_oracle():
    nnc = need_gpu()
    import synth
    X, _, G0, A0 = problem(65, (32, 32, 256), 3, (5, 5, 5))
    X64 = synth.round_bf16(X.astype(np.float64))
    for z in range(3):
        A0z = [a.copy() for a in A0]
        A0z[z][:, 1] = 0.0
        Go, Ao, clips_o, _ = oracle.nntucker(X64, G0, A0z, 4)
        G, A, rep = _fit(nnc, bf16_dev(X64), G0, A0z, 4)
        assert rep.eps_clips == clips_o > 0, (z, rep.eps_clips, clips_o)
        assert rel_fro(G, Go) <= 1e-4


def test_fused3_unaligned_factor_falls_back():
    """A factor 4 bytes off a 16-byte boundary takes the general schedule (same results)."""
    nnc = need_gpu()
    import synth
    X, _, G0, A0 = problem(66, (48, 32, 256), 3, (5, 6, 7))
    X64 = synth.round_bf16(X.astype(np.float64))
    Xd = bf16_dev(X64)
    G1, A1, _ = _fit(nnc, Xd, G0, A0, 3)
    buf = torch.zeros(A0[2].size + 1, device="cuda", dtype=torch.float32)
    A2u = buf[1:].view(A0[2].shape)
    A2u.copy_(torch.from_numpy(A0[2]))
    G = dev(G0)
    A = [dev(A0[0]), dev(A0[1]), A2u]
    nnc.nntucker_fit(Xd, G0.shape, 3, G, A)
    Gg, Ag, _ = _general(nnc, Xd, G0, A0, 3)
    assert torch.equal(G, dev(Gg)) and all(torch.equal(a, dev(b)) for a, b in zip(A, Ag))
    assert rel_fro(host(G), G1) <= 1e-5
