"""Real-valued CANDELINC on the GPU (Section 2.2: Tucker fit by alternating least squares with
orthonormalized factors, CP fit of the core by alternating least squares, lift) against the
FP64 oracle on the same seeded signed inputs."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import bf16_dev, dev, host, need_gpu, rel_fro

pytestmark = pytest.mark.gpu

SHAPES = [((48, 32, 256), (5, 7, 9)),
          ((40, 48, 512), (20, 20, 20)),
          ((64, 20, 33), (3, 4, 2)),
          ((24, 16, 20, 32), (4, 5, 3, 6)),
          ((10, 12, 8, 9, 16), (2, 3, 2, 3, 2))]


def _inputs(seed, dims, ranks, noise=1e-2):
    """Planted real Tucker data of the fitted multilinear rank (a clear gap in every mode's
    spectrum, so the fitted subspaces are well determined) and U[0,1) initial values."""
    X = synth.signed_planted_tucker(seed, dims, ranks, noise=noise)
    G0 = synth.init_core(seed, ranks)
    A0 = synth.init_factors(seed, dims, ranks)
    return X.astype(np.float32), None, G0, A0


def _check_same_fit(G, A, Go, Ao, model_tol, proj_tol):
    """Same model and same factor subspaces (projectors A_n A_n^T).  The core and the bases
    themselves are compared only through these: a basis of a well-determined subspace can
    still rotate under rounding when the least-squares systems are ill-conditioned."""
    assert rel_fro(oracle.tucker_full(G, A), oracle.tucker_full(Go, Ao)) <= model_tol
    for a, ao in zip(A, Ao):
        assert rel_fro(a @ a.T, ao @ ao.T) <= proj_tol
        assert np.abs(a.T @ a - np.eye(a.shape[1])).max() <= 1e-5


def _fit(nnc, Xd, G0, A0, iters, **kw):
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.tucker_ls_fit(Xd, G0.shape, iters, G, A, **kw)
    return host(G), [host(a) for a in A], rep


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_tucker_ls_few_sweeps_match_oracle(dims, ranks, dt):
    nnc = need_gpu()
    X, _, G0, A0 = _inputs(71, dims, ranks)
    X64 = X.astype(np.float64)
    if dt == "bf16":
        X64 = synth.round_bf16(X64)
        Xd = bf16_dev(X64)
    else:
        Xd = dev(X)
    print("case", dims, ranks, dt, flush=True)
    G, A, rep = _fit(nnc, Xd, G0, A0, 3)
    Go, Ao, _ = oracle.tucker_ls(X64, G0, A0, 3)
    _check_same_fit(G, A, Go, Ao, 1e-4, 1e-4)
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X64, Go, Ao)) <= 1e-5
    assert rep.eps_clips == 0


@pytest.mark.parametrize("use_graph", [False, True])
def test_tucker_ls_many_sweeps_deterministic_resumable_and_monotone(use_graph):
    nnc = need_gpu()
    dims, ranks = (64, 48, 256), (6, 5, 7)
    X, _, G0, A0 = _inputs(72, dims, ranks)
    Xd = dev(X)
    G1, A1, r1 = _fit(nnc, Xd, G0, A0, 30, use_graph=use_graph, objective_every=1)
    G2, A2, r2 = _fit(nnc, Xd, G0, A0, 30, use_graph=use_graph)
    assert np.array_equal(G1, G2) and all(np.array_equal(a, b) for a, b in zip(A1, A2))
    assert r1.rel_residual == r2.rel_residual
    f = np.array(r1.history) ** 2
    assert len(f) == 30 and (np.diff(f) <= 1e-6 * f[0]).all()
    Go, Ao, _ = oracle.tucker_ls(X.astype(np.float64), G0, A0, 30)
    assert abs(r1.rel_residual - oracle.tucker_rel_residual(X.astype(np.float64), Go, Ao)) <= 1e-6
    _check_same_fit(G1, A1, Go, Ao, 1e-5, 1e-5)
    # sweeps split over two calls continue from the returned (orthonormal) state; the second
    # call's orthonormalization of already orthonormal factors moves them by rounding only
    G = dev(G0)
    A = [dev(a) for a in A0]
    nnc.tucker_ls_fit(Xd, G0.shape, 17, G, A, use_graph=use_graph)
    nnc.tucker_ls_fit(Xd, G0.shape, 13, G, A, use_graph=use_graph)
    assert rel_fro(oracle.tucker_full(host(G), [host(a) for a in A]), oracle.tucker_full(G1, A1)) <= 1e-5


def test_tucker_ls_bf16_with_fp32_refinement():
    nnc = need_gpu()
    dims, ranks = (48, 32, 512), (8, 8, 8)
    X, _, G0, A0 = _inputs(73, dims, ranks)
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.tucker_ls_fit(bf16_dev(X.astype(np.float64)), G0.shape, 12, G, A, x_fp32=dev(X),
                            fp32_final_sweeps=4)
    Go, Ao, _ = oracle.tucker_ls(X.astype(np.float64), G0, A0, 12)
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X.astype(np.float64), Go, Ao)) <= 1e-4


def test_tucker_ls_zero_iterations_orthonormalizes_only():
    nnc = need_gpu()
    X, _, G0, A0 = _inputs(74, (40, 30, 64), (4, 3, 5))
    G, A, rep = _fit(nnc, dev(X), G0, A0, 0)
    Go, Ao, _ = oracle.tucker_ls(X.astype(np.float64), G0, A0, 0)
    assert rel_fro(oracle.tucker_full(G, A), oracle.tucker_full(G0.astype(np.float64), A0)) <= 1e-6
    # one QR of the caller's factors: a unique, well-conditioned representation here
    for a, ao in zip(A, Ao):
        assert rel_fro(a, ao) <= 1e-5
    assert rel_fro(G, Go) <= 1e-5


def test_tucker_ls_zero_core_is_reported():
    """A zero core makes every K_n zero: not positive definite, NNC_ENUMERIC (the oracle's
    solve raises on the same input)."""
    nnc = need_gpu()
    X, _, G0, A0 = _inputs(75, (32, 24, 64), (3, 3, 3))
    G0 = np.zeros_like(G0)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.tucker_ls(X.astype(np.float64), G0, A0, 1)
    with pytest.raises(nnc.NncError) as e:
        _fit(nnc, dev(X), G0, A0, 1)
    assert e.value.status == nnc.NNC_ENUMERIC


# --------------------------------------------------------------------------- CP of the core
def _core_problem(seed, dims, r, noise=1e-3):
    T, _ = synth.signed_planted(seed, dims, r, noise=noise)
    B0 = [2.0 * b - 1.0 for b in synth.init_cp_factors(seed, dims, r)]
    return T.astype(np.float32), [b.astype(np.float32) for b in B0]


@pytest.mark.parametrize("dims,r,iters", [((8, 8, 8), 5, 30), ((20, 20, 20), 10, 20), ((6, 7, 5, 4), 3, 40),
                                          ((4, 4), 2, 10), ((32, 30, 20), 16, 10)])
def test_cp_ls_matches_oracle(dims, r, iters):
    nnc = need_gpu()
    T, B0 = _core_problem(81, dims, r)
    print("case", dims, r, iters, flush=True)
    Bd = [dev(b) for b in B0]
    rep = nnc.cp_ls_fit(dev(T), r, iters, Bd, report=True)
    Bo, _ = oracle.cp_ls(T.astype(np.float64), B0, iters)
    assert abs(rep.rel_residual - oracle.cp_rel_residual(T.astype(np.float64), Bo)) <= 1e-5
    assert rel_fro(oracle.cp_full([host(b) for b in Bd]), oracle.cp_full(Bo)) <= 1e-4
    assert rep.eps_clips == 0


def test_cp_ls_singular_gram_is_reported():
    """A zero column in a factor makes H_n of the other modes singular: NNC_ENUMERIC (the
    oracle's solve raises on the same input)."""
    nnc = need_gpu()
    T, B0 = _core_problem(82, (6, 6, 6), 3)
    B0[2][:, 1] = 0.0
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cp_ls(T.astype(np.float64), B0, 1)
    with pytest.raises(nnc.NncError) as e:
        nnc.cp_ls_fit(dev(T), 3, 1, [dev(b) for b in B0], report=True)
    assert e.value.status == nnc.NNC_ENUMERIC


# --------------------------------------------------------------------------- end to end
def test_candelinc_recovers_a_cpd_with_a_rank_deficient_factor():
    """Section 2.2: a rank-4 CPD whose first factor has rank 3.  Tucker at the minimal
    multirank (3, 4, 4), a rank-4 CP of the core, the lift: the CPD comes back, on the GPU as
    in the oracle."""
    nnc = need_gpu()
    dims, m, r = (96, 64, 48), (3, 4, 4), 4
    X, P = synth.signed_planted(83, dims, r, noise=0.0, deficient_mode=0)
    X32 = X.astype(np.float32)
    Xd = dev(X32)
    G0 = synth.init_core(83, m)
    A0 = synth.init_factors(83, dims, m)
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.tucker_ls_fit(Xd, m, 10, G, A)
    assert rep.rel_residual <= 1e-6
    best = None
    for j in range(4):
        B0 = [2.0 * b - 1.0 for b in synth.init_cp_factors(83, m, r, restart=j)]
        B = [dev(b) for b in B0]
        nnc.cp_ls_fit(G, r, 500, B)
        C = nnc.nncandelinc_lift(A, B)
        res = nnc.reconstruct_residual(Xd, C)
        if best is None or res < best[0]:
            best = (res, [host(c) for c in C], B0)
    res, C, B0 = best
    assert res <= 1e-5
    assert oracle.mean_congruence(C, P) >= 1 - 1e-5
    out = oracle.candelinc(X32.astype(np.float64), G0, A0, B0, 10, 500)
    assert out["cp_rel"] <= 1e-6
    assert oracle.mean_congruence(out["C"], P) >= 1 - 1e-6
