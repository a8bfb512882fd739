"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force sums written
here with plain Python loops, the paper's printed integer examples (exact), algebraic
identities of the n-mode product (Appendix A), textbook special cases (Lee-Seung NMF),
finite differences, invariants of multiplicative updates, and planted recovery.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.paper_fixtures import arr, examples, fold, fold_ex6


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------- n-mode product
def _nmode_brute(X, n, M):
    shape = list(X.shape)
    shape[n] = M.shape[0]
    out = np.zeros(shape)
    for idx in itertools.product(*[range(s) for s in shape]):
        s = 0.0
        for l in range(X.shape[n]):
            src = list(idx)
            src[n] = l
            s += X[tuple(src)] * M[idx[n], l]
        out[idx] = s
    return out


@pytest.mark.parametrize("shape", [(3, 4), (2, 3, 4), (3, 2, 2, 3), (2, 2, 3, 2, 2)])
def test_nmode_matches_brute_force_every_mode(shape):
    rng = _rng(len(shape))
    X = rng.random(shape)
    for n in range(len(shape)):
        M = rng.random((3, shape[n]))
        np.testing.assert_allclose(oracle.nmode(X, n, M), _nmode_brute(X, n, M), rtol=1e-14, atol=0)
        A = rng.random((shape[n], 2))
        np.testing.assert_allclose(oracle.ttm_t(X, n, A), _nmode_brute(X, n, A.T), rtol=1e-14, atol=0)


def test_identity_factor_returns_x_exactly():
    X = _rng(1).random((5, 6, 7))
    for n in range(3):
        assert np.array_equal(oracle.ttm_t(X, n, np.eye(X.shape[n])), X)


def test_mode_products_commute_and_distribute():
    """(X x_i A) x_j B = (X x_j B) x_i A for i != j and X x_i (AB) = (X x_i B) x_i A."""
    rng = _rng(2)
    X = rng.random((4, 5, 6))
    A, B = rng.random((3, 4)), rng.random((2, 5))
    lhs = oracle.nmode(oracle.nmode(X, 0, A), 1, B)
    rhs = oracle.nmode(oracle.nmode(X, 1, B), 0, A)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)
    P, Q = rng.random((3, 2)), rng.random((2, 6))
    np.testing.assert_allclose(oracle.nmode(X, 2, P @ Q), oracle.nmode(oracle.nmode(X, 2, Q), 2, P),
                               rtol=1e-13)


def test_unfolding_property():
    """unfold_i(Y x_1 A1 x_2 A2 x_3 A3) = A_i unfold_i(Y x_j A_j x_k A_k) (Appendix A)."""
    rng = _rng(3)
    Y = rng.random((2, 3, 4))
    A = [rng.random((5, 2)), rng.random((4, 3)), rng.random((6, 4))]
    X = oracle.tucker_full(Y, A)
    for i in range(3):
        part = Y
        for j in range(3):
            if j != i:
                part = oracle.nmode(part, j, A[j])
        lhs = np.moveaxis(X, i, 0).reshape(X.shape[i], -1)
        rhs = A[i] @ np.moveaxis(part, i, 0).reshape(part.shape[i], -1)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-13)


# --------------------------------------------------------------------------- printed examples
def test_ex2_all_ones_from_rank2_core():
    e = examples()["ex2_rank_not_preserved"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    G = fold(e["G_unfold1"], 0, e["core_dims"])
    assert np.array_equal(oracle.nmode(G, 0, arr(e["M1"])), X)
    assert np.array_equal(oracle.ttm_t(G, 0, arr(e["M1"]).T), X)


def test_ex1_multirank_from_unfoldings():
    e = examples()["ex1_real_minTD_not_cpd"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    ranks = [np.linalg.matrix_rank(np.moveaxis(X, n, 0).reshape(2, -1)) for n in range(3)]
    assert ranks == e["multirank"]


def test_ex3_unfoldings_and_real_tucker():
    e = examples()["ex3_not_in_cones"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    assert np.array_equal(fold(e["X_unfold2"], 1, e["dims"]), X)
    assert np.array_equal(fold(e["X_unfold3"], 2, e["dims"]), X)
    G = fold(e["G_unfold1"], 0, e["core_dims"])
    assert np.array_equal(oracle.tucker_full(G, [arr(e["W1"]), arr(e["W2"]), arr(e["W3"])]), X)


def test_ex4_unfoldings_and_exact_factorizations():
    e = examples()["ex4_no_minimal_nntd"]
    dims = e["dims"]
    X = fold(e["X_unfold1"], 0, dims)
    assert np.array_equal(fold(e["X_unfold2"], 1, dims), X)
    assert np.array_equal(fold(e["X_unfold3"], 2, dims), X)
    assert np.array_equal(arr(e["W2"]) @ arr(e["H2"]), arr(e["X_unfold2"]))
    assert np.array_equal(arr(e["W"]) @ arr(e["H_unfold1"]), arr(e["X_unfold1"]))
    H = fold(e["H_unfold1"], 0, e["H_dims"])
    assert np.array_equal(fold(e["H_unfold2"], 1, e["H_dims"]), H)
    assert np.array_equal(oracle.tucker_full(H, [arr(e["W"]), np.eye(4), np.eye(3)]), X)


def test_ex5_cp_and_tucker_reconstructions():
    e = examples()["ex5_rank_not_preserved_nn"]
    X = oracle.cp_full([arr(e["A1"]), arr(e["A2"]), arr(e["A3"])])
    assert np.array_equal(fold(e["X_unfold1"], 0, e["dims"]), X)
    G = fold(e["G_unfold1"], 0, e["core_dims"])
    assert np.array_equal(oracle.tucker_full(G, [arr(e["F1"]), np.eye(4), np.eye(4)]), X)


def test_ex6_cp_and_two_minimal_nntds():
    e = examples()["ex6_not_every_minimal_preserves"]
    X = fold_ex6(e["X_display"], e["dims"])
    assert np.array_equal(oracle.cp_full([arr(e["A1"]), arr(e["A2"]), arr(e["A3"])]), X)
    G1 = fold_ex6(e["G1_display"], e["core_dims"])
    G2 = fold_ex6(e["G2_display"], e["core_dims"])
    assert np.array_equal(oracle.tucker_full(G1, [arr(e["F1_1"]), arr(e["F1_2"]), arr(e["F1_3"])]), X)
    assert np.array_equal(oracle.tucker_full(G2, [arr(e["F2_1"]), arr(e["F2_2"]), arr(e["F2_3"])]), X)


def test_lift_is_the_substitution_of_the_core_cp():
    """G = cp(B)  =>  G x {A} = cp(A_n B_n) (Section 2.1, lemma proof), exact on integers."""
    e = examples()["ex6_not_every_minimal_preserves"]
    rng = _rng(4)
    A = [arr(e["F1_1"]), arr(e["F1_2"]), arr(e["F1_3"])]
    B = [rng.integers(0, 4, size=(a.shape[1], 3)).astype(float) for a in A]
    lhs = oracle.tucker_full(oracle.cp_full(B), A)
    rhs = oracle.cp_full(oracle.lift(A, B))
    assert np.array_equal(lhs, rhs)
    for a, b, c in zip(A, B, oracle.lift(A, B)):
        assert np.array_equal(c, a @ b)


# --------------------------------------------------------------------------- MU fixed points
def test_tucker_mu_fixed_point_at_exact_integer_factorization():
    """At an exact nonnegative factorization num = den exactly, so a sweep changes nothing."""
    e = examples()["ex4_no_minimal_nntd"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    H = fold(e["H_unfold1"], 0, e["H_dims"])
    A0 = [arr(e["W"]), np.eye(4), np.eye(3)]
    G, A, clips, _ = oracle.nntucker(X, H, A0, 3)
    assert np.array_equal(G, H)
    for a, a0 in zip(A, A0):
        assert np.array_equal(a, a0)
    e5 = examples()["ex5_rank_not_preserved_nn"]
    X5 = oracle.cp_full([arr(e5["A1"]), arr(e5["A2"]), arr(e5["A3"])])
    G5 = fold(e5["G_unfold1"], 0, e5["core_dims"])
    A5 = [arr(e5["F1"]), np.eye(4), np.eye(4)]
    G, A, _, _ = oracle.nntucker(X5, G5, A5, 2)
    assert np.array_equal(G, G5) and all(np.array_equal(a, b) for a, b in zip(A, A5))


def test_cp_mu_fixed_point_at_exact_cp():
    e = examples()["ex5_rank_not_preserved_nn"]
    B0 = [arr(e["A1"]), arr(e["A2"]), arr(e["A3"])]
    X = oracle.cp_full(B0)
    B, _, _ = oracle.nncp(X, B0, 3)
    assert all(np.array_equal(b, b0) for b, b0 in zip(B, B0))
    e4 = examples()["ex4_no_minimal_nntd"]
    V = arr(e4["X_unfold1"])
    B, _, _ = oracle.nncp(V, [arr(e4["W"]), arr(e4["H_unfold1"]).T], 3)
    assert np.array_equal(B[0], arr(e4["W"])) and np.array_equal(B[1], arr(e4["H_unfold1"]).T)


# --------------------------------------------------------------------------- textbook cases
def test_two_way_nncp_is_lee_seung_nmf():
    """For d = 2 the CP multiplicative update is the Lee-Seung NMF update (Appendix B):
    W <- W * (V H^T) / (W H H^T), then H <- H * (W^T V) / (W^T W H), with B_1 = W, B_2 = H^T."""
    rng = _rng(5)
    V = rng.random((7, 9))
    W, H = rng.random((7, 3)), rng.random((3, 9))
    B, _, _ = oracle.nncp(V, [W, H.T], 6)
    for _ in range(6):
        W = W * (V @ H.T) / (W @ H @ H.T)
        H = H * (W.T @ V) / (W.T @ W @ H)
    np.testing.assert_allclose(B[0], W, rtol=1e-12)
    np.testing.assert_allclose(B[1], H.T, rtol=1e-12)


def test_mttkrp_matches_brute_force():
    rng = _rng(6)
    T = rng.random((3, 4, 2, 3))
    B = [rng.random((s, 2)) for s in T.shape]
    for n in range(4):
        M = np.zeros((T.shape[n], 2))
        for idx in np.ndindex(*T.shape):
            for rho in range(2):
                p = T[idx]
                for k in range(4):
                    if k != n:
                        p *= B[k][idx[k], rho]
                M[idx[n], rho] += p
        np.testing.assert_allclose(oracle.mttkrp(T, n, B), M, rtol=1e-13)


def test_tucker_full_and_residual_match_brute_force():
    rng = _rng(7)
    G = rng.random((2, 3, 2))
    A = [rng.random((3, 2)), rng.random((4, 3)), rng.random((2, 2))]
    Xh = np.zeros((3, 4, 2))
    for i, j, k in np.ndindex(3, 4, 2):
        for a, b, c in np.ndindex(2, 3, 2):
            Xh[i, j, k] += G[a, b, c] * A[0][i, a] * A[1][j, b] * A[2][k, c]
    np.testing.assert_allclose(oracle.tucker_full(G, A), Xh, rtol=1e-14)
    X = rng.random((3, 4, 2))
    ref = np.sqrt(((X - Xh) ** 2).sum() / (X ** 2).sum())
    assert abs(oracle.tucker_rel_residual(X, G, A) - ref) <= 1e-14 * ref
    C = [rng.random((s, 3)) for s in (3, 4, 2)]
    Xc = np.zeros((3, 4, 2))
    for i, j, k in np.ndindex(3, 4, 2):
        Xc[i, j, k] = sum(C[0][i, r] * C[1][j, r] * C[2][k, r] for r in range(3))
    refc = np.sqrt(((X - Xc) ** 2).sum() / (X ** 2).sum())
    assert abs(oracle.cp_rel_residual(X, C) - refc) <= 1e-14 * refc


# --------------------------------------------------------------------------- gradients
def _loss(X, G, A):
    return 0.5 * oracle.tucker_rel_residual(X, G, A) ** 2 * oracle.sumsq(X)


def test_gradient_matches_central_differences():
    rng = _rng(8)
    X = rng.random((6, 5, 4))
    G = rng.random((3, 2, 2))
    A = [rng.random((6, 3)), rng.random((5, 2)), rng.random((4, 2))]
    L, gG, gA = oracle.tucker_grad(X, G, A)
    assert abs(L - _loss(X, G, A)) <= 1e-12 * L
    for (blk, idx) in [(0, (2, 1)), (1, (4, 0)), (2, (1, 1)), ("G", (1, 0, 1)), ("G", (2, 1, 0))]:
        if blk == "G":
            theta, g = G, gG[idx]
        else:
            theta, g = A[blk], gA[blk][idx]
        h = 1e-6 * max(1.0, abs(theta[idx]))
        old = theta[idx]
        theta[idx] = old + h
        lp = _loss(X, G, A)
        theta[idx] = old - h
        lm = _loss(X, G, A)
        theta[idx] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (blk, idx, fd, g)


def test_mu_numerator_denominator_difference_is_gradient():
    """den - num of every block equals the gradient computed from the explicit residual."""
    rng = _rng(9)
    X = rng.random((5, 6, 4, 3))
    G = rng.random((2, 3, 2, 2))
    A = [rng.random((s, r)) for s, r in zip(X.shape, G.shape)]
    num, den, numG, denG = oracle.tucker_numden(X, G, A)
    _, gG, gA = oracle.tucker_grad(X, G, A)
    for n in range(4):
        np.testing.assert_allclose(den[n] - num[n], gA[n], rtol=1e-9, atol=1e-10 * np.abs(num[n]).max())
    np.testing.assert_allclose(denG - numG, gG, rtol=1e-9, atol=1e-10 * np.abs(numG).max())


# --------------------------------------------------------------------------- MU invariants
@pytest.mark.parametrize("dims,ranks", [((10, 9, 8), (3, 4, 2)), ((6, 5, 4, 3), (2, 3, 2, 2)),
                                        ((5, 4, 3, 3, 2), (2, 2, 2, 2, 2))])
def test_mu_nonnegative_and_monotone(dims, ranks):
    X, _ = synth.planted_tensor(11, dims, 3, dtype="f64")
    G0 = synth.init_core(11, ranks, dtype=np.float64)
    A0 = synth.init_factors(11, dims, ranks, dtype=np.float64)
    G, A, clips, f = oracle.nntucker(X, G0, A0, 40, history=True)
    assert clips == 0
    assert (G >= 0).all() and all((a >= 0).all() for a in A)
    f0 = 0.5 * oracle.tucker_rel_residual(X, G0, A0) ** 2 * oracle.sumsq(X)
    seq = np.concatenate([[f0], f])
    assert (np.diff(seq) <= 1e-12 * f0).all()
    assert seq[-1] < 0.5 * seq[0]


def test_nncp_monotone_and_nonnegative():
    rng = _rng(12)
    T = oracle.cp_full([rng.random((5, 3)), rng.random((4, 3)), rng.random((6, 3))]) + 1e-3 * rng.random((5, 4, 6))
    B0 = synth.init_cp_factors(12, T.shape, 3, dtype=np.float64)
    B, clips, f = oracle.nncp(T, B0, 50, history=True)
    assert clips == 0 and all((b >= 0).all() for b in B)
    assert (np.diff(f) <= 1e-12 * f[0]).all()


def test_scale_equivariance():
    """X -> cX with G0 -> cG0 leaves every factor iterate unchanged and scales G by c."""
    X, _ = synth.planted_tensor(13, (7, 6, 5), 2, dtype="f64")
    G0 = synth.init_core(13, (2, 3, 2), dtype=np.float64)
    A0 = synth.init_factors(13, X.shape, (2, 3, 2), dtype=np.float64)
    G1, A1, _, _ = oracle.nntucker(X, G0, A0, 5)
    G2, A2, _, _ = oracle.nntucker(4.0 * X, 4.0 * G0, A0, 5)
    assert np.array_equal(G2, 4.0 * G1)
    assert all(np.array_equal(a, b) for a, b in zip(A1, A2))


def test_zero_init_column_hits_eps_guard():
    X, _ = synth.planted_tensor(14, (6, 5, 4), 2, dtype="f64")
    G0 = synth.init_core(14, (2, 2, 2), dtype=np.float64)
    A0 = synth.init_factors(14, X.shape, (2, 2, 2), dtype=np.float64)
    A0[1][:, 1] = 0.0
    G, A, clips, _ = oracle.nntucker(X, G0, A0, 3)
    assert clips > 0
    assert np.isfinite(G).all() and all(np.isfinite(a).all() and (a >= 0).all() for a in A)
    assert (A[1][:, 1] == 0).all()


def test_zero_iterations_returns_init():
    X, _ = synth.planted_tensor(15, (4, 4, 4), 2, dtype="f64")
    G0 = synth.init_core(15, (2, 2, 2), dtype=np.float64)
    A0 = synth.init_factors(15, X.shape, (2, 2, 2), dtype=np.float64)
    G, A, clips, _ = oracle.nntucker(X, G0, A0, 0)
    assert np.array_equal(G, G0) and clips == 0


def test_multirank_may_exceed_dims():
    """Section 4.2 fits multirank [5,5,5] to a 4x4x4 tensor; the update stays well defined."""
    e = examples()["ex5_rank_not_preserved_nn"]
    X = oracle.cp_full([arr(e["A1"]), arr(e["A2"]), arr(e["A3"])])
    G0 = synth.init_core(16, (5, 5, 5), dtype=np.float64)
    A0 = synth.init_factors(16, X.shape, (5, 5, 5), dtype=np.float64)
    G, A, clips, f = oracle.nntucker(X, G0, A0, 30, history=True)
    assert clips == 0 and (np.diff(f) <= 1e-12 * f[0]).all()


# --------------------------------------------------------------------------- recovery
def test_planted_recovery_through_tucker_core():
    """Sparse nonnegative planted CP (rank preserved to the core), multirank = R, zero noise:
    Algorithm 1 recovers the planted components (Section 4.1 scores)."""
    dims, R = (8, 8, 8), 2
    X, planted = synth.planted_tensor(21, dims, R, zero_prob=0.5, noise=0.0, dtype="f64")
    G0 = synth.init_core(21, (R,) * 3, dtype=np.float64)
    A0 = synth.init_factors(21, dims, (R,) * 3, dtype=np.float64)
    G, A, _, _ = oracle.nntucker(X, G0, A0, 5000)
    tucker_rel = oracle.tucker_rel_residual(X, G, A)
    assert tucker_rel < 1e-3
    best = None
    for j in range(8):
        B0 = synth.init_cp_factors(21, G.shape, R, restart=j, dtype=np.float64)
        B, _, _ = oracle.nncp(G, B0, 5000)
        C = oracle.lift(A, B)
        rel = oracle.cp_rel_residual(X, C)
        if best is None or rel < best[0]:
            best = (rel, C)
    rel, C = best
    assert rel <= tucker_rel + 1e-3
    assert oracle.mean_congruence(C, planted) >= 0.999


def test_gradient_finite_differences_16cubed_core_4cubed():
    """The adjoint workload's FD instance: 16^3 planted data, core 4^3, FP64 central differences."""
    X, _ = synth.planted_tensor(4, (16, 16, 16), 12, zero_prob=0.3, noise=0.0, dtype="f64")
    G = synth.init_core(4, (4, 4, 4), dtype=np.float64)
    A = synth.init_factors(4, (16, 16, 16), (4, 4, 4), dtype=np.float64)
    _, gG, gA = oracle.tucker_grad(X, G, A)
    rng = _rng(40)
    for _ in range(6):
        blk = int(rng.integers(0, 4))
        theta = G if blk == 3 else A[blk]
        idx = tuple(int(rng.integers(0, s)) for s in theta.shape)
        g = gG[idx] if blk == 3 else gA[blk][idx]
        h = 1e-6 * max(1.0, abs(theta[idx]))
        old = theta[idx]
        theta[idx] = old + h
        lp = _loss(X, G, A)
        theta[idx] = old - h
        lm = _loss(X, G, A)
        theta[idx] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (blk, idx, fd, g)


# --------------------------------------------------------------------------- Algorithm 2
def _lee_seung(V, W, H, iters):
    """Textbook Lee-Seung Frobenius NMF sweeps, W first, then H (written out here)."""
    for _ in range(iters):
        W = W * (V @ H.T) / (W @ H @ H.T)
        H = H * (W.T @ V) / (W.T @ W @ H)
    return W, H


def test_nmf_is_lee_seung():
    rng = _rng(21)
    V = rng.random((11, 4))
    W0, H0 = rng.random((11, 6)), rng.random((6, 4))
    W, H, clips = oracle.nmf(V, W0, H0, 7)
    We, He = _lee_seung(V, W0, H0, 7)
    assert clips == 0
    np.testing.assert_allclose(W, We, rtol=1e-12)
    np.testing.assert_allclose(H, He, rtol=1e-12)


def test_alg2_is_nncp_of_x_then_nmf_of_each_factor():
    """Algorithm 2: nnCP of X first, then an NMF of each fitted CP factor (not of its initial
    value), then the lift C_n = F_n B_n; the NMF sweeps here are the explicit textbook loop."""
    rng = _rng(22)
    X = rng.random((5, 6, 4))
    r, m = 3, (4, 2, 3)
    B0 = [rng.random((n, r)) for n in X.shape]
    F0 = [rng.random((X.shape[k], m[k])) for k in range(3)]
    H0 = [rng.random((m[k], r)) for k in range(3)]
    out = oracle.nncandelinc_alg2(X, B0, F0, H0, 9, 5)
    Acp, _, _ = oracle.nncp(X, B0, 9)
    for k in range(3):
        np.testing.assert_array_equal(out["Acp"][k], Acp[k])
        We, He = _lee_seung(Acp[k], F0[k], H0[k], 5)
        np.testing.assert_allclose(out["F"][k], We, rtol=1e-12)
        np.testing.assert_allclose(out["B"][k], He, rtol=1e-12)
        np.testing.assert_allclose(out["C"][k], We @ He, rtol=1e-12)
    Xhat = np.einsum("ir,jr,kr->ijk", *out["C"])
    assert abs(out["cp_rel"] - np.linalg.norm(X - Xhat) / np.linalg.norm(X)) <= 1e-12


def test_alg2_fixed_point_at_exact_integer_factorizations():
    """X = cp(F_n B_n) with integer F_n, B_n: starting Algorithm 2 at (F_n B_n, F_n, B_n) every
    multiplicative ratio is exactly 1, so nothing moves and the lifted model is exact."""
    rng = _rng(23)
    dims, m, r = (4, 5, 3), (3, 2, 3), 2
    F = [rng.integers(1, 4, (dims[k], m[k])).astype(np.float64) for k in range(3)]
    B = [rng.integers(1, 4, (m[k], r)).astype(np.float64) for k in range(3)]
    A = [f @ b for f, b in zip(F, B)]
    X = oracle.cp_full(A)
    out = oracle.nncandelinc_alg2(X, A, F, B, 3, 3)
    for k in range(3):
        assert np.array_equal(out["Acp"][k], A[k])
        assert np.array_equal(out["F"][k], F[k])
        assert np.array_equal(out["B"][k], B[k])
    assert out["cp_rel"] == 0.0 and out["clips"] == 0


def test_mean_congruence_brute_force_and_invariances():
    """Mean congruence (Section 4.1 scoring): 1 for a model compared with itself, invariant
    under a permutation of its components and under a positive rescaling of a factor column;
    brute force over all matchings written out here for a random pair."""
    rng = _rng(24)
    P = [rng.random((4, 3)) for _ in range(3)]
    assert abs(oracle.mean_congruence(P, P) - 1.0) <= 1e-14
    perm = [2, 0, 1]
    Pp = [p[:, perm] * np.array([1.0, 3.0, 0.5]) for p in P]
    assert abs(oracle.mean_congruence(P, Pp) - 1.0) <= 1e-14
    Q = [rng.random((4, 3)) for _ in range(3)]
    best = -1.0
    for pm in itertools.permutations(range(3)):
        s = 0.0
        for i in range(3):
            c = 1.0
            for p, q in zip(P, Q):
                a, b = p[:, i], q[:, pm[i]]
                c *= a @ b / np.sqrt((a @ a) * (b @ b))
            s += c
        best = max(best, s / 3)
    assert abs(oracle.mean_congruence(P, Q) - best) <= 1e-14


def test_restart_fit_exact_fixed_points_of_the_example():
    """The Section 4.2 tensor (the 4x4x4 example with unique nnCPD): its exact factorizations are
    fixed points of both algorithms (relative error 0, congruence 1)."""
    e = examples()["ex5_rank_not_preserved_nn"]
    A = [arr(e["A1"]), arr(e["A2"]), arr(e["A3"])]
    X = oracle.cp_full(A)
    D = np.zeros((4, 4, 4))
    for i in range(4):
        D[i, i, i] = 1.0
    I4 = np.eye(4)
    rel, cong, C = oracle.restart_fit(X, 1, A + [D] + [I4] * 3, 20, 20, truth=A)
    assert rel == 0.0 and abs(cong - 1.0) <= 1e-14 and all(np.array_equal(c, a) for c, a in zip(C, A))
    rel, cong, C = oracle.restart_fit(X, 2, A + A + [I4] * 3, 20, 20, truth=A)
    assert rel == 0.0 and abs(cong - 1.0) <= 1e-14 and all(np.array_equal(c, a) for c, a in zip(C, A))
