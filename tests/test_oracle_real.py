"""Pins of the real-valued CANDELINC oracle (Section 2.2: Tucker fit, CP fit of its core,
substitution) against what the paper and the mathematics fix: Example 3's real Tucker
factorization (its core holds a negative entry), block optimality checked with the
finite-difference-pinned gradient and with central differences of the CP loss, the
Eckart-Young optimum of the two-way case, exact recovery at exact multilinear rank and at
exact CP rank, the rank-deficient-factor scenario that motivates CANDELINC, and the
non-increasing objective of alternating least squares.
"""
import numpy as np
import pytest

import oracle
from tests.paper_fixtures import arr, examples, fold


def _rng(seed):
    return np.random.default_rng(seed)


def _loss(X, G, A):
    return 0.5 * oracle.tucker_rel_residual(X, G, A) ** 2 * oracle.sumsq(X)


def _cp_loss(T, B):
    return 0.5 * float(np.sum((T - oracle.cp_full(B)) ** 2))


# --------------------------------------------------------------------------- Example 3
def _ex3():
    e = examples()["ex3_not_in_cones"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    W = [arr(e["W1"]), arr(e["W2"]), arr(e["W3"])]
    G = fold(e["G_unfold1"], 0, e["core_dims"])
    return X, W, G


def test_ex3_core_step_gives_the_printed_real_core():
    """With the factors fixed at Example 3's full-column-rank W^(i), the core's least-squares
    step returns the unique core the paper prints, including its -1 entry (Section 3)."""
    X, W, G = _ex3()
    Gs = oracle.tucker_ls_core(X, W)
    np.testing.assert_allclose(Gs, G, rtol=0, atol=1e-13)
    assert Gs.min() < -0.5  # the entry that leaves the nonnegative cone


def test_ex3_exact_factorization_is_a_fixed_point():
    """At an exact factorization each least-squares factor step returns the factor itself;
    a whole sweep (with the orthonormalization) keeps the exact model."""
    X, W, G = _ex3()
    for n in range(3):
        np.testing.assert_allclose(oracle.tucker_ls_factor(X, G, W, n), W[n], rtol=0, atol=1e-12)
    G1, A1, _ = oracle.tucker_ls(X, G, W, 2)
    np.testing.assert_allclose(oracle.tucker_full(G1, A1), X, rtol=0, atol=1e-12)
    for a, w in zip(A1, W):
        np.testing.assert_allclose(a.T @ a, np.eye(a.shape[1]), rtol=0, atol=1e-13)
        np.testing.assert_allclose(a @ (a.T @ w), w, rtol=0, atol=1e-12)  # same column space


def test_ex3_from_a_random_start_reaches_an_exact_fit():
    """The example's tensor has multilinear rank (2, 2, 2): the Tucker fit at that multirank
    is exact, and its core spans the same real core up to invertible factors."""
    X, W, G = _ex3()
    rng = _rng(31)
    Gf, Af, _ = oracle.tucker_ls(X, rng.standard_normal((2, 2, 2)),
                                 [rng.standard_normal((3, 2)), rng.standard_normal((3, 2)),
                                  rng.standard_normal((2, 2))], 30)
    assert oracle.tucker_rel_residual(X, Gf, Af) <= 1e-12
    # same column spaces as W^(i): A_n = W_n Q_n with Q_n invertible
    for a, w in zip(Af, W):
        Q, *_ = np.linalg.lstsq(w, a, rcond=None)
        np.testing.assert_allclose(w @ Q, a, rtol=0, atol=1e-10)
        assert abs(np.linalg.det(Q)) > 1e-6


# --------------------------------------------------------------------------- block optimality
def test_factor_and_core_steps_zero_their_block_gradient():
    """Each least-squares step is the block minimizer: after it, the gradient of
    0.5 ||X - G x {A}||^2 with respect to that block (the FD-pinned oracle gradient) is zero,
    and a random perturbation of the block raises the loss."""
    rng = _rng(32)
    X = rng.standard_normal((6, 5, 4))
    G = rng.standard_normal((3, 2, 2))
    A = [rng.standard_normal((6, 3)), rng.standard_normal((5, 2)), rng.standard_normal((4, 2))]
    for n in range(3):
        A[n] = oracle.tucker_ls_factor(X, G, A, n)
        L, _, gA = oracle.tucker_grad(X, G, A)
        assert np.abs(gA[n]).max() <= 1e-10 * max(1.0, L), (n, np.abs(gA[n]).max())
        for _ in range(3):
            P = [a.copy() for a in A]
            P[n] = P[n] + 1e-3 * rng.standard_normal(P[n].shape)
            assert _loss(X, G, P) > L
    G = oracle.tucker_ls_core(X, A)
    L, gG, _ = oracle.tucker_grad(X, G, A)
    assert np.abs(gG).max() <= 1e-10 * max(1.0, L)
    assert _loss(X, G + 1e-3 * rng.standard_normal(G.shape), A) > L


def test_cp_factor_step_zeroes_central_difference_gradient():
    """After B_n's least-squares step, central differences of the CP loss vanish in B_n."""
    rng = _rng(33)
    T = rng.standard_normal((4, 3, 5))
    B = [rng.standard_normal((4, 2)), rng.standard_normal((3, 2)), rng.standard_normal((5, 2))]
    for n in range(3):
        B[n] = oracle.cp_ls_factor(T, B, n)
        for idx in np.ndindex(*B[n].shape):
            old = B[n][idx]
            h = 1e-6 * max(1.0, abs(old))
            B[n][idx] = old + h
            lp = _cp_loss(T, B)
            B[n][idx] = old - h
            lm = _cp_loss(T, B)
            B[n][idx] = old
            assert abs(lp - lm) / (2 * h) <= 1e-7, (n, idx)


def test_mode_solve_inverts_the_mode_product():
    rng = _rng(34)
    T = rng.standard_normal((3, 4, 5))
    for n in range(3):
        S = rng.standard_normal((T.shape[n], T.shape[n]))
        S = S @ S.T + np.eye(T.shape[n])
        np.testing.assert_allclose(oracle.nmode(oracle.mode_solve(T, n, S), n, S), T, rtol=0, atol=1e-12)


def test_qr_pos_factors_with_positive_diagonal():
    rng = _rng(44)
    A = rng.standard_normal((9, 4))
    Q, R = oracle.qr_pos(A)
    np.testing.assert_allclose(Q @ R, A, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(4), rtol=0, atol=1e-14)
    assert np.array_equal(R, np.triu(R)) and (np.diag(R) > 0).all()
    # R^T R is the Gram of A, whose Cholesky factor is unique
    np.testing.assert_allclose(R.T, np.linalg.cholesky(A.T @ A), rtol=0, atol=1e-12)


def test_sweep_keeps_factors_orthonormal_and_the_core_metric():
    """With orthonormal factors ||G x {A} - cp(B) x {A}|| = ||G - cp(B)||: the core's CP
    error equals the lifted CP error on the Tucker model."""
    rng = _rng(45)
    X = rng.standard_normal((7, 6, 5))
    G, A, _ = oracle.tucker_ls(X, rng.standard_normal((3, 3, 2)),
                               [rng.standard_normal((n, r)) for n, r in zip(X.shape, (3, 3, 2))], 3)
    for a in A:
        np.testing.assert_allclose(a.T @ a, np.eye(a.shape[1]), rtol=0, atol=1e-13)
    B = [rng.standard_normal((r, 2)) for r in G.shape]
    M = oracle.tucker_full(G, A)
    lhs = np.linalg.norm(M - oracle.cp_full(oracle.lift(A, B)))
    assert abs(lhs - np.linalg.norm(G - oracle.cp_full(B))) <= 1e-12 * lhs


def test_orthonormalization_leaves_the_model_sequence_unchanged():
    """The QR step only re-parametrizes the model: a sweep with it gives the same model as
    plain alternating least squares (same sets of reachable models in every block)."""
    rng = _rng(46)
    X = rng.standard_normal((6, 5, 4))
    G0 = rng.standard_normal((2, 3, 2))
    A0 = [rng.standard_normal((n, r)) for n, r in zip(X.shape, G0.shape)]
    G, A = G0.copy(), [a.copy() for a in A0]
    for _ in range(3):
        for n in range(3):
            A[n] = oracle.tucker_ls_factor(X, G, A, n)
        G = oracle.tucker_ls_core(X, A)
    Go, Ao, _ = oracle.tucker_ls(X, G0, A0, 3)
    np.testing.assert_allclose(oracle.tucker_full(Go, Ao), oracle.tucker_full(G, A), rtol=0, atol=1e-11)
    # zero sweeps: the orthonormalized initial factors carry the initial model
    Gz, Az, _ = oracle.tucker_ls(X, G0, A0, 0)
    np.testing.assert_allclose(oracle.tucker_full(Gz, Az), oracle.tucker_full(G0, A0), rtol=0, atol=1e-12)
    for a in Az:
        np.testing.assert_allclose(a.T @ a, np.eye(a.shape[1]), rtol=0, atol=1e-14)


# --------------------------------------------------------------------------- special cases
def test_two_way_fit_reaches_the_eckart_young_optimum():
    """At d = 2 the Tucker model G x_1 A_1 x_2 A_2 = A_1 G A_2^T is a rank-k matrix, and the
    best one leaves exactly the trailing singular values (Eckart-Young)."""
    rng = _rng(35)
    U, _ = np.linalg.qr(rng.standard_normal((12, 9)))
    V, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    s = np.array([9.0, 7.0, 5.0, 1.0, 0.8, 0.5, 0.3, 0.2, 0.1])
    X = U @ np.diag(s) @ V.T
    k = 3
    G, A, h = oracle.tucker_ls(X, rng.standard_normal((k, k)),
                               [rng.standard_normal((12, k)), rng.standard_normal((9, k))], 60, history=True)
    best = np.sqrt(np.sum(s[k:] ** 2) / np.sum(s ** 2))
    assert abs(oracle.tucker_rel_residual(X, G, A) - best) <= 1e-12
    assert np.isclose(h[-1], 0.5 * np.sum(s[k:] ** 2), rtol=1e-12)


@pytest.mark.parametrize("dims,ranks", [((7, 8, 5), (3, 4, 2)), ((5, 4, 6, 3), (2, 3, 2, 2))])
def test_exact_multilinear_rank_is_recovered(dims, ranks):
    rng = _rng(36 + len(dims))
    X = oracle.tucker_full(rng.standard_normal(ranks), [rng.standard_normal((n, r)) for n, r in zip(dims, ranks)])
    G, A, _ = oracle.tucker_ls(X, rng.standard_normal(ranks),
                               [rng.standard_normal((n, r)) for n, r in zip(dims, ranks)], 5)
    assert oracle.tucker_rel_residual(X, G, A) <= 1e-12


def test_full_multirank_core_step_is_exact():
    """With m_n = N_n every full-rank factor set spans the whole space, so the core step alone
    fits any tensor exactly."""
    rng = _rng(38)
    X = rng.standard_normal((4, 3, 5))
    A = [rng.standard_normal((n, n)) for n in X.shape]
    assert oracle.tucker_rel_residual(X, oracle.tucker_ls_core(X, A), A) <= 1e-13


def test_objective_non_increasing():
    rng = _rng(39)
    X = rng.standard_normal((8, 7, 6))
    _, _, h = oracle.tucker_ls(X, rng.standard_normal((3, 3, 3)),
                               [rng.standard_normal((n, 3)) for n in X.shape], 40, history=True)
    assert (np.diff(h) <= 1e-12 * h[0]).all()
    T = rng.standard_normal((5, 4, 3))
    _, hc = oracle.cp_ls(T, [rng.standard_normal((n, 3)) for n in T.shape], 60, history=True)
    assert (np.diff(hc) <= 1e-12 * hc[0]).all()


def test_two_way_cp_fit_is_exact_at_the_matrix_rank():
    """At d = 2 the CP model is a rank-r matrix factorization; a rank-r matrix is fitted
    exactly after one sweep from a generic start."""
    rng = _rng(40)
    M = rng.standard_normal((7, 2)) @ rng.standard_normal((2, 6))
    B, _ = oracle.cp_ls(M, [rng.standard_normal((7, 2)), rng.standard_normal((6, 2))], 2)
    assert oracle.cp_rel_residual(M, B) <= 1e-13


def test_cp_fit_recovers_an_exact_rank_three_tensor():
    rng = _rng(41)
    P = [rng.standard_normal((n, 3)) for n in (4, 5, 6)]
    T = oracle.cp_full(P)
    B, _ = oracle.cp_ls(T, [rng.standard_normal((n, 3)) for n in (4, 5, 6)], 300)
    assert oracle.cp_rel_residual(T, B) <= 1e-9
    assert oracle.mean_congruence(B, P) >= 1 - 1e-9


# --------------------------------------------------------------------------- CANDELINC end to end
def test_candelinc_recovers_a_cpd_with_a_rank_deficient_factor():
    """Section 2.2's scenario: a unique rank-4 CPD whose first factor has rank 3, so the first
    multilinear rank is 3 < 4.  Tucker at the minimal multirank (3, 4, 4), a rank-4 CP of the
    core and the substitution give back the CPD (Kruskal: 3 + 4 + 4 >= 2*4 + 2)."""
    rng = _rng(42)
    A1 = rng.standard_normal((9, 3))
    A1 = np.hstack([A1, A1 @ rng.standard_normal((3, 1))])
    P = [A1, rng.standard_normal((8, 4)), rng.standard_normal((7, 4))]
    X = oracle.cp_full(P)
    m = (3, 4, 4)
    assert [np.linalg.matrix_rank(np.moveaxis(X, n, 0).reshape(X.shape[n], -1)) for n in range(3)] == list(m)
    best = None
    for s in range(4):
        r2 = _rng(100 + s)
        out = oracle.candelinc(X, r2.standard_normal(m), [r2.standard_normal((n, k)) for n, k in zip(X.shape, m)],
                               [r2.standard_normal((k, 4)) for k in m], 10, 500)
        if best is None or out["cp_rel"] < best["cp_rel"]:
            best = out
    assert best["tucker_rel"] <= 1e-12
    assert best["cp_rel"] <= 1e-8 and abs(best["cp_rel"] - best["core_rel"]) <= 1e-12
    assert oracle.mean_congruence(best["C"], P) >= 1 - 1e-8
    for a, b, c in zip(best["A"], best["B"], best["C"]):
        np.testing.assert_allclose(c, a @ b, rtol=1e-14, atol=1e-14)


def test_lift_of_signed_factors_is_the_substitution():
    """G = cp(B) implies G x {A} = cp(A_n B_n) for real (signed) factors too (Section 2.1)."""
    rng = _rng(43)
    A = [rng.standard_normal((n, m)) for n, m in ((5, 3), (4, 2), (6, 3))]
    B = [rng.standard_normal((m, 4)) for m in (3, 2, 3)]
    np.testing.assert_allclose(oracle.tucker_full(oracle.cp_full(B), A), oracle.cp_full(oracle.lift(A, B)),
                               rtol=0, atol=1e-12)
