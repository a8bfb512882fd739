"""Python access to the FP64 C oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the benchmark's
CPU-baseline leg.  The GPU library never imports or links it, and it never imports the
GPU library.  All arrays are float64, C-contiguous, row-major.

Function names follow the paper's notation: X the data tensor, A_n (= F^(n)) the Tucker
factors, G the core, B_n the CP factors of the core, C_n = A_n B_n the lifted factors.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dpp = ctypes.POINTER(_dp)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.orc_nmode.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.c_int, _dp, ctypes.c_int64, _dp]
        L.orc_ttm_t.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.c_int, _dp, ctypes.c_int64, _dp]
        L.orc_contract_except.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _dp, ctypes.c_int, _dp]
        L.orc_gram.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, _dp]
        L.orc_tucker_full.argtypes = [ctypes.c_int, _i64p, _i64p, _dp, _dpp, _dp]
        L.orc_cp_full.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _dpp, _dp]
        L.orc_sumsq.argtypes = [_dp, ctypes.c_int64]
        L.orc_sumsq.restype = ctypes.c_double
        L.orc_tucker_sq_residual.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _dp, _dpp]
        L.orc_tucker_sq_residual.restype = ctypes.c_double
        L.orc_cp_sq_residual.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.c_int64, _dpp]
        L.orc_cp_sq_residual.restype = ctypes.c_double
        L.orc_nntucker.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, ctypes.c_int, ctypes.c_double,
                                   _dp, _dpp, _dp]
        L.orc_nntucker.restype = ctypes.c_longlong
        L.orc_mttkrp.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int64, _dpp, _dp]
        L.orc_nncp.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.c_int64, ctypes.c_int,
                               ctypes.c_double, _dpp, _dp]
        L.orc_nncp.restype = ctypes.c_longlong
        L.orc_lift.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int64, _dpp, _dpp, _dpp]
        L.orc_tucker_grad.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _dp, _dpp, _dp, _dpp]
        L.orc_tucker_grad.restype = ctypes.c_double
        L.orc_tucker_numden.argtypes = [ctypes.c_int, _i64p, _dp, _i64p, _dp, _dpp, _dpp, _dpp,
                                        _dp, _dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _dims(shape):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return arr


def _ptrs(mats):
    arr = (_dp * len(mats))(*[_p(m) for m in mats])
    return arr


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def nmode(X, n: int, M) -> np.ndarray:
    """X x_n M (Appendix A): out[.., i, ..] = sum_l X[.., l, ..] M[i, l]."""
    X, M = _f64(X), _f64(M)
    assert M.ndim == 2 and M.shape[1] == X.shape[n]
    shape = list(X.shape)
    shape[n] = M.shape[0]
    out = np.empty(shape, dtype=np.float64)
    lib().orc_nmode(X.ndim, _dims(X.shape), _p(X), n, _p(M), M.shape[0], _p(out))
    return out


def ttm_t(X, n: int, A) -> np.ndarray:
    """X x_n A^T for a factor A of shape (dims[n], R)."""
    X, A = _f64(X), _f64(A)
    assert A.ndim == 2 and A.shape[0] == X.shape[n]
    shape = list(X.shape)
    shape[n] = A.shape[1]
    out = np.empty(shape, dtype=np.float64)
    lib().orc_ttm_t(X.ndim, _dims(X.shape), _p(X), n, _p(A), A.shape[1], _p(out))
    return out


def contract_except(U, V, n: int) -> np.ndarray:
    """out[i, j] = sum over every index but mode n of U[.., i, ..] V[.., j, ..]."""
    U, V = _f64(U), _f64(V)
    out = np.empty((U.shape[n], V.shape[n]), dtype=np.float64)
    lib().orc_contract_except(U.ndim, _dims(U.shape), _p(U), _dims(V.shape), _p(V), n, _p(out))
    return out


def gram(A) -> np.ndarray:
    A = _f64(A)
    S = np.empty((A.shape[1], A.shape[1]), dtype=np.float64)
    lib().orc_gram(_p(A), A.shape[0], A.shape[1], _p(S))
    return S


def tucker_full(G, A) -> np.ndarray:
    """G x_1 A_1 x_2 ... x_d A_d."""
    G = _f64(G)
    A = [_f64(a) for a in A]
    dims = [a.shape[0] for a in A]
    out = np.empty(dims, dtype=np.float64)
    lib().orc_tucker_full(G.ndim, _dims(dims), _dims(G.shape), _p(G), _ptrs(A), _p(out))
    return out


def cp_full(C) -> np.ndarray:
    """sum_rho outer(C_1[:, rho], ..., C_d[:, rho])."""
    C = [_f64(c) for c in C]
    dims = [c.shape[0] for c in C]
    out = np.empty(dims, dtype=np.float64)
    lib().orc_cp_full(len(C), _dims(dims), C[0].shape[1], _ptrs(C), _p(out))
    return out


def sumsq(X) -> float:
    X = _f64(X)
    return float(lib().orc_sumsq(_p(X), X.size))


def tucker_rel_residual(X, G, A) -> float:
    """||X - G x {A}||_F / ||X||_F (Section 4.1 relative error)."""
    X, G = _f64(X), _f64(G)
    A = [_f64(a) for a in A]
    s = lib().orc_tucker_sq_residual(X.ndim, _dims(X.shape), _p(X), _dims(G.shape), _p(G), _ptrs(A))
    return float(np.sqrt(s / sumsq(X)))


def cp_rel_residual(X, C) -> float:
    X = _f64(X)
    C = [_f64(c) for c in C]
    s = lib().orc_cp_sq_residual(X.ndim, _dims(X.shape), _p(X), C[0].shape[1], _ptrs(C))
    return float(np.sqrt(s / sumsq(X)))


def nntucker(X, G0, A0, iters: int, eps: float = 1e-12, history: bool = False):
    """nnTucker by multiplicative updates; returns (G, [A_n], clips, f_hist or None)."""
    X = _f64(X)
    G = _f64(G0).copy()
    A = [_f64(a).copy() for a in A0]
    d = X.ndim
    R = [a.shape[1] for a in A]
    assert tuple(G.shape) == tuple(R)
    hist = np.zeros(max(iters, 1), dtype=np.float64) if history else None
    clips = lib().orc_nntucker(d, _dims(X.shape), _p(X), _dims(R), int(iters), float(eps), _p(G),
                               _ptrs(A), _p(hist) if history else None)
    return G, A, int(clips), (hist[:iters] if history else None)


def mttkrp(T, n: int, B) -> np.ndarray:
    T = _f64(T)
    B = [_f64(b) for b in B]
    r = B[0].shape[1]
    out = np.empty((T.shape[n], r), dtype=np.float64)
    lib().orc_mttkrp(T.ndim, _dims(T.shape), _p(T), n, r, _ptrs(B), _p(out))
    return out


def nncp(T, B0, iters: int, eps: float = 1e-12, history: bool = False):
    """nnCP of T by multiplicative updates; returns ([B_n], clips, f_hist or None)."""
    T = _f64(T)
    B = [_f64(b).copy() for b in B0]
    r = B[0].shape[1]
    hist = np.zeros(max(iters, 1), dtype=np.float64) if history else None
    clips = lib().orc_nncp(T.ndim, _dims(T.shape), _p(T), r, int(iters), float(eps), _ptrs(B),
                           _p(hist) if history else None)
    return B, int(clips), (hist[:iters] if history else None)


def lift(A, B):
    """C_n = A_n B_n (substitution of the core's CP into the Tucker model)."""
    A = [_f64(a) for a in A]
    B = [_f64(b) for b in B]
    r = B[0].shape[1]
    dims = [a.shape[0] for a in A]
    ranks = [a.shape[1] for a in A]
    C = [np.empty((dims[k], r), dtype=np.float64) for k in range(len(A))]
    lib().orc_lift(len(A), _dims(dims), _dims(ranks), r, _ptrs(A), _ptrs(B), _ptrs(C))
    return C


def tucker_grad(X, G, A):
    """(L, dL/dG, [dL/dA_n]) for L = 0.5 ||X - G x {A}||^2, from the explicit residual."""
    X, G = _f64(X), _f64(G)
    A = [_f64(a) for a in A]
    gG = np.empty_like(G)
    gA = [np.empty_like(a) for a in A]
    L = lib().orc_tucker_grad(X.ndim, _dims(X.shape), _p(X), _dims(G.shape), _p(G), _ptrs(A),
                              _p(gG), _ptrs(gA))
    return float(L), gG, gA


def tucker_numden(X, G, A):
    """Block numerators/denominators at a fixed point: ([num_n], [den_n], num_G, den_G)."""
    X, G = _f64(X), _f64(G)
    A = [_f64(a) for a in A]
    num = [np.empty_like(a) for a in A]
    den = [np.empty_like(a) for a in A]
    numG, denG = np.empty_like(G), np.empty_like(G)
    lib().orc_tucker_numden(X.ndim, _dims(X.shape), _p(X), _dims(G.shape), _p(G), _ptrs(A),
                            _ptrs(num), _ptrs(den), _p(numG), _p(denG))
    return num, den, numG, denG


def mean_congruence(P, Q) -> float:
    """Mean congruence of two rank-r CP models after the best matching of components
    (Section 4.1 scoring): the congruence of two rank-one tensors is the product over
    modes of the cosines between their factor vectors.  Brute force over permutations."""
    import itertools
    P = [_f64(p) for p in P]
    Q = [_f64(q) for q in Q]
    r = P[0].shape[1]
    assert r <= 8 and all(q.shape[1] == r for q in Q)
    cos = np.ones((r, r))
    for p, q in zip(P, Q):
        pn = p / np.linalg.norm(p, axis=0, keepdims=True)
        qn = q / np.linalg.norm(q, axis=0, keepdims=True)
        cos *= pn.T @ qn
    best = max(np.mean([cos[i, perm[i]] for i in range(r)])
               for perm in itertools.permutations(range(r)))
    return float(best)


def nncandelinc(X, G0, A0, B0, tucker_iters: int, cp_iters: int, eps: float = 1e-12):
    """Algorithm 1 end to end: nnTucker, nnCP of the core, lift, residuals."""
    G, A, c1, _ = nntucker(X, G0, A0, tucker_iters, eps)
    B, c2, _ = nncp(G, B0, cp_iters, eps)
    C = lift(A, B)
    return dict(G=G, A=A, B=B, C=C, clips=c1 + c2,
                tucker_rel=tucker_rel_residual(X, G, A), cp_rel=cp_rel_residual(X, C))


def nmf(A, W0, H0, iters: int, eps: float = 1e-12):
    """NMF A ~ W H by Lee-Seung multiplicative updates (the NMF step of Algorithm 2): each
    sweep W <- W * (A H^T) / max(W H H^T, eps), then H <- H * (W^T A) / max(W^T W H, eps).
    These are the two-way nnCP updates with factors W and H^T, so the nnCP routine computes
    them.  Returns (W, H, clips)."""
    (W, Ht), clips, _ = nncp(A, [W0, _f64(H0).T.copy()], iters, eps)
    return W, Ht.T.copy(), clips


def nncandelinc_alg2(X, B0, F0, H0, cp_iters: int, nmf_iters: int, eps: float = 1e-12):
    """Algorithm 2 end to end: nnCP of X with initial factors B0 (dims[n] x r), then an NMF
    of each fitted factor A^(n) ~ F^(n) B^(n) from initial F0[n] (dims[n] x m_n) and
    H0[n] (m_n x r), the lift C_n = F^(n) B^(n) and the relative error of that model."""
    Acp, c1, _ = nncp(X, B0, cp_iters, eps)
    F, B, c2 = [], [], 0
    for n in range(len(Acp)):
        f, b, c = nmf(Acp[n], F0[n], H0[n], nmf_iters, eps)
        F.append(f)
        B.append(b)
        c2 += c
    C = lift(F, B)
    return dict(Acp=Acp, F=F, B=B, C=C, clips=c1 + c2, cp_x_rel=cp_rel_residual(X, Acp),
                cp_rel=cp_rel_residual(X, C))


def restart_fit(X, alg: int, parts, outer: int, inner: int, truth=None, eps: float = 1e-12):
    """One start of the Section 4.2 study: Algorithm 1 (parts = A_0..A_2, G, B_0..B_2) or
    Algorithm 2 (parts = B_0..B_2, W_0..W_2, H_0..H_2) with `outer` sweeps of the first fit and
    `inner` of the second; returns (relative error of the lifted CP, mean congruence with
    `truth` or None, lifted factors)."""
    if alg == 1:
        out = nncandelinc(X, parts[3], parts[0:3], parts[4:7], outer, inner, eps)
    else:
        out = nncandelinc_alg2(X, parts[0:3], parts[3:6], parts[6:9], outer, inner, eps)
    C = out["C"]
    return out["cp_rel"], (mean_congruence(C, truth) if truth is not None else None), C


# ------------------------------------------------------------------ real-valued CANDELINC
# Section 2.2: a (minimal) Tucker decomposition of X, a CPD of its core, and the substitution
# of that CPD into the Tucker model, which gives a CPD of X with factors F^(i) A_G^(i).  The
# paper names no algorithm for either fit ("readily available tools", Section 4, beside the
# optimization problem nnCANDELINC without its constraints).  The reading taken here is
# alternating least squares for both, in the same Gauss-Seidel order as the nonnegative
# sweep (Tucker factors 1..d, then the core; CP factors 1..d).  Each block update is the exact
# minimizer of 0.5 ||X - model||_F^2 over that block with the others fixed, written with a
# dense solve (numpy.linalg.solve) as the library step.  After each Tucker factor's step the
# factor is replaced by the Q of its thin QR (R with a positive diagonal) and R is absorbed
# into the core: the model is unchanged, the factors stay orthonormal, so the core's CP fit
# measures the same error as the lifted CP fit of X.


def mode_solve(T, n: int, S) -> np.ndarray:
    """T x_n S^{-1} for a nonsingular S (R x R, R = T.shape[n]): every mode-n fibre of T
    replaced by the solution of S y = fibre."""
    T, S = _f64(T), _f64(S)
    assert S.shape == (T.shape[n], T.shape[n])
    moved = np.moveaxis(T, n, 0)
    sol = np.linalg.solve(S, moved.reshape(T.shape[n], -1))
    return np.ascontiguousarray(np.moveaxis(sol.reshape(moved.shape), 0, n))


def qr_pos(A):
    """Thin QR A = Q R with R upper triangular and its diagonal positive (unique for a full
    column rank A): numpy's Householder QR with the signs of R's rows fixed."""
    Q, R = np.linalg.qr(_f64(A))
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    return np.ascontiguousarray(Q * sg), np.ascontiguousarray(R * sg[:, None])


def tucker_ls_factor(X, G, A, n: int) -> np.ndarray:
    """Least-squares update of F^(n) (= A_n) with the core and the other factors fixed.
    Writing the model's mode-n unfolding as A_n G_(n) Z^T (Z the Kronecker product of the
    other factors), the minimizer is A_n = X_(n) Z G_(n)^T K_n^{-1} with
    X_(n) Z G_(n)^T = contraction of Y = X x_{k!=n} A_k^T with G over every mode but n, and
    K_n = G_(n) (Z^T Z) G_(n)^T = contraction of G x_{k!=n} S_k with G over every mode but n
    (S_k = A_k^T A_k)."""
    d = len(A)
    Y = _f64(X)
    H = _f64(G)
    for k in range(d):
        if k != n:
            Y = ttm_t(Y, k, A[k])
            H = nmode(H, k, gram(A[k]))
    num = contract_except(Y, G, n)
    K = contract_except(H, G, n)
    return np.ascontiguousarray(np.linalg.solve(K, num.T).T)


def tucker_ls_core(X, A) -> np.ndarray:
    """Least-squares update of the core with every factor fixed: the normal equations read
    G x_1 S_1 ... x_d S_d = X x_1 A_1^T ... x_d A_d^T, solved one mode at a time."""
    num = _f64(X)
    for k in range(len(A)):
        num = ttm_t(num, k, A[k])
    G = num
    for k in range(len(A)):
        G = mode_solve(G, k, gram(A[k]))
    return G


def tucker_ls(X, G0, A0, iters: int, history: bool = False):
    """Real Tucker fit by alternating least squares with orthonormalized factors; returns
    (G, [A_n], f_hist or None) with f_t = 0.5 ||X - G x {A}||_F^2 after sweep t.  The initial
    factors are orthonormalized first (A_n = Q R, A_n <- Q, G <- G x_n R): the same initial
    model, with well-conditioned least-squares systems from the first step on."""
    X = _f64(X)
    G = _f64(G0).copy()
    A = [_f64(a).copy() for a in A0]
    for n in range(len(A)):
        A[n], R = qr_pos(A[n])
        G = nmode(G, n, R)
    hist = []
    for _ in range(iters):
        for n in range(len(A)):
            A[n], R = qr_pos(tucker_ls_factor(X, G, A, n))
            G = nmode(G, n, R)
        G = tucker_ls_core(X, A)
        if history:
            hist.append(0.5 * tucker_rel_residual(X, G, A) ** 2 * sumsq(X))
    return G, A, (np.array(hist) if history else None)


def cp_ls_factor(T, B, n: int) -> np.ndarray:
    """Least-squares update of CP factor n with the others fixed: B_n = M_n H_n^{-1}, with
    M_n the MTTKRP of T with the other factors and H_n the Hadamard product of their Grams."""
    H = np.ones((B[0].shape[1], B[0].shape[1]))
    for k in range(len(B)):
        if k != n:
            H = H * gram(B[k])
    M = mttkrp(T, n, B)
    return np.ascontiguousarray(np.linalg.solve(H, M.T).T)


def cp_ls(T, B0, iters: int, history: bool = False):
    """Real CP fit of T by alternating least squares; returns ([B_n], f_hist or None)."""
    T = _f64(T)
    B = [_f64(b).copy() for b in B0]
    hist = []
    for _ in range(iters):
        for n in range(len(B)):
            B[n] = cp_ls_factor(T, B, n)
        if history:
            hist.append(0.5 * cp_rel_residual(T, B) ** 2 * sumsq(T))
    return B, (np.array(hist) if history else None)


def candelinc(X, G0, A0, B0, tucker_iters: int, cp_iters: int):
    """Real-valued CANDELINC end to end (Section 2.2): Tucker fit, CP fit of its core, lift
    C_n = F^(n) A_G^(n), residuals of the three models."""
    G, A, _ = tucker_ls(X, G0, A0, tucker_iters)
    B, _ = cp_ls(G, B0, cp_iters)
    C = lift(A, B)
    return dict(G=G, A=A, B=B, C=C, tucker_rel=tucker_rel_residual(X, G, A),
                core_rel=cp_rel_residual(G, B), cp_rel=cp_rel_residual(X, C))
