"""GPU parity of the rank-deficient study of Section 4.3 (generated 40^3 tensors of nonnegative
rank 5 with canonical multiranks [3, 4, 5], Algorithms 1 and 2 on each) against the FP64
oracle, tensor by tensor, and of the mean-congruence score."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import dev, host, need_gpu

pytestmark = pytest.mark.gpu

DIMS, RANKS, R = (40, 40, 40), (3, 4, 5), 5


@pytest.mark.parametrize("dims,r", [((7, 9, 5), 3), ((40, 40, 40), 5), ((12, 6, 8, 5), 8), ((30, 1, 4), 1)])
def test_mean_congruence_matches_oracle(dims, r):
    nnc = need_gpu()
    rng = np.random.default_rng(sum(dims) + r)
    P = [rng.random((n, r)).astype(np.float32) for n in dims]
    Q = [rng.random((n, r)).astype(np.float32) for n in dims]
    got = nnc.mean_congruence([dev(p) for p in P], [dev(q) for q in Q])
    assert abs(got - oracle.mean_congruence(P, Q)) <= 1e-12
    assert abs(nnc.mean_congruence([dev(p) for p in P], [dev(p) for p in P]) - 1.0) <= 1e-12


@pytest.mark.parametrize("j", [0, 1])
def test_sec43_both_algorithms_match_oracle(j):
    nnc = need_gpu()
    X, F, B, C = synth.rank_deficient_tensor(43, j)
    ini = synth.init_sec43(43, j, DIMS, RANKS, R)
    X64 = X.astype(np.float64)
    Xd = dev(X)
    Ct = [dev(c) for c in C]
    sweeps = 60
    # Algorithm 1
    G = dev(ini["G"])
    A = [dev(a) for a in ini["A"]]
    Bc = [dev(b) for b in ini["Bc"]]
    nnc.nntucker_fit(Xd, RANKS, sweeps, G, A, report=False)
    nnc.nncp_fit(G, R, sweeps, Bc, residual=False)
    C1 = nnc.nncandelinc_lift(A, Bc)
    ref1 = oracle.nncandelinc(X64, ini["G"], ini["A"], ini["Bc"], sweeps, sweeps)
    assert abs(nnc.reconstruct_residual(Xd, C1) - ref1["cp_rel"]) <= 1e-4
    assert abs(nnc.mean_congruence(C1, Ct) - oracle.mean_congruence(ref1["C"], C)) <= 1e-4
    # Algorithm 2
    Bx = [dev(b) for b in ini["Bx"]]
    W = [dev(w) for w in ini["W"]]
    H = [dev(h) for h in ini["H"]]
    nnc.nncandelinc_alg2(Xd, R, RANKS, sweeps, sweeps, Bx, W, H)
    C2 = nnc.nncandelinc_lift(W, H)
    ref2 = oracle.nncandelinc_alg2(X64, ini["Bx"], ini["W"], ini["H"], sweeps, sweeps)
    assert abs(nnc.reconstruct_residual(Xd, C2) - ref2["cp_rel"]) <= 1e-4
    assert abs(nnc.mean_congruence(C2, Ct) - oracle.mean_congruence(ref2["C"], C)) <= 1e-4
