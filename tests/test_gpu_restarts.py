"""GPU parity of the random-restart study of Section 4.2 (many complete Algorithm 1 / 2 fits
of the paper's 4 x 4 x 4 example in one launch) against the FP64 oracle, start by start.

- Every assumed multirank of the study ([3,3,3], [3,4,4], [4,4,4], [5,5,5]) and both
  algorithms, a few sweeps: relative error and mean congruence within 1e-4 of the oracle's.
- Longer fits: relative error within 1e-3.
- The exact nonnegative factorizations of the example are fixed points of both algorithms:
  relative error exactly 0 and congruence exactly 1.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import dev, host, need_gpu
from tests.paper_fixtures import arr, examples

pytestmark = pytest.mark.gpu

MULTIRANKS = [(3, 3, 3), (3, 4, 4), (4, 4, 4), (5, 5, 5)]


def _example():
    e = examples()["ex5_rank_not_preserved_nn"]
    A = [arr(e["A1"]), arr(e["A2"]), arr(e["A3"])]
    return oracle.cp_full(A), A


def _run(nnc, X, A, alg, m, inits, outer, inner):
    res = nnc.nncandelinc_restarts(dev(X), alg, m, 4, dev(inits), outer, inner, truth=[dev(a) for a in A],
                                   lifted=True)
    return host(res.rel_errors), host(res.congruences), host(res.lifted), res.clips


@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("m", MULTIRANKS)
def test_restarts_match_oracle_few_sweeps(alg, m):
    nnc = need_gpu()
    X, A = _example()
    inits = synth.init_restarts(40 + alg, alg, X.shape, m, 4, 6)
    rel, cong, lifted, _ = _run(nnc, X, A, alg, m, inits, 30, 30)
    for j in range(6):
        parts = synth.unpack_restart(inits[j].astype(np.float64), alg, X.shape, m, 4)
        r_o, c_o, C_o = oracle.restart_fit(X, alg, parts, 30, 30, truth=A)
        assert abs(rel[j] - r_o) <= 1e-4, (alg, m, j, rel[j], r_o)
        assert abs(cong[j] - c_o) <= 1e-4, (alg, m, j, cong[j], c_o)
        C = np.split(lifted[j], np.cumsum(X.shape)[:-1])
        for c, co in zip(C, C_o):
            assert np.linalg.norm(c - co) <= 1e-4 * max(1.0, np.linalg.norm(co))


@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("m", MULTIRANKS[:3])
def test_restarts_long_fits(alg, m):
    nnc = need_gpu()
    X, A = _example()
    inits = synth.init_restarts(50 + alg, alg, X.shape, m, 4, 3)
    rel, cong, _, _ = _run(nnc, X, A, alg, m, inits, 300, 300)
    for j in range(3):
        parts = synth.unpack_restart(inits[j].astype(np.float64), alg, X.shape, m, 4)
        r_o, c_o, _ = oracle.restart_fit(X, alg, parts, 300, 300, truth=A)
        assert abs(rel[j] - r_o) <= 1e-3, (alg, m, j, rel[j], r_o)
        assert np.isfinite(cong[j]) and -1.0 - 1e-6 <= cong[j] <= 1.0 + 1e-6


def test_exact_factorizations_are_fixed_points():
    nnc = need_gpu()
    X, A = _example()
    I4 = np.eye(4)
    D = np.zeros((4, 4, 4))
    for i in range(4):
        D[i, i, i] = 1.0
    alg1 = np.concatenate([a.ravel() for a in A] + [D.ravel()] + [I4.ravel()] * 3)
    alg2 = np.concatenate([a.ravel() for a in A] * 2 + [I4.ravel()] * 3)
    for alg, v in ((1, alg1), (2, alg2)):
        inits = np.stack([v, v]).astype(np.float32)
        rel, cong, lifted, _ = _run(nnc, X, A, alg, (4, 4, 4), inits, 50, 50)
        assert rel[0] == 0.0 and rel[1] == 0.0, (alg, rel)
        assert cong[0] == 1.0 and cong[1] == 1.0, (alg, cong)
        assert np.array_equal(lifted[0], np.concatenate(A))


def test_zero_restarts_and_without_truth():
    nnc = need_gpu()
    X, _ = _example()
    empty = torch.empty(0, nnc.lib().nncandelinc_restart_init_floats(1, nnc._dims(X.shape), nnc._dims((3, 3, 3)), 4),
                        device="cuda")
    res = nnc.nncandelinc_restarts(dev(X), 1, (3, 3, 3), 4, empty, 10, 10)
    assert res.rel_errors.numel() == 0 and res.congruences is None
    inits = synth.init_restarts(60, 1, X.shape, (3, 3, 3), 4, 2)
    res = nnc.nncandelinc_restarts(dev(X), 1, (3, 3, 3), 4, dev(inits), 10, 10)
    assert res.congruences is None and np.all(np.isfinite(host(res.rel_errors)))
