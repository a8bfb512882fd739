"""The shared seeded input generator: determinism, slicing and rounding."""
import numpy as np
import torch

import synth


def test_uniform_is_counter_based():
    a = synth.uniform(7, 3, 1000)
    b = synth.uniform(7, 3, 400, offset=600)
    assert np.array_equal(a[600:], b)
    assert ((a >= 0) & (a < 1)).all()
    assert not np.array_equal(a, synth.uniform(7, 4, 1000))
    assert not np.array_equal(a, synth.uniform(8, 3, 1000))
    assert abs(a.mean() - 0.5) < 0.05


def test_splitmix_finaliser_known_value():
    # SplitMix64 with state 0: the first output is mix64(GAMMA) = 0xE220A8397B1DCDAF
    assert synth._mix64_int(synth.GAMMA) == 0xE220A8397B1DCDAF


def test_bf16_rounding_matches_torch():
    x = np.concatenate([synth.uniform(1, 0, 5000) * 7.0, [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 2.0 - 2 ** -9]])
    ref = torch.tensor(x, dtype=torch.float64).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(synth.round_bf16(x), ref)
    bits = synth.to_bf16_bits(synth.round_bf16(x))
    assert np.array_equal(synth.bf16_bits_to_f64(bits), ref)


def test_planted_tensor_shapes_and_chunking():
    X1, f1 = synth.planted_tensor(5, (6, 5, 4), 3, zero_prob=0.5, dtype="f64", chunk_elems=7)
    X2, f2 = synth.planted_tensor(5, (6, 5, 4), 3, zero_prob=0.5, dtype="f64")
    assert np.array_equal(X1, X2)
    exact = np.einsum("ir,jr,kr->ijk", *f1)
    assert np.all(X1 - exact >= 0) and np.all(X1 - exact < 1e-3 + 1e-15)
    assert all((f[:, c] != 0).any() for f in f1 for c in range(3))
    X32, _ = synth.planted_tensor(5, (6, 5, 4), 3, zero_prob=0.5, dtype="f32")
    assert np.array_equal(X32, X2.astype(np.float32))


def test_kruskal_rank_small_cases():
    assert synth.kruskal_rank(np.eye(4)) == 4
    M = np.array([[1.0, 2.0, 1.0], [0.0, 0.0, 1.0], [1.0, 2.0, 0.0]])  # columns 0 and 1 parallel
    assert synth.kruskal_rank(M) == 1
    Z = np.array([[0.0, 1.0], [0.0, 2.0]])  # a zero column
    assert synth.kruskal_rank(Z) == 0
    V = np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 1.0]])  # any two independent, three not
    assert synth.kruskal_rank(V) == 2


def test_rank_deficient_generator():
    """Tensors of the rank-deficient study: C_n = F_n B_n with Kruskal ranks (3, 4, 5) meeting
    k_1 + k_2 + k_3 >= 2r + 2, and X the rank-5 CP of the float32 C_n."""
    for j in range(3):
        X, F, B, C = synth.rank_deficient_tensor(7, j)
        assert X.shape == (40, 40, 40) and X.dtype == np.float32
        ks = [synth.kruskal_rank(f.astype(np.float64) @ b.astype(np.float64)) for f, b in zip(F, B)]
        assert ks == [3, 4, 5] and sum(ks) >= 12
        for f, b, c in zip(F, B, C):
            assert np.array_equal(c, (f.astype(np.float64) @ b.astype(np.float64)).astype(np.float32))
        Xr = np.zeros((40, 40, 40))
        for rho in range(5):
            Xr += np.multiply.outer(np.multiply.outer(C[0][:, rho].astype(np.float64), C[1][:, rho]), C[2][:, rho])
        assert np.array_equal(X, Xr.astype(np.float32))
    a, b = synth.rank_deficient_tensor(7, 0), synth.rank_deficient_tensor(7, 0)
    assert np.array_equal(a[0], b[0])
