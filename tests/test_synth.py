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
