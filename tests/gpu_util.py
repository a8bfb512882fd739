"""Helpers shared by the GPU tests: device tensors from the seeded generators, error norms."""
import numpy as np
import pytest
import torch

import synth


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_07570_amd as nnc
    if not nnc.device_ok():
        raise RuntimeError("GPU visible but libnncandelinc cannot use it (not gfx950?)")
    return nnc


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def bf16_dev(x64):
    """bfloat16 device tensor holding the RNE rounding of float64 values (via bit patterns)."""
    bits = synth.to_bf16_bits(synth.round_bf16(x64))
    t = torch.from_numpy(bits.view(np.int16).copy()).to("cuda")
    return t.view(torch.bfloat16)


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def problem(seed, dims, R_planted, ranks, zero_prob=0.0, noise=1e-3, dtype="f32"):
    """Planted X (rounded to dtype) plus float32 initial core and factors (all host numpy)."""
    X, planted = synth.planted_tensor(seed, dims, R_planted, zero_prob=zero_prob, noise=noise, dtype=dtype)
    G0 = synth.init_core(seed, ranks)
    A0 = synth.init_factors(seed, dims, ranks)
    return X, planted, G0, A0
