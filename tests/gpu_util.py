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


def planted_tensor_dev(seed, dims, R, zero_prob=0.0, noise=1e-3, chunk_rows=1 << 18):
    """FP32 device copy of synth.planted_tensor(seed, dims, R, zero_prob, noise, "f32"), built
    on the GPU: the planted factors come from synth, the noise stream from nnc_fill_uniform_f64
    (the same counter-based draws), and each chunk of leading rows is formed in float64 and
    rounded once.  The product of the Khatri-Rao rows with the last factor runs in a different
    summation order than the host's, so a rare entry may differ in its last bit."""
    import paper_1909_07570_amd as nnc
    dims = [int(n) for n in dims]
    d = len(dims)
    facs = [torch.from_numpy(f).to("cuda") for f in synth.planted_factors(seed, dims, R, zero_prob)]
    last = dims[-1]
    lead = int(np.prod(dims[:-1]))
    X = torch.empty(lead * last, dtype=torch.float32, device="cuda")
    for r0 in range(0, lead, chunk_rows):
        r1 = min(lead, r0 + chunk_rows)
        rem = torch.arange(r0, r1, dtype=torch.int64, device="cuda")
        kr = torch.ones((r1 - r0, R), dtype=torch.float64, device="cuda")
        for k in range(d - 2, -1, -1):
            ik = rem % dims[k]
            rem = rem // dims[k]
            kr *= facs[k][ik, :]
        blk = kr @ facs[-1].T.contiguous()
        if noise > 0.0:
            u = nnc.nnc_fill_uniform_f64(seed, synth.STREAM_NOISE, (r1 - r0) * last, offset=r0 * last)
            blk += noise * u.view(blk.shape)
        X[r0 * last:r1 * last] = blk.reshape(-1).to(torch.float32)
        del kr, blk
    return X.view(dims)


def signed_planted_dev(seed, dims, R, noise=1e-3, chunk_rows=1 << 18):
    """FP32 device copy of synth.signed_planted(seed, dims, R, noise) rounded to float32, built
    on the GPU from the same planted factors and the same counter-based noise draws; each
    chunk of leading rows is formed in float64 and rounded once.  The sum over components
    runs in a different order than the host's, so a rare entry may differ in its last bit."""
    import paper_1909_07570_amd as nnc
    dims = [int(n) for n in dims]
    d = len(dims)
    facs = [torch.from_numpy(2.0 * synth.uniform_matrix(seed, synth.STREAM_SIGNED + n, N, R) - 1.0).to("cuda")
            for n, N in enumerate(dims)]
    last = dims[-1]
    lead = int(np.prod(dims[:-1]))
    X = torch.empty(lead * last, dtype=torch.float32, device="cuda")
    for r0 in range(0, lead, chunk_rows):
        r1 = min(lead, r0 + chunk_rows)
        rem = torch.arange(r0, r1, dtype=torch.int64, device="cuda")
        kr = torch.ones((r1 - r0, R), dtype=torch.float64, device="cuda")
        for k in range(d - 2, -1, -1):
            ik = rem % dims[k]
            rem = rem // dims[k]
            kr *= facs[k][ik, :]
        blk = kr @ facs[-1].T.contiguous()
        if noise > 0.0:
            u = nnc.nnc_fill_uniform_f64(seed, synth.STREAM_SIGNED + 16, (r1 - r0) * last, offset=r0 * last)
            blk += noise * (2.0 * u.view(blk.shape) - 1.0)
        X[r0 * last:r1 * last] = blk.reshape(-1).to(torch.float32)
        del kr, blk
    return X.view(dims)
