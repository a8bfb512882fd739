"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the decomposition method itself: it only draws
numbers and assembles the planted test tensors (sums of outer products, the
construction of a rank-R tensor in the paper's Section 2 definition of the tensor
product) that both sides then receive as identical inputs.

Random numbers come from a counter-based form of SplitMix64 (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): the 64-bit value for
element ``i`` of stream ``s`` under seed ``seed`` is

    key   = mix64(mix64(seed + GAMMA) ^ (s * GOLDEN2))
    u64   = mix64(key + (i + 1) * GAMMA)          (all arithmetic mod 2**64)

with SplitMix64's finaliser ``mix64`` and ``GAMMA = 0x9E3779B97F4A7C15``.  A uniform
double in [0, 1) is ``(u64 >> 11) * 2**-53``.  Values are independent of the order of
generation, so any slice of a stream can be produced on its own.

Stream ids (one per role):  planted factor n -> n;  zero mask of planted factor n ->
16 + n;  additive noise -> 32;  initial core G0 -> 48;  initial Tucker factor n ->
64 + n;  nnCP restart j, factor n -> 1024 + 16 j + n;  NMF of factor n (Algorithm 2):
W0 -> 2048 + n, H0 -> 2064 + n;  restart j of the small-tensor study -> 4096 + j (one stream per
start, laid out as unpack_restart() splits it);  generated tensor j of the rank-deficient study,
attempt a, its F_n / B_n -> 1 << 20 + 64 (16 j + a) + n / + 8 + n, and the fits' initial values
-> 1 << 24 + 64 j + role.
"""

from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
GOLDEN2 = 0xD1B54A32D192ED03
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1

STREAM_PLANTED = 0
STREAM_MASK = 16
STREAM_NOISE = 32
STREAM_CORE0 = 48
STREAM_FACTOR0 = 64
STREAM_CP_RESTART = 1024
STREAM_NMF_W = 2048
STREAM_NMF_H = 2064
STREAM_RESTART = 4096
STREAM_GEN43 = 1 << 20
STREAM_INIT43 = 1 << 24


def _mix64_int(z: int) -> int:
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> int:
    return _mix64_int(_mix64_int(seed + GAMMA) ^ ((stream * GOLDEN2) & _MASK))


def raw_u64(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` raw 64-bit draws of ``stream`` starting at element ``offset``."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + idx * np.uint64(GAMMA)
    return _mix64(z)


def uniform(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` doubles in [0, 1) (53-bit resolution)."""
    u = raw_u64(seed, stream, n, offset) >> np.uint64(11)
    return u.astype(np.float64) * (2.0 ** -53)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even); returns float64.

    bfloat16 keeps 8 significant bits.  Only finite normal-range values are expected.
    """
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()                  # zeros (of either sign) are already exact
    nz = x != 0
    _, e = np.frexp(x[nz])          # x = m * 2**e with 0.5 <= |m| < 1
    q = np.ldexp(1.0, e - 8)        # spacing of 8-significant-bit values in that binade
    # np.round is round-half-to-even
    out[nz] = np.round(x[nz] / q) * q
    return out


def to_bf16_bits(x64: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of float64 values that are already bf16-exact."""
    f32 = np.asarray(x64, dtype=np.float32)
    return (f32.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    u32 = bits.astype(np.uint32) << np.uint32(16)
    return u32.view(np.float32).astype(np.float64)


def uniform_matrix(seed: int, stream: int, rows: int, cols: int) -> np.ndarray:
    return uniform(seed, stream, rows * cols).reshape(rows, cols)


def init_factors(seed: int, dims, ranks, dtype=np.float32):
    """Initial Tucker factors A0_n ~ U[0,1), each dims[n] x ranks[n], rounded to ``dtype``."""
    return [uniform_matrix(seed, STREAM_FACTOR0 + n, int(dims[n]), int(ranks[n])).astype(dtype)
            for n in range(len(dims))]


def init_core(seed: int, ranks, dtype=np.float32):
    """Initial core G0 ~ U[0,1) of shape ranks, rounded to ``dtype``."""
    size = int(np.prod(ranks))
    return uniform(seed, STREAM_CORE0, size).reshape(tuple(int(r) for r in ranks)).astype(dtype)


def init_cp_factors(seed: int, core_dims, rank: int, restart: int = 0, dtype=np.float32):
    """Initial nnCP factors B0_n ~ U[0,1), each core_dims[n] x rank."""
    return [uniform_matrix(seed, STREAM_CP_RESTART + 16 * restart + n, int(core_dims[n]), rank)
            .astype(dtype) for n in range(len(core_dims))]


def init_nmf(seed: int, dims, ranks, rank: int, dtype=np.float32):
    """Initial NMF factors of the CP factors A^(n) ~ W_n H_n (Algorithm 2): W0_n ~ U[0,1)
    dims[n] x ranks[n] and H0_n ~ U[0,1) ranks[n] x rank."""
    W = [uniform_matrix(seed, STREAM_NMF_W + n, int(dims[n]), int(ranks[n])).astype(dtype)
         for n in range(len(dims))]
    H = [uniform_matrix(seed, STREAM_NMF_H + n, int(ranks[n]), int(rank)).astype(dtype)
         for n in range(len(dims))]
    return W, H


def restart_init_sizes(alg: int, dims, multirank, rank: int):
    """Shapes of the initial values of one start of the small-tensor study, in storage order:
    Algorithm 1: A_n (dims[n] x m_n), G (m), B_n (m_n x r); Algorithm 2: B_n (dims[n] x r),
    W_n (dims[n] x m_n), H_n (m_n x r)."""
    d, m = [int(x) for x in dims], [int(x) for x in multirank]
    if alg == 1:
        return [(d[n], m[n]) for n in range(3)] + [tuple(m)] + [(m[n], rank) for n in range(3)]
    return [(d[n], rank) for n in range(3)] + [(d[n], m[n]) for n in range(3)] + [(m[n], rank) for n in range(3)]


def init_restarts(seed: int, alg: int, dims, multirank, rank: int, nres: int, dtype=np.float32):
    """U[0,1) initial values of `nres` starts, one stream each, as an nres x per-start array."""
    size = sum(int(np.prod(s)) for s in restart_init_sizes(alg, dims, multirank, rank))
    return np.stack([uniform(seed, STREAM_RESTART + j, size) for j in range(nres)]).astype(dtype)


def unpack_restart(vec, alg: int, dims, multirank, rank: int):
    """Split one start's vector into its arrays (storage order of restart_init_sizes)."""
    out, off = [], 0
    for shp in restart_init_sizes(alg, dims, multirank, rank):
        k = int(np.prod(shp))
        out.append(np.asarray(vec[off:off + k]).reshape(shp))
        off += k
    return out


def kruskal_rank(M) -> int:
    """Largest k such that every set of k columns of M is linearly independent."""
    import itertools
    M = np.asarray(M, dtype=np.float64)
    k = 0
    for size in range(1, M.shape[1] + 1):
        if all(np.linalg.matrix_rank(M[:, list(c)]) == size
               for c in itertools.combinations(range(M.shape[1]), size)):
            k = size
        else:
            break
    return k


def rank_deficient_tensor(seed: int, j: int, dims=(40, 40, 40), ranks=(3, 4, 5), r: int = 5,
                          max_attempts: int = 16):
    """Tensor j of the rank-deficient study: X = sum_rho outer(C_1[:, rho], .., C_3[:, rho]) with
    C_n = F_n B_n, F_n ~ U[0,1) dims[n] x ranks[n] and B_n ~ U[0,1) ranks[n] x r, redrawn until the
    Kruskal ranks of the C_n sum to at least 2r + 2.  Returns (X float32, F, B, C) with F, B and
    C float32 and X formed in float64 from the float32 C and rounded once."""
    for a in range(max_attempts):
        base = STREAM_GEN43 + 64 * (16 * j + a)
        F = [uniform_matrix(seed, base + n, int(dims[n]), int(ranks[n])).astype(np.float32) for n in range(3)]
        B = [uniform_matrix(seed, base + 8 + n, int(ranks[n]), r).astype(np.float32) for n in range(3)]
        C64 = [f.astype(np.float64) @ b.astype(np.float64) for f, b in zip(F, B)]
        # the criterion on the exact products (rounding them to float32 would add full rank)
        if sum(kruskal_rank(c) for c in C64) >= 2 * r + 2:
            C = [c.astype(np.float32) for c in C64]
            X = np.einsum("ir,jr,kr->ijk", *[c.astype(np.float64) for c in C])
            return X.astype(np.float32), F, B, C
    raise RuntimeError("no draw met the Kruskal criterion")


def init_sec43(seed: int, j: int, dims, ranks, r: int, dtype=np.float32):
    """Initial values of both algorithms on tensor j: Algorithm 1 (A_n dims[n] x ranks[n], G,
    core CP factors ranks[n] x r) and Algorithm 2 (CP factors dims[n] x r, NMF W_n, H_n)."""
    base = STREAM_INIT43 + 64 * j
    A = [uniform_matrix(seed, base + n, int(dims[n]), int(ranks[n])).astype(dtype) for n in range(3)]
    G = uniform(seed, base + 3, int(np.prod(ranks))).reshape(tuple(int(x) for x in ranks)).astype(dtype)
    Bc = [uniform_matrix(seed, base + 4 + n, int(ranks[n]), r).astype(dtype) for n in range(3)]
    Bx = [uniform_matrix(seed, base + 8 + n, int(dims[n]), r).astype(dtype) for n in range(3)]
    W = [uniform_matrix(seed, base + 12 + n, int(dims[n]), int(ranks[n])).astype(dtype) for n in range(3)]
    H = [uniform_matrix(seed, base + 16 + n, int(ranks[n]), r).astype(dtype) for n in range(3)]
    return dict(A=A, G=G, Bc=Bc, Bx=Bx, W=W, H=H)


def planted_factors(seed: int, dims, R: int, zero_prob: float = 0.0):
    """Planted nonnegative CP factors a_n (dims[n] x R), entries U[0,1).

    With ``zero_prob`` > 0 each entry is zeroed when its own mask draw is below
    ``zero_prob``; a column left entirely zero keeps the entry with the largest mask draw.
    """
    facs = []
    for n, N in enumerate(dims):
        a = uniform_matrix(seed, STREAM_PLANTED + n, int(N), R)
        if zero_prob > 0.0:
            u = uniform_matrix(seed, STREAM_MASK + n, int(N), R)
            keep = u >= zero_prob
            for c in range(R):
                if not keep[:, c].any():
                    keep[int(np.argmax(u[:, c])), c] = True
            a = np.where(keep, a, 0.0)
        facs.append(a)
    return facs


def planted_tensor(seed: int, dims, R: int, zero_prob: float = 0.0, noise: float = 1e-3,
                   dtype: str = "f32", chunk_elems: int = 1 << 24):
    """Dense planted tensor X = sum_rho outer(a_1[:,rho], ..., a_d[:,rho]) + E, E ~ U[0, noise).

    X is formed in float64 and rounded once to ``dtype``:
      "f64" -> float64 array, "f32" -> float32 array (RNE),
      "bf16" -> uint16 array of bfloat16 bit patterns (RNE of the float64 value).
    Returns (X, planted_factors).  Built in chunks of leading-mode rows to bound memory.
    """
    dims = [int(n) for n in dims]
    d = len(dims)
    facs = planted_factors(seed, dims, R, zero_prob)
    total = int(np.prod(dims))
    last = dims[-1]
    lead = total // last
    out_dt = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[dtype]
    X = np.empty(total, dtype=out_dt)
    rows_per_chunk = max(1, chunk_elems // last)
    lead_dims = dims[:-1]
    for r0 in range(0, lead, rows_per_chunk):
        r1 = min(lead, r0 + rows_per_chunk)
        m = np.arange(r0, r1, dtype=np.int64)
        # Khatri-Rao rows of the leading factors for flattened leading indices m.
        kr = np.ones((r1 - r0, R), dtype=np.float64)
        rem = m.copy()
        for k in range(d - 2, -1, -1):
            ik = rem % lead_dims[k]
            rem //= lead_dims[k]
            kr *= facs[k][ik, :]
        blk = kr @ facs[-1].T
        flat0, flat1 = r0 * last, r1 * last
        if noise > 0.0:
            blk = blk + noise * uniform(seed, STREAM_NOISE, flat1 - flat0, flat0).reshape(blk.shape)
        if dtype == "f64":
            X[flat0:flat1] = blk.ravel()
        elif dtype == "f32":
            X[flat0:flat1] = blk.ravel().astype(np.float32)
        else:
            X[flat0:flat1] = to_bf16_bits(round_bf16(blk.ravel()))
    return X.reshape(dims), facs


STREAM_SIGNED = 1 << 28


def signed_planted(seed: int, dims, R: int, noise: float = 1e-2, deficient_mode: int = -1):
    """Real-valued planted CP tensor for the unconstrained (real) CANDELINC path:
    X = sum_rho outer(a_1[:,rho], ..., a_d[:,rho]) + E with factor entries 2u - 1 and
    E = noise * (2u - 1).  With deficient_mode = k the last column of a_k is the mean of its
    other columns, so the CPD factor of mode k has rank R - 1 (the rank-deficient factor
    that Section 2.2 discusses).  Returns (X float64, planted factors)."""
    dims = [int(n) for n in dims]
    facs = [2.0 * uniform_matrix(seed, STREAM_SIGNED + n, N, R) - 1.0 for n, N in enumerate(dims)]
    if deficient_mode >= 0:
        a = facs[deficient_mode]
        a[:, R - 1] = a[:, :R - 1].mean(axis=1)
    X = np.zeros(dims)
    for rho in range(R):
        t = facs[0][:, rho]
        for a in facs[1:]:
            t = np.multiply.outer(t, a[:, rho])
        X += t
    if noise > 0.0:
        X += noise * (2.0 * uniform(seed, STREAM_SIGNED + 16, int(np.prod(dims))).reshape(dims) - 1.0)
    return X, facs


def signed_planted_tucker(seed: int, dims, ranks, noise: float = 1e-2):
    """Real-valued planted Tucker tensor X = G x_1 A_1 ... x_d A_d + E with core and factor
    entries 2u - 1 and E = noise * (2u - 1): multilinear rank `ranks` up to the noise.
    Returns X as float64."""
    dims = [int(n) for n in dims]
    ranks = [int(r) for r in ranks]
    X = 2.0 * uniform(seed, STREAM_SIGNED + 32, int(np.prod(ranks))).reshape(ranks) - 1.0
    for n, (N, R) in enumerate(zip(dims, ranks)):
        A = 2.0 * uniform_matrix(seed, STREAM_SIGNED + 40 + n, N, R) - 1.0
        X = np.moveaxis(np.tensordot(A, X, axes=([1], [n])), 0, n)
    if noise > 0.0:
        X = X + noise * (2.0 * uniform(seed, STREAM_SIGNED + 17, int(np.prod(dims))).reshape(dims) - 1.0)
    return np.ascontiguousarray(X)
