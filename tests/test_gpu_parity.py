"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances: FP32 TTM <= 1e-5 relative Frobenius; BF16-MFMA TTM <= 2e-2 (the library applies
the factor as a hi+lo bf16 pair, so in practice only X's rounding matters and the observed
error is far below that bar); final relative residual within 1e-3 of the oracle after equal
sweeps; integer work (conversion, exact examples, fixed points) bit-exact.
"""
import os
import zlib

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import bf16_dev, dev, host, need_gpu, problem, rel_fro
from tests.paper_fixtures import arr, examples, fold

pytestmark = pytest.mark.gpu

TTM_SHAPES = [
    (37, 29, 18),          # ragged everywhere
    (64, 48, 40),          # several MFMA tiles
    (130, 24, 72),         # ragged leading mode, Q multiple of 8
    (12, 10, 9, 8),        # 4-way
    (6, 5, 8, 4, 8),       # 5-way
    (200, 96),             # 2-way
]


@pytest.mark.parametrize("shape", TTM_SHAPES)
@pytest.mark.parametrize("R", [1, 5, 16, 20, 32, 40])
def test_ttm_fp32_every_mode(shape, R):
    nnc = need_gpu()
    rng = np.random.default_rng(zlib.crc32(repr((shape, R)).encode()))
    X = rng.random(shape).astype(np.float32)
    Xd = dev(X)
    for n in range(len(shape)):
        A = rng.random((shape[n], R)).astype(np.float32)
        out = host(nnc.nnc_ttm(Xd, n, dev(A)))
        ref = oracle.ttm_t(X.astype(np.float64), n, A.astype(np.float64))
        assert rel_fro(out, ref) <= 1e-5, (shape, R, n, rel_fro(out, ref))


@pytest.mark.parametrize("shape", TTM_SHAPES)
@pytest.mark.parametrize("R", [3, 16, 20, 32])
def test_ttm_bf16_every_mode(shape, R):
    nnc = need_gpu()
    rng = np.random.default_rng(zlib.crc32(repr((shape, R, 1)).encode()))
    X64 = synth.round_bf16(rng.random(shape))
    Xd = bf16_dev(X64)
    for n in range(len(shape)):
        A = rng.random((shape[n], R)).astype(np.float32)
        out = host(nnc.nnc_ttm(Xd, n, dev(A)))
        ref = oracle.ttm_t(X64, n, A.astype(np.float64))
        err = rel_fro(out, ref)
        assert err <= 2e-2, (shape, R, n, err)
        # hi+lo factor split: only accumulation rounding remains
        assert err <= 1e-4, (shape, R, n, err)


# Earlier-mode bf16 pass with more 128-column tiles than waves (several tiles per wave, the
# next tile's loads issued before the current tile's output) and a ragged last tile.
@pytest.mark.parametrize("shape", [(16, 1000, 524), (24, 1000, 1048)])
@pytest.mark.parametrize("R", [12, 20])
def test_ttm_mid_bf16_several_tiles_per_wave(shape, R):
    nnc = need_gpu()
    rng = np.random.default_rng(zlib.crc32(repr((shape, R, 2)).encode()))
    X64 = synth.round_bf16(rng.random(shape))
    A = rng.random((shape[0], R)).astype(np.float32)
    out = host(nnc.nnc_ttm(bf16_dev(X64), 0, dev(A)))
    ref = oracle.ttm_t(X64, 0, A.astype(np.float64))
    assert rel_fro(out, ref) <= 1e-4
    # every column (tile) checked on its own, the ragged last one included
    col_err = np.abs(out - ref).max(axis=0) / np.abs(ref).max(axis=0)
    assert col_err.max() <= 1e-4, int(np.argmax(col_err))


# Last-mode (contraction index contiguous) shapes chosen for the row-contiguous pass kernel:
# every piece width (64/128/256 k for bf16, 32/64/128 for f32), partial last pieces, fewer
# rows than one tile, ragged row counts, and enough tiles that waves get 1..3 pieces each.
LAST_SHAPES = [(5, 64), (77, 520), (45, 136), (1000, 256), (70001, 128), (3000, 512), (33, 40)]


@pytest.mark.parametrize("shape", LAST_SHAPES)
@pytest.mark.parametrize("R", [3, 16, 20, 32])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_ttm_last_mode_row_contiguous(shape, R, dt):
    nnc = need_gpu()
    rng = np.random.default_rng(zlib.crc32(repr((shape, R, dt)).encode()))
    M, K = shape
    A = rng.random((K, R)).astype(np.float32)
    if dt == "bf16":
        X64 = synth.round_bf16(rng.random(shape))
        Xd, tol = bf16_dev(X64), 1e-4
    else:
        X32 = rng.random(shape).astype(np.float32)
        X64, Xd, tol = X32.astype(np.float64), dev(X32), 1e-5
    out = host(nnc.nnc_ttm(Xd, 1, dev(A)))
    ref = X64 @ A.astype(np.float64)
    assert out.shape == (M, R)
    err = rel_fro(out, ref)
    assert err <= tol, (shape, R, dt, err)
    # every row individually (a wrong tile or piece shows up even when the total is close)
    rows = np.linalg.norm(out - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-30)
    assert rows.max() <= 10 * tol, (shape, R, dt, int(rows.argmax()), rows.max())


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_identity_factor_returns_x_bit_exact(dt):
    nnc = need_gpu()
    rng = np.random.default_rng(3)
    shape = (40, 24, 32)
    X64 = synth.round_bf16(rng.random(shape))  # bf16-exact values are fp32-exact too
    Xd = bf16_dev(X64) if dt == "bf16" else dev(X64.astype(np.float32))
    for n in range(3):
        out = host(nnc.nnc_ttm(Xd, n, dev(np.eye(shape[n], dtype=np.float32))))
        assert np.array_equal(out, X64), n


def test_ex2_bit_exact():
    nnc = need_gpu()
    e = examples()["ex2_rank_not_preserved"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    G = fold(e["G_unfold1"], 0, e["core_dims"])
    out = host(nnc.nnc_ttm(dev(G), 0, dev(arr(e["M1"]).T)))
    assert np.array_equal(out, X)


def test_convert_bf16_bit_exact():
    nnc = need_gpu()
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.random(100000) * 13.0, rng.standard_normal(1000) * 1e-30,
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 0.0, -0.0, 65504.0]]).astype(np.float32)
    got = nnc.nnc_convert_f32_bf16(dev(x)).view(torch.int16).cpu().numpy().view(np.uint16)
    ref = synth.to_bf16_bits(synth.round_bf16(x.astype(np.float64)))
    assert np.array_equal(got, ref)


# ------------------------------------------------------------------------------ nnTucker
def _fit_gpu(nnc, X, G0, A0, iters, dt="f32", **kw):
    Xd = dev(X) if dt == "f32" else bf16_dev(np.asarray(X, np.float64))
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.nntucker_fit(Xd, G0.shape, iters, G, A, **kw)
    return host(G), [host(a) for a in A], rep


@pytest.mark.parametrize("dims,ranks", [((40, 40, 40), (5, 5, 5)), ((37, 29, 18), (4, 3, 5)),
                                        ((12, 10, 9, 8), (3, 4, 2, 5)), ((6, 5, 8, 4, 7), (2, 3, 2, 2, 3)),
                                        ((50, 44), (4, 6)), ((4, 4, 4), (5, 5, 5)),
                                        # core slices wider than one staged chunk of the row
                                        # update (several chunks, a ragged last one)
                                        ((14, 13, 12, 11), (10, 10, 10, 10)),
                                        ((40, 36, 34), (32, 32, 32)),
                                        # small contractions split over blocks along the
                                        # contracted mode (ragged splits, two rounds each)
                                        ((300, 40, 260), (4, 5, 6)),
                                        ((45, 1100, 37), (3, 7, 2)),
                                        # cores beyond the whole-core kernels: mode slices in
                                        # LDS, each row of M over several blocks
                                        ((20, 18, 17, 19), (16, 16, 16, 16)),
                                        ((10, 9, 8, 9, 10), (8, 8, 8, 8, 8)),
                                        # uneven slices; mode 0's row update in the scalar
                                        # path over several chunks (a ragged last one)
                                        ((9, 8, 34, 35), (5, 5, 30, 31))])
@pytest.mark.parametrize("use_graph", [False, True])
def test_nntucker_few_sweeps_match_oracle(dims, ranks, use_graph):
    nnc = need_gpu()
    X, _, G0, A0 = problem(31, dims, 3, ranks)
    G, A, rep = _fit_gpu(nnc, X, G0, A0, 3, use_graph=use_graph)
    Go, Ao, _, _ = oracle.nntucker(X.astype(np.float64), G0, A0, 3)
    assert rel_fro(oracle.tucker_full(G, A), oracle.tucker_full(Go, Ao)) <= 1e-4
    for a, ao in zip(A, Ao):
        assert rel_fro(a, ao) <= 1e-3
    assert (G >= 0).all() and all((a >= 0).all() for a in A)
    ref = oracle.tucker_rel_residual(X.astype(np.float64), Go, Ao)
    assert abs(rep.rel_residual - ref) <= 1e-5
    assert rep.eps_clips == 0


@pytest.mark.parametrize("dims,ranks", [((20, 18, 17, 19), (16, 16, 16, 16)), ((40, 36, 34), (32, 32, 32)),
                                        ((10, 9, 8, 9, 10), (8, 8, 8, 8, 8)), ((24, 20, 22, 18), (16, 16, 16, 8))])
def test_big_core_slice_steps_match_grid_wide_steps(dims, ranks):
    """Cores beyond the whole-core kernels: the core-space steps on mode slices (rows of M
    over several blocks, the core update slice by slice) against the grid-wide chain of
    small contractions (NNC_NO_BIG_SLICES), the same sweeps in other summation orders."""
    nnc = need_gpu()
    X, _, G0, A0 = problem(38, dims, 3, ranks)
    print("case", dims, ranks, flush=True)
    G, A, rep = _fit_gpu(nnc, X, G0, A0, 3)
    os.environ["NNC_NO_BIG_SLICES"] = "1"
    try:
        Gg, Ag, repg = _fit_gpu(nnc, X, G0, A0, 3)
    finally:
        del os.environ["NNC_NO_BIG_SLICES"]
    assert rel_fro(G, Gg) <= 1e-5
    for a, ag in zip(A, Ag):
        assert rel_fro(a, ag) <= 1e-5
    assert rep.eps_clips == repg.eps_clips == 0
    Go, Ao, _, _ = oracle.nntucker(X.astype(np.float64), G0, A0, 3)
    assert rel_fro(oracle.tucker_full(G, A), oracle.tucker_full(Go, Ao)) <= 1e-4


def _offset_view(a):
    """Device copy of `a` starting one float past a 256-byte boundary (4-byte aligned only)."""
    buf = torch.zeros(a.size + 1, device="cuda", dtype=torch.float32)
    v = buf[1:].view(a.shape)
    v.copy_(torch.from_numpy(np.ascontiguousarray(a, np.float32)))
    return v


@pytest.mark.parametrize("dims,ranks", [((12, 10, 9, 8), (3, 4, 2, 5)),      # quad rows, padded
                                        ((14, 13, 12, 11), (10, 10, 10, 10)),  # several chunks
                                        ((40, 36, 34), (32, 32, 32))])
def test_nntucker_unaligned_core_and_factors(dims, ranks):
    """Core and factors 4 bytes off a 16-byte boundary take the row update's scalar staging;
    staging only moves data, so the fit equals the aligned one bit for bit and the oracle
    to the usual bar."""
    nnc = need_gpu()
    X, _, G0, A0 = problem(37, dims, 3, ranks)
    Xd = dev(X)
    G, A = dev(G0), [dev(a) for a in A0]
    nnc.nntucker_fit(Xd, G0.shape, 3, G, A)
    Gu, Au = _offset_view(G0), [_offset_view(a) for a in A0]
    assert Gu.data_ptr() % 16 == 4
    rep = nnc.nntucker_fit(Xd, G0.shape, 3, Gu, Au)
    assert torch.equal(Gu, G) and all(torch.equal(x, y) for x, y in zip(Au, A))
    Go, Ao, _, _ = oracle.nntucker(X.astype(np.float64), G0, A0, 3)
    assert rel_fro(oracle.tucker_full(host(Gu), [host(a) for a in Au]),
                   oracle.tucker_full(Go, Ao)) <= 1e-4
    assert rep.eps_clips == 0


def test_c1_workload_final_residual_matches_oracle():
    """40^3, planted rank 3, multirank (5,5,5), 200 sweeps; nnCP rank 3, 300 sweeps; lift."""
    nnc = need_gpu()
    X, _, G0, A0 = problem(1, (40, 40, 40), 3, (5, 5, 5))
    B0 = synth.init_cp_factors(1, (5, 5, 5), 3)
    G, A, rep = _fit_gpu(nnc, X, G0, A0, 200)
    X64 = X.astype(np.float64)
    ref = oracle.nncandelinc(X64, G0, A0, B0, 200, 300)
    assert abs(rep.rel_residual - ref["tucker_rel"]) <= 1e-3
    Gd = dev(G)
    Bd = [dev(b) for b in B0]
    nnc.nncp_fit(Gd, 3, 300, Bd)
    C = nnc.nncandelinc_lift([dev(a) for a in A], Bd)
    cp_rel = nnc.reconstruct_residual(dev(X), C)
    assert abs(cp_rel - ref["cp_rel"]) <= 1e-3


def test_objective_monotone_and_history():
    nnc = need_gpu()
    X, _, G0, A0 = problem(5, (30, 26, 22), 4, (4, 4, 4))
    G, A, rep = _fit_gpu(nnc, X, G0, A0, 60, objective_every=1)
    h = np.array(rep.history)
    assert len(h) == 60
    f = 0.5 * h ** 2
    assert (np.diff(f) <= 1e-6 * f[0]).all()


def test_tucker_fixed_point_bit_exact():
    """At an exact integer factorization num = den, so a GPU sweep changes nothing."""
    nnc = need_gpu()
    e = examples()["ex4_no_minimal_nntd"]
    X = fold(e["X_unfold1"], 0, e["dims"])
    H = fold(e["H_unfold1"], 0, e["H_dims"])
    A0 = [arr(e["W"]), np.eye(4), np.eye(3)]
    G, A, _ = _fit_gpu(nnc, X.astype(np.float32), H.astype(np.float32), [a.astype(np.float32) for a in A0], 4)
    assert np.array_equal(G, H) and all(np.array_equal(a, b) for a, b in zip(A, A0))


def test_bf16_form_matches_oracle_on_bf16_values():
    nnc = need_gpu()
    X64, _, G0, A0 = problem(7, (48, 40, 32), 3, (4, 4, 4), dtype="f64")
    Xb = synth.round_bf16(X64)
    G, A, rep = _fit_gpu(nnc, Xb, G0, A0, 20, dt="bf16")
    Go, Ao, _, _ = oracle.nntucker(Xb, G0, A0, 20)
    ref = oracle.tucker_rel_residual(Xb, Go, Ao)
    assert abs(rep.rel_residual - ref) <= 1e-3
    assert rel_fro(oracle.tucker_full(G, A), oracle.tucker_full(Go, Ao)) <= 1e-3


def test_bf16_with_fp32_refinement_sweeps():
    nnc = need_gpu()
    X, _, G0, A0 = problem(8, (48, 40, 32), 3, (4, 4, 4))
    Xb = bf16_dev(X.astype(np.float64))
    G = dev(G0)
    A = [dev(a) for a in A0]
    rep = nnc.nntucker_fit(Xb, G0.shape, 30, G, A, x_fp32=dev(X), fp32_final_sweeps=10)
    Go, Ao, _, _ = oracle.nntucker(X.astype(np.float64), G0, A0, 30)
    ref = oracle.tucker_rel_residual(X.astype(np.float64), Go, Ao)
    assert abs(rep.rel_residual - ref) <= 1e-3


def test_deterministic_bitwise():
    nnc = need_gpu()
    X, _, G0, A0 = problem(9, (33, 40, 24), 3, (5, 4, 3))
    G1, A1, r1 = _fit_gpu(nnc, X, G0, A0, 10)
    G2, A2, r2 = _fit_gpu(nnc, X, G0, A0, 10)
    assert np.array_equal(G1, G2) and all(np.array_equal(a, b) for a, b in zip(A1, A2))
    assert r1.rel_residual == r2.rel_residual


def test_resume_equals_continuous():
    nnc = need_gpu()
    X, _, G0, A0 = problem(10, (30, 20, 26), 3, (3, 4, 3))
    G1, A1, _ = _fit_gpu(nnc, X, G0, A0, 8)
    Xd = dev(X)
    G = dev(G0)
    A = [dev(a) for a in A0]
    nnc.nntucker_fit(Xd, G0.shape, 5, G, A)
    nnc.nntucker_fit(Xd, G0.shape, 3, G, A)
    assert np.array_equal(host(G), G1) and all(np.array_equal(host(a), b) for a, b in zip(A, A1))


@pytest.mark.parametrize("dims,ranks", [((12, 10, 9, 8), (3, 4, 2, 5)), ((9, 8, 7, 6, 5), (2, 3, 2, 3, 2)),
                                        ((30, 20, 26), (3, 4, 3))])
def test_graph_replays_match_eager_sweeps(dims, ranks):
    """The general schedule (FP32 X; orders 3 to 5) replayed from captured graphs (several
    sweeps per graph and a remainder graph) gives the eager sweeps' results bit for bit."""
    nnc = need_gpu()
    X, _, G0, A0 = problem(12, dims, 2, ranks)
    out = [_fit_gpu(nnc, X, G0, A0, 11, use_graph=g) for g in (False, True)]
    (Ge, Ae, re_), (Gg, Ag, rg) = out
    assert np.array_equal(Ge, Gg) and all(np.array_equal(a, b) for a, b in zip(Ae, Ag))
    assert re_.rel_residual == rg.rel_residual


def test_cached_sweep_graphs_follow_buffers_and_settings():
    """Graph fits that repeat an earlier fit's buffers and sizes replay its cached graphs: new
    contents written into the same buffers are read, a least-squares fit on the same buffers
    and another eps take graphs of their own, and more configurations than the cache keeps
    (20 X buffers, several sweep counts) still give the eager sweeps' results bit for bit."""
    nnc = need_gpu()
    dims, ranks = (30, 20, 26), (3, 4, 3)
    size = int(np.prod(dims))
    ws = torch.empty(nnc.nntucker_workspace_bytes(dims, ranks), dtype=torch.uint8, device="cuda")
    xbuf = torch.empty(20 * size, device="cuda")
    G = torch.empty(ranks, device="cuda")
    A = [torch.empty(n, r, device="cuda") for n, r in zip(dims, ranks)]

    def run(fit, slot, X, G0, A0, iters, use_graph, **kw):
        Xd = xbuf[slot * size:(slot + 1) * size].view(dims)
        Xd.copy_(torch.from_numpy(X))
        G.copy_(torch.from_numpy(G0))
        for a, a0 in zip(A, A0):
            a.copy_(torch.from_numpy(a0))
        fit(Xd, ranks, iters, G, A, use_graph=use_graph, workspace=ws, report=False, **kw)
        return host(G), [host(a) for a in A]

    cases = [(nnc.nntucker_fit, 0, 31, 11, {}), (nnc.nntucker_fit, 0, 32, 11, {}),
             (nnc.tucker_ls_fit, 0, 32, 11, {}), (nnc.nntucker_fit, 0, 32, 11, {"eps": 1e-3}),
             (nnc.nntucker_fit, 0, 33, 11, {})]
    cases += [(nnc.nntucker_fit, slot, 40 + slot, 5 + slot % 7, {}) for slot in range(20)]
    cases += [(nnc.nntucker_fit, 3, 70, 13, {}), (nnc.tucker_ls_fit, 3, 71, 9, {})]
    for fit, slot, seed, iters, kw in cases:
        X, _, G0, A0 = problem(seed, dims, 2, ranks)
        Ge, Ae = run(fit, slot, X, G0, A0, iters, False, **kw)
        Gg, Ag = run(fit, slot, X, G0, A0, iters, True, **kw)
        assert np.array_equal(Ge, Gg) and all(np.array_equal(a, b) for a, b in zip(Ae, Ag)), \
            (fit.__name__, slot, seed, iters, kw)


def test_nan_in_x_is_reported():
    nnc = need_gpu()
    X, _, G0, A0 = problem(11, (16, 16, 16), 2, (2, 2, 2))
    X = X.copy()
    X[3, 4, 5] = np.nan
    with pytest.raises(nnc.NncError) as ei:
        _fit_gpu(nnc, X, G0, A0, 2)
    assert ei.value.status == nnc.NNC_ENUMERIC


def test_zero_iterations_reports_init_residual():
    nnc = need_gpu()
    X, _, G0, A0 = problem(12, (20, 18, 16), 2, (3, 3, 3))
    G, A, rep = _fit_gpu(nnc, X, G0, A0, 0)
    assert np.array_equal(G, G0)
    assert abs(rep.rel_residual - oracle.tucker_rel_residual(X.astype(np.float64), G0, A0)) <= 1e-6


# ------------------------------------------------------------------------------ residual / lift
@pytest.mark.parametrize("dims,ranks", [((40, 33, 27), (5, 4, 6)), ((9, 8, 7, 6), (2, 3, 4, 2)),
                                        ((64, 50), (7, 3))])
def test_residuals_match_oracle(dims, ranks):
    nnc = need_gpu()
    X, _, G0, A0 = problem(13, dims, 3, ranks)
    X64 = X.astype(np.float64)
    r = nnc.reconstruct_residual(dev(X), [dev(a) for a in A0], dev(G0))
    assert abs(r - oracle.tucker_rel_residual(X64, G0, A0)) <= 1e-6 * max(1.0, r)
    C = synth.init_cp_factors(13, dims, 4)
    rc = nnc.reconstruct_residual(dev(X), [dev(c) for c in C])
    assert abs(rc - oracle.cp_rel_residual(X64, C)) <= 1e-6 * max(1.0, rc)
    Xb = synth.round_bf16(X64)
    rb = nnc.reconstruct_residual(bf16_dev(Xb), [dev(a) for a in A0], dev(G0))
    assert abs(rb - oracle.tucker_rel_residual(Xb, G0, A0)) <= 1e-6 * max(1.0, rb)


def test_lift_bit_exact_on_integers():
    nnc = need_gpu()
    rng = np.random.default_rng(14)
    A = [rng.integers(0, 5, size=(n, m)).astype(np.float32) for n, m in [(30, 4), (17, 3), (9, 5)]]
    B = [rng.integers(0, 5, size=(m, 6)).astype(np.float32) for m in (4, 3, 5)]
    C = nnc.nncandelinc_lift([dev(a) for a in A], [dev(b) for b in B])
    for c, a, b in zip(C, A, B):
        assert np.array_equal(host(c), a.astype(np.float64) @ b.astype(np.float64))


# ------------------------------------------------------------------------------ nnCP
@pytest.mark.parametrize("core_dims,r", [((5, 5, 5), 3), ((20, 20, 20), 10), ((8, 7, 6, 5), 4),
                                         ((8, 8, 8, 8, 8), 6), ((12, 9), 5)])
def test_nncp_matches_oracle(core_dims, r):
    nnc = need_gpu()
    rng = np.random.default_rng(15)
    T = (oracle.cp_full([rng.random((n, r)) for n in core_dims]) + 1e-3 * rng.random(core_dims)).astype(np.float32)
    B0 = synth.init_cp_factors(15, core_dims, r)
    Bd = [dev(b) for b in B0]
    rel = nnc.nncp_fit(dev(T), r, 5, Bd)
    Bo, _, _ = oracle.nncp(T.astype(np.float64), B0, 5)
    for b, bo in zip(Bd, Bo):
        assert rel_fro(host(b), bo) <= 1e-4
    assert abs(rel - oracle.cp_rel_residual(T.astype(np.float64), Bo)) <= 1e-5
    Bd = [dev(b) for b in B0]
    rel = nnc.nncp_fit(dev(T), r, 200, Bd)
    Bo, _, _ = oracle.nncp(T.astype(np.float64), B0, 200)
    assert abs(rel - oracle.cp_rel_residual(T.astype(np.float64), Bo)) <= 1e-3


def test_nncp_fixed_point_bit_exact():
    nnc = need_gpu()
    e = examples()["ex5_rank_not_preserved_nn"]
    B0 = [arr(e["A1"]).astype(np.float32), arr(e["A2"]).astype(np.float32), arr(e["A3"]).astype(np.float32)]
    T = oracle.cp_full(B0).astype(np.float32)
    Bd = [dev(b) for b in B0]
    rel = nnc.nncp_fit(dev(T), 4, 5, Bd)
    assert rel == 0.0 and all(np.array_equal(host(b), b0) for b, b0 in zip(Bd, B0))


def test_batched_nncp_uneven_ranks():
    nnc = need_gpu()
    rng = np.random.default_rng(16)
    core_dims = (8, 8, 8, 8, 8)
    T = (oracle.cp_full([rng.random((8, 6)) for _ in range(5)]) + 1e-3 * rng.random(core_dims)).astype(np.float32)
    ranks = [2 + (j % 15) for j in range(20)]
    inits = [synth.init_cp_factors(16, core_dims, r, restart=j) for j, r in enumerate(ranks)]
    facs = [[dev(b) for b in B0] for B0 in inits]
    res = nnc.nncp_fit_batched(dev(T), ranks, 30, facs)
    for j in (0, 7, 14, 19):
        Bo, _, _ = oracle.nncp(T.astype(np.float64), inits[j], 30)
        assert abs(res[j] - oracle.cp_rel_residual(T.astype(np.float64), Bo)) <= 1e-4
        for b, bo in zip(facs[j], Bo):
            assert rel_fro(host(b), bo) <= 1e-3
    # a batched fit equals the same fit launched alone with the same threads per fit
    threads = nnc.last_tune()["threads"]
    single = [dev(b) for b in inits[3]]
    r1 = nnc.nncp_fit_batched(dev(T), [ranks[3]], 30, [single], threads_per_fit=threads)
    assert r1[0] == res[3] and all(np.array_equal(host(a), host(b)) for a, b in zip(single, facs[3]))


def _device_tag():
    p = torch.cuda.get_device_properties(0)
    return "%s/%dcu" % (p.gcnArchName.split(":")[0], p.multi_processor_count)


def test_batched_tuner_persists_and_reuses(tmp_path, monkeypatch):
    """The tuner measures once per (device, core shape, rank multiset), writes its choice to
    the cache file, reuses it (same results bit for bit), and takes a choice found in a file."""
    nnc = need_gpu()
    path = tmp_path / "tune.json"
    monkeypatch.setenv("NNC_TUNE_CACHE", str(path))
    rng = np.random.default_rng(161)
    core_dims = (7, 9, 8)
    T = dev((oracle.cp_full([rng.random((n, 4)) for n in core_dims]) + 1e-3 * rng.random(core_dims)).astype(np.float32))
    ranks = [3, 5, 5, 9]
    inits = [synth.init_cp_factors(161, core_dims, r, restart=j) for j, r in enumerate(ranks)]
    f1 = [[dev(b) for b in B0] for B0 in inits]
    r1 = nnc.nncp_fit_batched(T, ranks, 20, f1)
    c1 = nnc.last_tune()
    assert c1["source"] == "measured" and c1["threads"] in (256, 512, 1024), c1
    key = "%s|7x9x8|3,5,5,9" % _device_tag()
    lines = path.read_text().splitlines()
    assert any(('"key": "%s"' % key) in l and ('"threads": %d' % c1["threads"]) in l for l in lines), lines
    f2 = [[dev(b) for b in B0] for B0 in inits]
    r2 = nnc.nncp_fit_batched(T, ranks[::-1], 20, f2[::-1])  # same multiset, other order
    c2 = nnc.last_tune()
    assert c2["source"] == "cache" and c2["threads"] == c1["threads"], c2
    assert r2[::-1] == r1
    assert all(np.array_equal(host(a), host(b)) for fa, fb in zip(f1, f2) for a, b in zip(fa, fb))
    # a choice written to another file is picked up when the path changes
    path2 = tmp_path / "other.json"
    path2.write_text('{"key": "%s|6x6x6|2,4", "threads": 320, "t_global": 0, "lpt": 0, "ms": 1.0}\n' % _device_tag())
    monkeypatch.setenv("NNC_TUNE_CACHE", str(path2))
    T3 = dev(rng.random((6, 6, 6)).astype(np.float32))
    f3 = [[dev(b) for b in synth.init_cp_factors(162, (6, 6, 6), r, restart=j)] for j, r in enumerate([4, 2])]
    nnc.nncp_fit_batched(T3, [4, 2], 10, f3)
    c3 = nnc.last_tune()
    assert c3["source"] == "cache" and c3["threads"] == 320, c3


# ------------------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("dims,ranks", [((24, 20, 18), (4, 5, 3)),
                                        # cores beyond the whole-core kernels; factor rows
                                        # with the contracted index split over blocks
                                        ((20, 18, 17, 19), (16, 16, 16, 16)),
                                        ((10, 9, 8, 9, 10), (8, 8, 8, 8, 8)),
                                        ((40, 36, 34), (32, 32, 32))])
def test_gradient_matches_oracle(dims, ranks):
    nnc = need_gpu()
    print("case", dims, ranks, flush=True)
    X, _, G0, A0 = problem(17, dims, 3, ranks)
    L, gG, gA = nnc.nntucker_grad(dev(X), dev(G0), [dev(a) for a in A0])
    Lo, gGo, gAo = oracle.tucker_grad(X.astype(np.float64), G0, A0)
    assert abs(L - Lo) <= 1e-6 * Lo
    assert rel_fro(host(gG), gGo) <= 1e-4
    for g, go in zip(gA, gAo):
        assert rel_fro(host(g), go) <= 1e-4


def test_autograd_function():
    nnc = need_gpu()
    X, _, G0, A0 = problem(18, (16, 14, 12), 3, (3, 4, 2))
    G = dev(G0).requires_grad_(True)
    A = [dev(a).requires_grad_(True) for a in A0]
    loss = nnc.nntucker_loss(dev(X), G, A)
    loss.backward()
    Lo, gGo, gAo = oracle.tucker_grad(X.astype(np.float64), G0, A0)
    assert abs(loss.item() - Lo) <= 1e-6 * Lo
    assert rel_fro(host(G.grad), gGo) <= 1e-4
    for a, go in zip(A, gAo):
        assert rel_fro(host(a.grad), go) <= 1e-4
