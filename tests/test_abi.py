"""The C ABI on the CPU: every declared symbol is exported, and argument validation runs
before any HIP call, so invalid calls return the documented status without a GPU."""
import ctypes
import os
import re

import pytest

import paper_1909_07570_amd as nnc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nncandelinc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 15, names
    L = nnc.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(nnc.EXPORTED)


def D(*xs):
    return (ctypes.c_int64 * len(xs))(*xs)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _ptrs(n, null_at=None):
    return (ctypes.c_void_p * n)(*[None if i == null_at else 0x1000 for i in range(n)])


def test_workspace_queries():
    L = nnc.lib()
    b = L.nntucker_workspace_bytes(3, D(512, 512, 512), D(20, 20, 20))
    assert b >= 4 * (512 * 512 * 20 * 2)
    assert L.nntucker_workspace_bytes(1, D(5), D(5)) == 0
    assert L.nntucker_workspace_bytes(3, D(5, 0, 5), D(2, 2, 2)) == 0
    assert L.reconstruct_workspace_bytes(3, D(8, 8, 8), D(3, 0, 0), 1) > 0
    assert L.nncp_workspace_bytes(3, D(5, 5, 5), 3) > 0


def test_nntucker_fit_validation():
    L = nnc.lib()
    opt = nnc.Options()
    opt.workspace = 0x1000
    opt.workspace_bytes = 1 << 40
    f = L.nntucker_fit
    assert f(FAKE, 0, 1, D(4), D(2), 1, FAKE, _ptrs(1), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 9, D(*[2] * 9), D(*[2] * 9), 1, FAKE, _ptrs(9), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(None, 0, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3, 1), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert "factors[1]" in nnc.last_error()
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 0, 2), 1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), -1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 7, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    # refinement sweeps need bf16 X and an fp32 copy
    o2 = nnc.Options()
    o2.workspace, o2.workspace_bytes, o2.fp32_final_sweeps = 0x1000, 1 << 40, 5
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), 10, FAKE, _ptrs(3), ctypes.byref(o2), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 1, 3, D(4, 4, 4), D(2, 2, 2), 10, FAKE, _ptrs(3), ctypes.byref(o2), None, None) == nnc.NNC_EINVAL
    # workspace
    o3 = nnc.Options()
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3), ctypes.byref(o3), None, None) == nnc.NNC_EWORKSPACE
    o3.workspace, o3.workspace_bytes = 0x1000, 16
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3), ctypes.byref(o3), None, None) == nnc.NNC_EWORKSPACE
    # unsupported multirank
    assert f(FAKE, 0, 3, D(400, 4, 4), D(300, 2, 2), 1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EUNSUPPORTED


def test_other_entry_points_validate():
    L = nnc.lib()
    assert L.nnc_ttm(FAKE, 0, 3, D(4, 4, 4), 3, FAKE, 2, FAKE, None) == nnc.NNC_EINVAL
    assert L.nnc_ttm(FAKE, 0, 3, D(4, 4, 4), 0, FAKE, 0, FAKE, None) == nnc.NNC_EINVAL
    assert L.nnc_ttm(FAKE, 2, 3, D(4, 4, 4), 0, FAKE, 2, FAKE, None) == nnc.NNC_EINVAL
    assert L.nnc_convert_f32_bf16(None, FAKE, 4, None) == nnc.NNC_EINVAL
    assert L.nnc_convert_f32_bf16(FAKE, FAKE, -1, None) == nnc.NNC_EINVAL
    wopt = nnc.Options()
    wopt.workspace = 0x1000
    wopt.workspace_bytes = 1 << 20
    W = ctypes.byref(wopt)
    assert L.nncp_fit(FAKE, 3, D(5, 5, 5), 0, 10, _ptrs(3), W, None, None) == nnc.NNC_EINVAL
    assert L.nncp_fit(FAKE, 3, D(5, 5, 5), 3, 10, _ptrs(3, 2), W, None, None) == nnc.NNC_EINVAL
    assert L.nncp_fit(FAKE, 3, D(5, 5, 5), 3, 10, _ptrs(3), None, None, None) == nnc.NNC_EWORKSPACE
    assert L.nncp_fit(FAKE, 3, D(5, 5, 5), 65, 10, _ptrs(3), W, None, None) == nnc.NNC_EUNSUPPORTED
    neg = nnc.Options()
    neg.eps = -1.0
    neg.workspace = 0x1000
    neg.workspace_bytes = 1 << 20
    assert L.nncp_fit(FAKE, 3, D(5, 5, 5), 3, 10, _ptrs(3), ctypes.byref(neg), None, None) == nnc.NNC_EINVAL
    rk = (ctypes.c_int * 2)(3, 40)
    res = (ctypes.c_double * 2)()
    assert L.nncp_fit_batched(FAKE, 3, D(5, 5, 5), 2, rk, 10, _ptrs(6), 0.0, res, 0, FAKE, 1 << 20, None) == nnc.NNC_EUNSUPPORTED
    rk0 = (ctypes.c_int * 2)(3, 0)
    assert L.nncp_fit_batched(FAKE, 3, D(5, 5, 5), 2, rk0, 10, _ptrs(6), 0.0, res, 0, FAKE, 1 << 20, None) == nnc.NNC_EINVAL
    rk1 = (ctypes.c_int * 2)(3, 4)
    assert L.nncp_fit_batched(FAKE, 3, D(5, 5, 5), 2, rk1, 10, _ptrs(6), 0.0, res, 100, FAKE, 1 << 20, None) == nnc.NNC_EINVAL
    assert L.nncandelinc_lift(3, D(4, 4, 4), D(2, 2, 2), 0, _ptrs(3), _ptrs(3), _ptrs(3), None) == nnc.NNC_EINVAL
    assert L.nncandelinc_lift(3, D(4, 4, 4), D(2, 2, 2), 2, _ptrs(3), _ptrs(3, 0), _ptrs(3), None) == nnc.NNC_EINVAL
    r = ctypes.c_double()
    assert L.reconstruct_residual(FAKE, 0, 3, D(4, 4, 4), None, D(0, 0, 0), _ptrs(3), ctypes.byref(r), FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert L.reconstruct_residual(FAKE, 0, 3, D(4, 4, 4), FAKE, D(2, 2, 2), _ptrs(3), None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert L.reconstruct_residual(FAKE, 0, 3, D(4, 4, 4), FAKE, D(2, 2, 2), _ptrs(3), ctypes.byref(r), FAKE, 8, None) == nnc.NNC_EWORKSPACE
    assert L.nntucker_grad(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), FAKE, _ptrs(3), None, _ptrs(3), None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert L.nntucker_grad(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), FAKE, _ptrs(3), FAKE, _ptrs(3), None, FAKE, 8, None) == nnc.NNC_EWORKSPACE


def test_algorithm2_entry_points_validate():
    L = nnc.lib()
    assert L.nncpx_workspace_bytes(3, D(40, 40, 40), 3) > 0
    assert L.nncpx_workspace_bytes(3, D(40, 40, 40), 33) == 0
    assert L.nmf_workspace_bytes(512, 10, 20) > 0
    assert L.nmf_workspace_bytes(512, 0, 20) == 0
    opt = nnc.Options()
    opt.workspace = 0x1000
    opt.workspace_bytes = 1 << 40
    f = L.nncpx_fit
    assert f(None, 0, 3, D(4, 4, 4), 2, 1, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(4, 4, 4), 2, 1, _ptrs(3, 2), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert "factors[2]" in nnc.last_error()
    assert f(FAKE, 0, 3, D(4, 0, 4), 2, 1, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(4, 4, 4), 0, 1, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(4, 4, 4), 33, 1, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EUNSUPPORTED
    assert f(FAKE, 0, 3, D(4, 4, 4), 2, -1, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 5, 3, D(4, 4, 4), 2, 1, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    o2 = nnc.Options()
    o2.workspace, o2.workspace_bytes, o2.fp32_final_sweeps = 0x1000, 1 << 40, 5
    assert f(FAKE, 0, 3, D(4, 4, 4), 2, 10, _ptrs(3), ctypes.byref(o2), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 1, 3, D(4, 4, 4), 2, 10, _ptrs(3), ctypes.byref(o2), None, None) == nnc.NNC_EINVAL
    o3 = nnc.Options()
    assert f(FAKE, 0, 3, D(4, 4, 4), 2, 1, _ptrs(3), ctypes.byref(o3), None, None) == nnc.NNC_EWORKSPACE
    o3.workspace, o3.workspace_bytes = 0x1000, 16
    assert f(FAKE, 0, 3, D(4, 4, 4), 2, 1, _ptrs(3), ctypes.byref(o3), None, None) == nnc.NNC_EWORKSPACE
    g = L.nmf_fit
    assert g(None, 8, 3, 2, 5, FAKE, FAKE, 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert g(FAKE, 8, 3, 2, 5, None, FAKE, 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert g(FAKE, 0, 3, 2, 5, FAKE, FAKE, 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert g(FAKE, 8, 3, 0, 5, FAKE, FAKE, 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert g(FAKE, 8, 3, 40, 5, FAKE, FAKE, 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EUNSUPPORTED
    assert g(FAKE, 8, 3, 2, -2, FAKE, FAKE, 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert g(FAKE, 8, 3, 2, 5, FAKE, FAKE, -1.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert g(FAKE, 8, 3, 2, 5, FAKE, FAKE, 0.0, None, FAKE, 8, None) == nnc.NNC_EWORKSPACE
    h = L.nmf_fit_batched
    rk = (ctypes.c_int * 2)(2, 3)
    assert L.nmf_batched_workspace_bytes(2, D(8, 9), 3, rk) > 0
    assert h(0, _ptrs(2), D(8, 9), 3, rk, 5, _ptrs(2), _ptrs(2), 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert h(2, _ptrs(2, 1), D(8, 9), 3, rk, 5, _ptrs(2), _ptrs(2), 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    assert h(2, _ptrs(2), D(8, 0), 3, rk, 5, _ptrs(2), _ptrs(2), 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EINVAL
    rk40 = (ctypes.c_int * 2)(2, 40)
    assert h(2, _ptrs(2), D(8, 9), 3, rk40, 5, _ptrs(2), _ptrs(2), 0.0, None, FAKE, 1 << 30, None) == nnc.NNC_EUNSUPPORTED
    assert h(2, _ptrs(2), D(8, 9), 3, rk, 5, _ptrs(2), _ptrs(2), 0.0, None, FAKE, 8, None) == nnc.NNC_EWORKSPACE


def test_restart_study_validates():
    L = nnc.lib()
    assert L.nncandelinc_restart_init_floats(1, D(4, 4, 4), D(4, 4, 4), 4) == 160
    assert L.nncandelinc_restart_init_floats(2, D(4, 4, 4), D(3, 4, 4), 4) == 136
    assert L.nncandelinc_restart_init_floats(3, D(4, 4, 4), D(3, 4, 4), 4) == 0
    f = L.nncandelinc_restarts
    ok = dict(X=FAKE, dims=D(4, 4, 4), alg=1, m=D(3, 3, 3), r=4, n=8, o=10, i=10, inits=FAKE, truth=None,
              eps=0.0, rel=FAKE, cong=None, lifted=None, clips=None)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["X"], a["dims"], a["alg"], a["m"], a["r"], a["n"], a["o"], a["i"], a["inits"], a["truth"],
                 a["eps"], a["rel"], a["cong"], a["lifted"], a["clips"], None)
    assert call(X=None) == nnc.NNC_EINVAL
    assert call(rel=None) == nnc.NNC_EINVAL
    assert call(alg=3) == nnc.NNC_EINVAL
    assert call(r=0) == nnc.NNC_EINVAL
    assert call(n=-1) == nnc.NNC_EINVAL
    assert call(o=-1) == nnc.NNC_EINVAL
    assert call(eps=-1.0) == nnc.NNC_EINVAL
    assert call(dims=D(4, 0, 4)) == nnc.NNC_EINVAL
    assert call(truth=_ptrs(3)) == nnc.NNC_EINVAL          # truth without congruences
    assert call(truth=_ptrs(3, 1), cong=FAKE) == nnc.NNC_EINVAL
    assert call(dims=D(9, 4, 4)) == nnc.NNC_EUNSUPPORTED
    assert call(m=D(3, 9, 3)) == nnc.NNC_EUNSUPPORTED
    assert call(r=9) == nnc.NNC_EUNSUPPORTED
    assert call(n=0) == nnc.NNC_OK                        # nothing to launch
    assert call(n=0, X=None, inits=None, rel=None) == nnc.NNC_OK
    assert call(n=0, dims=D(9, 4, 4)) == nnc.NNC_EUNSUPPORTED


def test_binding_rejects_cpu_tensors():
    import torch
    with pytest.raises(ValueError):
        nnc.nnc_ttm(torch.zeros(4, 4, 4), 0, torch.zeros(4, 2))


def test_nncp_refuses_index_ranges_past_2_22():
    """The nnCP kernel splits loop indices with a float-reciprocal division that is exact
    below 2^22; cores whose index ranges reach it are refused before any HIP call."""
    L = nnc.lib()
    big = nnc.Options()
    big.workspace = 0x1000
    big.workspace_bytes = 1 << 40
    B = ctypes.byref(big)
    # 256 x 256 x 256 x 4 core at rank 4: the first updates contract mode 3 and run
    # ceil(4/4) * 2^26 / 4 = 2^24 items
    st = L.nncp_fit(FAKE, 4, D(256, 256, 256, 4), 4, 10, _ptrs(4), B, None, None)
    assert st == nnc.NNC_EUNSUPPORTED, st
    assert "2^22" in nnc.last_error()
    rk = (ctypes.c_int * 2)(4, 2)
    res = (ctypes.c_double * 2)()
    st = L.nncp_fit_batched(FAKE, 4, D(256, 256, 256, 4), 2, rk, 10, _ptrs(8), 0.0, res, 0, FAKE, 1 << 40, None)
    assert st == nnc.NNC_EUNSUPPORTED, st
    # a mode of 2^20 rows at rank 4 reaches the limit in the update's pairs
    st = L.nncp_fit(FAKE, 2, D(1 << 20, 2), 4, 10, _ptrs(2), B, None, None)
    assert st == nnc.NNC_EUNSUPPORTED, st


def test_qdiv_float_reciprocal_division_exact_below_2_22():
    """Brute force of the kernels' index division (a + 0.5) * RN(1/b) truncated, in IEEE
    float32 with round-to-nearest-even, against integer division for every a < 2^22 and
    a spread of divisors b (all of 1..96, then sampled up to 2^22)."""
    import numpy as np
    a = np.arange(1 << 22, dtype=np.int64)
    af = a.astype(np.float32) + np.float32(0.5)
    rng = np.random.default_rng(22)
    bs = list(range(1, 97)) + [int(b) for b in rng.integers(97, 1 << 22, 40)] + [(1 << 22) - 1, 4093, 65521]
    for b in bs:
        inv = np.float32(1.0) / np.float32(b)
        q = (af * inv).astype(np.int64)
        assert np.array_equal(q, a // b), b


def test_nncp_noalloc_validation():
    L = nnc.lib()
    assert L.nncp_noalloc_max_scratch_bytes() == 8 << 20
    assert L.nncp_fit_noalloc(None, 3, D(5, 5, 5), 3, 10, _ptrs(3), None, None, None) == nnc.NNC_EINVAL
    assert L.nncp_fit_noalloc(FAKE, 3, D(5, 5, 5), 3, -1, _ptrs(3), None, None, None) == nnc.NNC_EINVAL
    assert L.nncp_fit_noalloc(FAKE, 3, D(5, 5, 5), 40, 10, _ptrs(3), None, None, None) == nnc.NNC_EUNSUPPORTED
    # 64 x 64 x 64 x 16 at rank 32: the contraction scratch alone is 2^16 rows x 32 floats =
    # 8 MiB, so the total is above the maximum
    assert L.nncp_workspace_bytes(4, D(64, 64, 64, 16), 32) > (8 << 20)
    st = L.nncp_fit_noalloc(FAKE, 4, D(64, 64, 64, 16), 32, 10, _ptrs(4), None, None, None)
    assert st == nnc.NNC_EUNSUPPORTED and "static maximum" in nnc.last_error()


def test_fill_uniform_validation():
    L = nnc.lib()
    assert L.nnc_fill_uniform(1, 2, None, 4, None) == nnc.NNC_EINVAL
    assert L.nnc_fill_uniform(1, 2, FAKE, -1, None) == nnc.NNC_EINVAL
    assert L.nnc_fill_uniform(1, 2, None, 0, None) == nnc.NNC_OK
    assert L.nnc_fill_uniform_f64(1, 2, -1, FAKE, 4, None) == nnc.NNC_EINVAL
    assert L.nnc_fill_uniform_f64(1, 2, 0, None, 4, None) == nnc.NNC_EINVAL


def test_real_valued_fits_validate():
    """The least-squares fits share the nonnegative fits' checks, with ranks capped at 32."""
    L = nnc.lib()
    opt = nnc.Options()
    opt.workspace = 0x1000
    opt.workspace_bytes = 1 << 40
    f = L.tucker_ls_fit
    assert L.tucker_ls_workspace_bytes(3, D(64, 48, 40), D(5, 6, 7)) == L.nntucker_workspace_bytes(
        3, D(64, 48, 40), D(5, 6, 7)) > 0
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3, 2), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(40, 40, 40), D(33, 2, 2), 1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EUNSUPPORTED
    assert "above 32" in nnc.last_error()
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), -1, FAKE, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert f(FAKE, 0, 3, D(4, 4, 4), D(2, 2, 2), 1, FAKE, _ptrs(3), None, None, None) == nnc.NNC_EWORKSPACE
    g = L.cp_ls_fit
    assert L.cp_ls_workspace_bytes(3, D(5, 5, 5), 3) == L.nncp_workspace_bytes(3, D(5, 5, 5), 3) > 0
    assert g(FAKE, 3, D(5, 5, 5), 0, 10, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert g(FAKE, 3, D(5, 5, 5), 33, 10, _ptrs(3), ctypes.byref(opt), None, None) == nnc.NNC_EUNSUPPORTED
    assert g(FAKE, 3, D(5, 5, 5), 3, 10, _ptrs(3, 0), ctypes.byref(opt), None, None) == nnc.NNC_EINVAL
    assert g(FAKE, 3, D(5, 5, 5), 3, 10, _ptrs(3), None, None, None) == nnc.NNC_EWORKSPACE


def test_bench_refuses_more_than_one_gpu_and_needs_the_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so; without a GPU it
    exits with status 1 and names what it needs (no CPU stand-in is timed)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)
    import torch
    if not torch.cuda.is_available():
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "0"],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 1 and "needs an MI355X" in (r.stderr + r.stdout), (r.returncode, r.stderr)
        assert not r.stdout.lstrip().startswith("{")
