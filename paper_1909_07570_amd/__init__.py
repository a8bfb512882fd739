"""Python binding of libnncandelinc (include/nncandelinc.h): nonnegative CANDELINC on
AMD Instinct MI355X (gfx950), computed as Algorithm 1 of arXiv 1909.07570 -- a nonnegative
Tucker compression by multiplicative updates, a nonnegative CP of the core, and the lift
of the CP factors through the Tucker factors (Section 4.1).

The binding only marshals arguments: torch tensors provide device memory and the current
stream; every step runs in the library's HIP kernels.  There is no CPU fallback: if the
shared library is missing or no gfx950 device is visible, calls raise.

Names follow the paper: X the data tensor, A_n (= F^(n)) the Tucker factors, G the core,
B_n the CP factors of the core, C_n = A_n B_n the lifted (constrained) CP factors.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnncandelinc.so")

NNC_OK, NNC_EINVAL, NNC_EUNSUPPORTED, NNC_EWORKSPACE, NNC_EHIP, NNC_ENUMERIC = 0, -1, -2, -3, -4, -5
NNC_F32, NNC_BF16 = 0, 1
STATUS_NAMES = {0: "NNC_OK", -1: "NNC_EINVAL", -2: "NNC_EUNSUPPORTED", -3: "NNC_EWORKSPACE",
                -4: "NNC_EHIP", -5: "NNC_ENUMERIC"}

_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p
_vpp = ctypes.POINTER(ctypes.c_void_p)
_dp = ctypes.POINTER(ctypes.c_double)


class NncError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("fp32_final_sweeps", ctypes.c_int), ("x_fp32", _vp), ("eps", ctypes.c_double),
                ("objective_every", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t)]


class Report(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("eps_clips", ctypes.c_longlong), ("objective_history", _dp),
                ("history_len", ctypes.c_int), ("seconds", ctypes.c_double),
                ("ttm_pass_ms", ctypes.c_double), ("ttm_pass_launches", ctypes.c_longlong)]


EXPORTED = ["nnc_last_error", "nnc_device_ok", "nnc_set_timing", "nnc_ttm", "nnc_convert_f32_bf16",
            "nntucker_workspace_bytes", "nntucker_fit", "nncp_workspace_bytes", "nncp_fit",
            "nncp_batched_workspace_bytes", "nncp_fit_batched", "nncandelinc_lift",
            "reconstruct_workspace_bytes", "reconstruct_residual", "reconstruct_sq_sums",
            "nntucker_grad", "nncpx_workspace_bytes", "nncpx_fit", "nmf_workspace_bytes", "nmf_fit",
            "nmf_batched_workspace_bytes", "nmf_fit_batched", "nncandelinc_restart_init_floats",
            "nncandelinc_restarts", "nnc_mean_congruence", "nnc_fill_uniform", "nnc_fill_uniform_f64",
            "nncp_noalloc_max_scratch_bytes", "nncp_fit_noalloc", "tucker_ls_workspace_bytes",
            "tucker_ls_fit", "cp_ls_workspace_bytes", "cp_ls_fit", "nnc_last_pass_times", "nnc_last_ttm_kernel",
            "nnc_last_tune"]

_lib = None


def lib():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnncandelinc.so is not built; run `python -m paper_1909_07570_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.nnc_last_error.restype = ctypes.c_char_p
        L.nnc_device_ok.restype = ctypes.c_int
        L.nnc_set_timing.argtypes = [ctypes.c_int]
        L.nnc_last_pass_times.argtypes = [_dp, ctypes.POINTER(ctypes.c_longlong)]
        L.nnc_last_pass_times.restype = None
        L.nnc_last_ttm_kernel.argtypes = []
        L.nnc_last_ttm_kernel.restype = ctypes.c_char_p
        L.nnc_last_tune.argtypes = []
        L.nnc_last_tune.restype = ctypes.c_char_p
        L.nnc_ttm.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int, _vp, _i64, _vp, _vp]
        L.nnc_convert_f32_bf16.argtypes = [_vp, _vp, _i64, _vp]
        L.nnc_fill_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _vp, _i64, _vp]
        L.nnc_fill_uniform_f64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _i64, _vp, _i64, _vp]
        L.nntucker_workspace_bytes.argtypes = [ctypes.c_int, _i64p, _i64p]
        L.nntucker_workspace_bytes.restype = ctypes.c_size_t
        L.nntucker_fit.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64p, _i64p, ctypes.c_int, _vp,
                                   _vpp, ctypes.POINTER(Options), ctypes.POINTER(Report), _vp]
        L.tucker_ls_workspace_bytes.argtypes = [ctypes.c_int, _i64p, _i64p]
        L.tucker_ls_workspace_bytes.restype = ctypes.c_size_t
        L.tucker_ls_fit.argtypes = L.nntucker_fit.argtypes
        L.cp_ls_workspace_bytes.argtypes = [ctypes.c_int, _i64p, ctypes.c_int]
        L.cp_ls_workspace_bytes.restype = ctypes.c_size_t
        L.cp_ls_fit.argtypes = [_vp, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _vpp,
                                ctypes.POINTER(Options), ctypes.POINTER(Report), _vp]
        L.nncp_workspace_bytes.argtypes = [ctypes.c_int, _i64p, ctypes.c_int]
        L.nncp_workspace_bytes.restype = ctypes.c_size_t
        L.nncp_fit.argtypes = [_vp, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _vpp,
                               ctypes.POINTER(Options), ctypes.POINTER(Report), _vp]
        L.nncp_noalloc_max_scratch_bytes.argtypes = []
        L.nncp_noalloc_max_scratch_bytes.restype = ctypes.c_size_t
        L.nncp_fit_noalloc.argtypes = [_vp, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _vpp,
                                       ctypes.POINTER(Options), ctypes.POINTER(Report), _vp]
        L.nncp_batched_workspace_bytes.argtypes = [ctypes.c_int, _i64p, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_int)]
        L.nncp_batched_workspace_bytes.restype = ctypes.c_size_t
        L.nncp_fit_batched.argtypes = [_vp, ctypes.c_int, _i64p, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int), ctypes.c_int, _vpp,
                                       ctypes.c_double, _dp, ctypes.c_int, _vp, ctypes.c_size_t, _vp]
        L.nncpx_workspace_bytes.argtypes = [ctypes.c_int, _i64p, ctypes.c_int]
        L.nncpx_workspace_bytes.restype = ctypes.c_size_t
        L.nncpx_fit.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _vpp,
                                _vp, _vp, _vp]
        L.nmf_workspace_bytes.argtypes = [_i64, _i64, ctypes.c_int]
        L.nmf_workspace_bytes.restype = ctypes.c_size_t
        L.nmf_fit.argtypes = [_vp, _i64, _i64, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_double, _vp,
                              _vp, ctypes.c_size_t, _vp]
        L.nmf_batched_workspace_bytes.argtypes = [ctypes.c_int, _i64p, _i64, ctypes.POINTER(ctypes.c_int)]
        L.nmf_batched_workspace_bytes.restype = ctypes.c_size_t
        L.nmf_fit_batched.argtypes = [ctypes.c_int, _vpp, _i64p, _i64, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                      _vpp, _vpp, ctypes.c_double, _dp, _vp, ctypes.c_size_t, _vp]
        L.nncandelinc_restart_init_floats.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int]
        L.nncandelinc_restart_init_floats.restype = ctypes.c_int64
        L.nncandelinc_restarts.argtypes = [_vp, _i64p, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, _vp, _vpp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
        L.nnc_mean_congruence.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, _vpp, _vpp, _vp, _vp]
        L.nncandelinc_lift.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, _vpp, _vpp, _vpp, _vp]
        L.reconstruct_workspace_bytes.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int]
        L.reconstruct_workspace_bytes.restype = ctypes.c_size_t
        L.reconstruct_residual.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64p, _vp, _i64p, _vpp,
                                           _dp, _vp, ctypes.c_size_t, _vp]
        L.reconstruct_sq_sums.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64p, _vp, _i64p, _vpp,
                                          _dp, _dp, _vp, ctypes.c_size_t, _vp]
        L.nntucker_grad.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64p, _i64p, _vp, _vpp, _vp,
                                    _vpp, _dp, _vp, ctypes.c_size_t, _vp]
        for name in EXPORTED:
            if name not in ("nnc_last_error", "nnc_device_ok", "nnc_set_timing", "nnc_last_pass_times",
                            "nnc_last_ttm_kernel", "nnc_last_tune") and \
                    not name.endswith("_bytes") and not name.endswith("_floats"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().nnc_last_error().decode()


def _check(status: int) -> None:
    if status != NNC_OK:
        raise NncError(status, last_error())


def _dims(seq):
    seq = [int(x) for x in seq]
    return (ctypes.c_int64 * len(seq))(*seq)


def _ptrs(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() if t is not None else None for t in tensors])


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, dtypes=(torch.float32,)) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype not in dtypes:
        raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _xdt(X: torch.Tensor) -> int:
    if X.dtype == torch.float32:
        return NNC_F32
    if X.dtype == torch.bfloat16:
        return NNC_BF16
    raise ValueError("X must be float32 or bfloat16")


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def set_timing(on: bool) -> None:
    lib().nnc_set_timing(1 if on else 0)


def last_tune() -> dict:
    """The launch configuration of this thread's last nncp_fit_batched."""
    import json
    return json.loads(lib().nnc_last_tune().decode())


def last_ttm_kernel() -> str:
    """The kernel this thread's last nnc_ttm launched."""
    return lib().nnc_last_ttm_kernel().decode()


def last_pass_times():
    """((ms of pass 1, launches), (ms of pass 2, launches)) of this thread's last timed fit."""
    ms = (ctypes.c_double * 2)()
    n = (ctypes.c_longlong * 2)()
    lib().nnc_last_pass_times(ms, n)
    return (ms[0], n[0]), (ms[1], n[1])


def device_ok() -> bool:
    return bool(lib().nnc_device_ok())


# ------------------------------------------------------------------------------- primitives
def nnc_ttm(X: torch.Tensor, n: int, A: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """X x_n A^T (Appendix A n-mode product with the transposed factor A, dims[n] x R)."""
    _dev(X, "X", (torch.float32, torch.bfloat16))
    _dev(A, "A")
    shape = list(X.shape)
    shape[n] = A.shape[1]
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=X.device)
    _dev(out, "out")
    _check(lib().nnc_ttm(X.data_ptr(), _xdt(X), X.dim(), _dims(X.shape), n, A.data_ptr(), A.shape[1],
                         out.data_ptr(), _stream()))
    return out


def nnc_convert_f32_bf16(x: torch.Tensor) -> torch.Tensor:
    """Round-to-nearest-even FP32 -> bfloat16 on the GPU."""
    _dev(x, "x")
    out = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    _check(lib().nnc_convert_f32_bf16(x.data_ptr(), out.data_ptr(), x.numel(), _stream()))
    return out


def nnc_fill_uniform(seed: int, stream_id: int, n_or_out, device="cuda") -> torch.Tensor:
    """Seeded U[0,1) float32 draws (counter-based SplitMix64, rounded to nearest) on the GPU.
    Pass a length (a new tensor is returned) or a contiguous float32 device tensor to fill."""
    if isinstance(n_or_out, torch.Tensor):
        out = _dev(n_or_out, "out")
    else:
        out = torch.empty(int(n_or_out), dtype=torch.float32, device=device)
    _check(lib().nnc_fill_uniform(int(seed) & (2**64 - 1), int(stream_id) & (2**64 - 1), out.data_ptr(),
                                  out.numel(), _stream()))
    return out


def nnc_fill_uniform_f64(seed: int, stream_id: int, n_or_out, offset: int = 0, device="cuda") -> torch.Tensor:
    """Seeded U[0,1) float64 draws of elements offset .. offset + n - 1 of a stream."""
    if isinstance(n_or_out, torch.Tensor):
        out = _dev(n_or_out, "out", (torch.float64,))
    else:
        out = torch.empty(int(n_or_out), dtype=torch.float64, device=device)
    _check(lib().nnc_fill_uniform_f64(int(seed) & (2**64 - 1), int(stream_id) & (2**64 - 1), int(offset),
                                      out.data_ptr(), out.numel(), _stream()))
    return out


# ------------------------------------------------------------------------------- nnTucker
@dataclass
class FitReport:
    sweeps_done: int
    rel_residual: float
    eps_clips: int
    seconds: float
    history: List[float] = field(default_factory=list)
    ttm_pass_ms: float = 0.0
    ttm_pass_launches: int = 0


def nntucker_workspace_bytes(dims: Sequence[int], multirank: Sequence[int]) -> int:
    return int(lib().nntucker_workspace_bytes(len(dims), _dims(dims), _dims(multirank)))


def nntucker_fit(X: torch.Tensor, multirank: Sequence[int], iters: int, core: torch.Tensor,
                 factors: Sequence[torch.Tensor], *, x_fp32: Optional[torch.Tensor] = None,
                 fp32_final_sweeps: int = 0, eps: float = 1e-12, objective_every: int = 0,
                 use_graph: bool = True, report: bool = True,
                 workspace: Optional[torch.Tensor] = None) -> Optional[FitReport]:
    """nnTucker by multiplicative updates, `iters` sweeps, in place on core and factors."""
    return _tucker_fit(lib().nntucker_fit, X, multirank, iters, core, factors, x_fp32, fp32_final_sweeps,
                       eps, objective_every, use_graph, report, workspace)


def tucker_ls_fit(X: torch.Tensor, multirank: Sequence[int], iters: int, core: torch.Tensor,
                  factors: Sequence[torch.Tensor], *, x_fp32: Optional[torch.Tensor] = None,
                  fp32_final_sweeps: int = 0, objective_every: int = 0, use_graph: bool = True,
                  report: bool = True, workspace: Optional[torch.Tensor] = None) -> Optional[FitReport]:
    """Real-valued Tucker fit by alternating least squares with orthonormalized factors,
    `iters` sweeps, in place (the Tucker step of CANDELINC, Section 2.2)."""
    return _tucker_fit(lib().tucker_ls_fit, X, multirank, iters, core, factors, x_fp32, fp32_final_sweeps,
                       0.0, objective_every, use_graph, report, workspace)


def _tucker_fit(fn, X, multirank, iters, core, factors, x_fp32, fp32_final_sweeps, eps, objective_every,
                use_graph, report, workspace):
    _dev(X, "X", (torch.float32, torch.bfloat16))
    _dev(core, "core")
    for k, f in enumerate(factors):
        _dev(f, "factors[%d]" % k)
    d = X.dim()
    need = nntucker_workspace_bytes(X.shape, multirank)
    if workspace is None:
        workspace = _workspace(need, X.device)
    opt = Options()
    opt.fp32_final_sweeps = int(fp32_final_sweeps)
    opt.x_fp32 = _dev(x_fp32, "x_fp32").data_ptr() if x_fp32 is not None else None
    opt.eps = float(eps)
    opt.objective_every = int(objective_every)
    opt.use_graph = 1 if use_graph else 0
    opt.workspace = workspace.data_ptr()
    opt.workspace_bytes = workspace.numel()
    rep = Report()
    hist = None
    if objective_every > 0:
        hist = (ctypes.c_double * max(1, iters // objective_every + 1))()
        rep.objective_history = ctypes.cast(hist, _dp)
    st = fn(X.data_ptr(), _xdt(X), d, _dims(X.shape), _dims(multirank), int(iters),
            core.data_ptr(), _ptrs(factors), ctypes.byref(opt),
            ctypes.byref(rep) if (report or objective_every) else None, _stream())
    _check(st)
    if not (report or objective_every):
        return None
    return FitReport(rep.sweeps_done, rep.rel_residual, rep.eps_clips, rep.seconds,
                     [hist[i] for i in range(rep.history_len)] if hist is not None else [],
                     rep.ttm_pass_ms, rep.ttm_pass_launches)


# ------------------------------------------------------------------------------- nnCP
def _cp_report(rep, full: bool):
    if full:
        return FitReport(rep.sweeps_done, rep.rel_residual, rep.eps_clips, rep.seconds)
    return rep.rel_residual


def nncp_fit(core: torch.Tensor, rank: int, iters: int, cp_factors: Sequence[torch.Tensor], *,
             eps: float = 1e-12, residual: bool = True, report: bool = False):
    """nnCP of the core by multiplicative updates in one persistent launch, in place.
    Returns the relative residual ||core - cp(B)|| / ||core|| (residual=True), the full
    FitReport with the clip count (report=True), or None."""
    _dev(core, "core")
    for k, f in enumerate(cp_factors):
        _dev(f, "cp_factors[%d]" % k)
    d = core.dim()
    ws = _workspace(lib().nncp_workspace_bytes(d, _dims(core.shape), int(rank)), core.device)
    opt = Options()
    opt.eps = float(eps)
    opt.workspace = ws.data_ptr()
    opt.workspace_bytes = ws.numel()
    rep = Report()
    want = residual or report
    _check(lib().nncp_fit(core.data_ptr(), d, _dims(core.shape), int(rank), int(iters), _ptrs(cp_factors),
                          ctypes.byref(opt), ctypes.byref(rep) if want else None, _stream()))
    return _cp_report(rep, report) if want else None


def cp_ls_fit(core: torch.Tensor, rank: int, iters: int, cp_factors: Sequence[torch.Tensor], *,
              residual: bool = True, report: bool = False):
    """Real-valued CP of the core by alternating least squares in one persistent launch, in
    place (the CPD step of CANDELINC, Section 2.2).  Returns as nncp_fit."""
    _dev(core, "core")
    for k, f in enumerate(cp_factors):
        _dev(f, "cp_factors[%d]" % k)
    d = core.dim()
    ws = _workspace(lib().cp_ls_workspace_bytes(d, _dims(core.shape), int(rank)), core.device)
    opt = Options()
    opt.workspace = ws.data_ptr()
    opt.workspace_bytes = ws.numel()
    rep = Report()
    want = residual or report
    _check(lib().cp_ls_fit(core.data_ptr(), d, _dims(core.shape), int(rank), int(iters), _ptrs(cp_factors),
                           ctypes.byref(opt), ctypes.byref(rep) if want else None, _stream()))
    return _cp_report(rep, report) if want else None


def nncp_fit_noalloc(core: torch.Tensor, rank: int, iters: int, cp_factors: Sequence[torch.Tensor], *,
                     eps: float = 1e-12, residual: bool = True, report: bool = False):
    """nncp_fit without a workspace: the library's static device scratch serves instead, so
    the call allocates no device memory.  Returns as nncp_fit."""
    _dev(core, "core")
    for k, f in enumerate(cp_factors):
        _dev(f, "cp_factors[%d]" % k)
    d = core.dim()
    opt = Options()
    opt.eps = float(eps)
    rep = Report()
    want = residual or report
    _check(lib().nncp_fit_noalloc(core.data_ptr(), d, _dims(core.shape), int(rank), int(iters),
                                  _ptrs(cp_factors), ctypes.byref(opt), ctypes.byref(rep) if want else None,
                                  _stream()))
    return _cp_report(rep, report) if want else None


def nncpx_workspace_bytes(dims: Sequence[int], rank: int) -> int:
    return int(lib().nncpx_workspace_bytes(len(dims), _dims(dims), int(rank)))


def nncpx_fit(X: torch.Tensor, rank: int, iters: int, factors: Sequence[torch.Tensor], *,
              x_fp32: Optional[torch.Tensor] = None, fp32_final_sweeps: int = 0, eps: float = 1e-12,
              objective_every: int = 0, use_graph: bool = True, report: bool = True,
              workspace: Optional[torch.Tensor] = None) -> Optional[FitReport]:
    """nnCP of the data tensor X (the nnCPD step of Algorithm 2), `iters` multiplicative
    sweeps, in place on the factors (dims[n] x rank)."""
    _dev(X, "X", (torch.float32, torch.bfloat16))
    for k, f in enumerate(factors):
        _dev(f, "factors[%d]" % k)
    d = X.dim()
    need = nncpx_workspace_bytes(X.shape, rank)
    if workspace is None:
        workspace = _workspace(need, X.device)
    opt = Options()
    opt.fp32_final_sweeps = int(fp32_final_sweeps)
    opt.x_fp32 = _dev(x_fp32, "x_fp32").data_ptr() if x_fp32 is not None else None
    opt.eps = float(eps)
    opt.objective_every = int(objective_every)
    opt.use_graph = 1 if use_graph else 0
    opt.workspace = workspace.data_ptr()
    opt.workspace_bytes = workspace.numel()
    rep = Report()
    hist = None
    if objective_every > 0:
        hist = (ctypes.c_double * max(1, iters // objective_every + 1))()
        rep.objective_history = ctypes.cast(hist, _dp)
    st = lib().nncpx_fit(X.data_ptr(), _xdt(X), d, _dims(X.shape), int(rank), int(iters), _ptrs(factors),
                         ctypes.byref(opt), ctypes.byref(rep) if (report or objective_every) else None,
                         _stream())
    _check(st)
    if not (report or objective_every):
        return None
    return FitReport(rep.sweeps_done, rep.rel_residual, rep.eps_clips, rep.seconds,
                     [hist[i] for i in range(rep.history_len)] if hist is not None else [],
                     rep.ttm_pass_ms, rep.ttm_pass_launches)


def nmf_fit(A: torch.Tensor, rank: int, iters: int, W: torch.Tensor, H: torch.Tensor, *,
            eps: float = 1e-12, residual: bool = True) -> Optional[float]:
    """NMF A ~ W H (the NMF step of Algorithm 2) by multiplicative updates, in place on W
    (rows x rank) and H (rank x cols); returns ||A - W H|| / ||A|| when `residual`."""
    _dev(A, "A")
    _dev(W, "W")
    _dev(H, "H")
    if A.dim() != 2:
        raise NncError(NNC_EINVAL, "A must be a matrix")
    rows, cols = A.shape
    ws = _workspace(lib().nmf_workspace_bytes(rows, cols, int(rank)), A.device)
    res = ctypes.c_double(0.0)
    _check(lib().nmf_fit(A.data_ptr(), rows, cols, int(rank), int(iters), W.data_ptr(), H.data_ptr(),
                         float(eps), ctypes.byref(res) if residual else None, ws.data_ptr(), ws.numel(),
                         _stream()))
    return res.value if residual else None


def nmf_fit_batched(A: Sequence[torch.Tensor], ranks: Sequence[int], iters: int, W: Sequence[torch.Tensor],
                    H: Sequence[torch.Tensor], *, eps: float = 1e-12, residual: bool = True) -> Optional[List[float]]:
    """Several NMFs A[j] ~ W[j] H[j] with a common column count, in place; returns the
    relative residuals when `residual`."""
    n = len(A)
    for j in range(n):
        _dev(A[j], "A[%d]" % j)
        _dev(W[j], "W[%d]" % j)
        _dev(H[j], "H[%d]" % j)
    cols = int(A[0].shape[1])
    rows = _dims([int(a.shape[0]) for a in A])
    rk = (ctypes.c_int * n)(*[int(r) for r in ranks])
    ws = _workspace(lib().nmf_batched_workspace_bytes(n, rows, cols, rk), A[0].device)
    res = (ctypes.c_double * n)()
    _check(lib().nmf_fit_batched(n, _ptrs(A), rows, cols, rk, int(iters), _ptrs(W), _ptrs(H), float(eps),
                                 res if residual else None, ws.data_ptr(), ws.numel(), _stream()))
    return [res[j] for j in range(n)] if residual else None


def mean_congruence(P: Sequence[torch.Tensor], Q: Sequence[torch.Tensor]) -> float:
    """Mean congruence of two CP models (factor n: dims[n] x rank, rank <= 8) under the best
    matching of their components (Section 4.1 scoring)."""
    for k in range(len(P)):
        _dev(P[k], "P[%d]" % k)
        _dev(Q[k], "Q[%d]" % k)
    out = torch.empty(1, dtype=torch.float64, device=P[0].device)
    _check(lib().nnc_mean_congruence(len(P), _dims([p.shape[0] for p in P]), int(P[0].shape[1]), _ptrs(P),
                                     _ptrs(Q), out.data_ptr(), _stream()))
    return float(out.item())


@dataclass
class RestartResult:
    rel_errors: "torch.Tensor"            # [nrestarts] float64 (device)
    congruences: Optional["torch.Tensor"]  # [nrestarts] float64 (device) or None
    lifted: Optional["torch.Tensor"]       # [nrestarts, sum(dims), rank] or None
    clips: int


def nncandelinc_restarts(X: torch.Tensor, algorithm: int, multirank: Sequence[int], rank: int,
                         inits: torch.Tensor, outer_iters: int, inner_iters: int, *,
                         truth: Optional[Sequence[torch.Tensor]] = None, eps: float = 1e-12,
                         lifted: bool = False) -> RestartResult:
    """The Section 4.2 study: inits.shape[0] complete fits of the small 3-way tensor X (Algorithm 1
    or 2) in one launch, one workgroup per start (inits: [nrestarts, per-start floats])."""
    _dev(X, "X")
    _dev(inits, "inits")
    if X.dim() != 3 or inits.dim() != 2:
        raise NncError(NNC_EINVAL, "X must be 3-way and inits a [nrestarts, floats] matrix")
    dims = _dims(X.shape)
    mr = _dims(multirank)
    per = int(lib().nncandelinc_restart_init_floats(int(algorithm), dims, mr, int(rank)))
    if per <= 0 or inits.shape[1] != per:
        raise NncError(NNC_EINVAL, "inits must have %d floats per start" % per)
    n = int(inits.shape[0])
    rel = torch.empty(n, dtype=torch.float64, device=X.device)
    cong = torch.empty(n, dtype=torch.float64, device=X.device) if truth is not None else None
    out = torch.empty(n, sum(X.shape), int(rank), dtype=torch.float32, device=X.device) if lifted else None
    clips = torch.zeros(1, dtype=torch.int64, device=X.device)
    tp = None
    if truth is not None:
        for k, t in enumerate(truth):
            _dev(t, "truth[%d]" % k)
        tp = _ptrs(truth)
    _check(lib().nncandelinc_restarts(X.data_ptr(), dims, int(algorithm), mr, int(rank), n, int(outer_iters),
                                      int(inner_iters), inits.data_ptr(), tp, float(eps), rel.data_ptr(),
                                      cong.data_ptr() if cong is not None else None,
                                      out.data_ptr() if out is not None else None, clips.data_ptr(), _stream()))
    return RestartResult(rel, cong, out, int(clips.item()))


def nncandelinc_alg2(X: torch.Tensor, rank: int, multirank: Sequence[int], cp_iters: int, nmf_iters: int,
                     cp_factors: Sequence[torch.Tensor], F: Sequence[torch.Tensor], B: Sequence[torch.Tensor],
                     *, x_fp32: Optional[torch.Tensor] = None, fp32_final_sweeps: int = 0,
                     eps: float = 1e-12) -> FitReport:
    """Algorithm 2: nnCP of X (cp_factors, dims[n] x rank, in place), then NMF of each CP
    factor into F[n] (dims[n] x multirank[n]) and B[n] (multirank[n] x rank), in place.  The
    nnCANDELINC model is C_n = F[n] B[n] (nncandelinc_lift).  Returns the nnCP report."""
    rep = nncpx_fit(X, rank, cp_iters, cp_factors, x_fp32=x_fp32, fp32_final_sweeps=fp32_final_sweeps,
                    eps=eps)
    nmf_fit_batched(list(cp_factors), [int(m) for m in multirank], nmf_iters, list(F), list(B), eps=eps,
                    residual=False)
    return rep


def nncp_fit_batched(core: torch.Tensor, ranks: Sequence[int], iters: int,
                     cp_factors: Sequence[Sequence[torch.Tensor]], *, eps: float = 1e-12,
                     threads_per_fit: int = 0) -> List[float]:
    """Independent nnCP fits of one core (restart j: rank ranks[j], factors cp_factors[j])
    in a single persistent launch.  Returns each fit's relative residual."""
    _dev(core, "core")
    d = core.dim()
    nb = len(ranks)
    flat = []
    for j, fs in enumerate(cp_factors):
        assert len(fs) == d
        for k, f in enumerate(fs):
            flat.append(_dev(f, "cp_factors[%d][%d]" % (j, k)))
    rk = (ctypes.c_int * nb)(*[int(r) for r in ranks])
    ws = _workspace(lib().nncp_batched_workspace_bytes(d, _dims(core.shape), nb, rk), core.device)
    res = (ctypes.c_double * nb)()
    _check(lib().nncp_fit_batched(core.data_ptr(), d, _dims(core.shape), nb, rk, int(iters),
                                  _ptrs(flat), float(eps), res, int(threads_per_fit), ws.data_ptr(),
                                  ws.numel(), _stream()))
    return [res[j] for j in range(nb)]


# ------------------------------------------------------------------------------- lift, residual
def nncandelinc_lift(tucker_factors: Sequence[torch.Tensor], cp_factors: Sequence[torch.Tensor],
                     out: Optional[Sequence[torch.Tensor]] = None) -> List[torch.Tensor]:
    """C_n = A_n B_n for every mode."""
    d = len(tucker_factors)
    rank = cp_factors[0].shape[1]
    dims = [a.shape[0] for a in tucker_factors]
    mr = [a.shape[1] for a in tucker_factors]
    for k in range(d):
        _dev(tucker_factors[k], "tucker_factors[%d]" % k)
        _dev(cp_factors[k], "cp_factors[%d]" % k)
    if out is None:
        out = [torch.empty(dims[k], rank, dtype=torch.float32, device=tucker_factors[0].device)
               for k in range(d)]
    _check(lib().nncandelinc_lift(d, _dims(dims), _dims(mr), int(rank), _ptrs(tucker_factors),
                                  _ptrs(cp_factors), _ptrs(out), _stream()))
    return list(out)


def reconstruct_residual(X: torch.Tensor, factors: Sequence[torch.Tensor],
                         core: Optional[torch.Tensor] = None) -> float:
    """||X - Xhat||_F / ||X||_F for a Tucker model (core given) or a CP model (core None)."""
    _dev(X, "X", (torch.float32, torch.bfloat16))
    d = X.dim()
    if core is not None:
        _dev(core, "core")
        model = list(core.shape)
        is_cp = 0
    else:
        model = [factors[0].shape[1]] + [0] * (d - 1)
        is_cp = 1
    for k, f in enumerate(factors):
        _dev(f, "factors[%d]" % k)
    ws = _workspace(lib().reconstruct_workspace_bytes(d, _dims(X.shape), _dims(model), is_cp), X.device)
    res = ctypes.c_double(0.0)
    _check(lib().reconstruct_residual(X.data_ptr(), _xdt(X), d, _dims(X.shape),
                                      core.data_ptr() if core is not None else None, _dims(model),
                                      _ptrs(factors), ctypes.byref(res), ws.data_ptr(), ws.numel(),
                                      _stream()))
    return res.value


# ------------------------------------------------------------------------------- adjoint
def nntucker_grad(X: torch.Tensor, core: torch.Tensor, factors: Sequence[torch.Tensor],
                  want_loss: bool = True):
    """(loss, dL/dG, [dL/dA_n]) for L = 0.5 ||X - G x {A}||^2 from the library's adjoint."""
    _dev(X, "X", (torch.float32, torch.bfloat16))
    _dev(core, "core")
    d = X.dim()
    mr = list(core.shape)
    ws = _workspace(nntucker_workspace_bytes(X.shape, mr), X.device)
    gG = torch.empty_like(core)
    gA = [torch.empty_like(_dev(f, "factors[%d]" % k)) for k, f in enumerate(factors)]
    loss = ctypes.c_double(0.0)
    _check(lib().nntucker_grad(X.data_ptr(), _xdt(X), d, _dims(X.shape), _dims(mr), core.data_ptr(),
                               _ptrs(factors), gG.data_ptr(), _ptrs(gA),
                               ctypes.byref(loss) if want_loss else None, ws.data_ptr(), ws.numel(),
                               _stream()))
    return (loss.value if want_loss else None), gG, gA


def reconstruct_sq_sums(X: torch.Tensor, factors: Sequence[torch.Tensor],
                        core: Optional[torch.Tensor] = None):
    """(||X - Xhat||_F^2, ||X||_F^2) in double precision (Tucker if core given, else CP)."""
    _dev(X, "X", (torch.float32, torch.bfloat16))
    d = X.dim()
    if core is not None:
        _dev(core, "core")
        model, is_cp = list(core.shape), 0
    else:
        model, is_cp = [factors[0].shape[1]] + [0] * (d - 1), 1
    for k, f in enumerate(factors):
        _dev(f, "factors[%d]" % k)
    ws = _workspace(lib().reconstruct_workspace_bytes(d, _dims(X.shape), _dims(model), is_cp), X.device)
    e, n = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().reconstruct_sq_sums(X.data_ptr(), _xdt(X), d, _dims(X.shape),
                                     core.data_ptr() if core is not None else None, _dims(model),
                                     _ptrs(factors), ctypes.byref(e), ctypes.byref(n), ws.data_ptr(),
                                     ws.numel(), _stream()))
    return e.value, n.value


class NNTuckerLoss(torch.autograd.Function):
    """L = 0.5 ||X - G x_1 A_1 ... x_d A_d||_F^2 with the hand-written adjoint as backward.

    forward(X, G, A_1, ..., A_d) -> 0-dim float64 tensor (fused residual pass, FP64 sum).
    backward recomputes the contraction chain from X (nothing but the inputs is saved) and
    returns dL/dG = den_G - num_G and dL/dA_n = den_n - num_n; X gets no gradient.
    """

    @staticmethod
    def forward(ctx, X, G, *A):
        ctx.save_for_backward(X, G, *A)
        sq, _ = reconstruct_sq_sums(X, [a.contiguous() for a in A], G.contiguous())
        return torch.tensor(0.5 * sq, dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, gout):
        X, G, *A = ctx.saved_tensors
        _, gG, gA = nntucker_grad(X, G.contiguous(), [a.contiguous() for a in A], want_loss=False)
        s = gout.to(torch.float32)
        return (None, gG * s, *[g * s for g in gA])


def nntucker_loss(X: torch.Tensor, G: torch.Tensor, factors: Sequence[torch.Tensor]) -> torch.Tensor:
    return NNTuckerLoss.apply(X, G, *factors)
