"""MI355X (gfx950) hot path of the sketch-preconditioned interior point method.

Python binding of the C ABI in include/ipmsk.h. The functions carry the C names
(``ipm_sketch``, ``ipm_precond_factor``, ``ipm_pcg_solve``, ``ipm_step``,
``ipm_normal_matvec``) and take torch tensors on a ROCm device; they only
marshal arguments. ``solve`` repeats ``ipm_step`` until the stop test holds
(Algorithm 3's outer loop).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional

from . import native
from .native import (IPM_BF16, IPM_CONVERGED, IPM_CSR, IPM_F32, IPM_F64, IPM_MIXED, IPM_MIXED_F32ACC, IPM_OK, IPM_PLAIN,
                     IPM_WARM_GIVEN, IPM_WARM_NONE, IPM_WARM_PREV, IpmMatrix, IpmParams, IpmPcgInfo,
                     IpmProblem, IpmState, IpmStepInfo)

__all__ = ["IpmError", "Context", "Matrix", "SparseMatrix", "Problem", "State", "Params", "ipm_sketch",
           "ipm_sketch_gaussian", "ipm_precond_factor", "ipm_pcg_solve", "ipm_step", "ipm_step_warm", "ipm_last_dy",
           "ipm_normal_matvec", "ipm_stream_read", "ipm_stream_copy", "solve", "IPM_OK", "IPM_CONVERGED", "IPM_F64", "IPM_F32", "IPM_BF16",
           "IPM_CSR", "IPM_PLAIN", "IPM_MIXED", "IPM_MIXED_F32ACC", "IPM_WARM_NONE", "IPM_WARM_PREV", "IPM_WARM_GIVEN"]


def _torch():
    import torch
    return torch


class IpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{native.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return IPM_F64
    if t.dtype == torch.float32:
        return IPM_F32
    if t.dtype == torch.bfloat16:
        return IPM_BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need_dev(t, name, dtype=None):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    return t


class Context:
    """Library context bound to a device and (by default) its current torch stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = native.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.ipm_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != IPM_OK:
            raise IpmError(rc, "ipm_ctx_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ipm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, allow_positive: bool = True) -> int:
        if rc < 0 or (rc > 0 and not allow_positive):
            msg = self.lib.ipm_last_error(self.h)
            raise IpmError(rc, msg.decode() if msg else "")
        return rc

    def set_timing(self, on):
        """False/0: off; True/1: time every launch of the measured kernels; N: every N-th."""
        period = int(on) if not isinstance(on, bool) else (1 if on else 0)
        self.check(self.lib.ipm_ctx_set_timing(self.h, period))

    def kernel_time(self, kernel: int):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self.check(self.lib.ipm_kernel_time(self.h, kernel, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


@dataclass
class Matrix:
    """Dense row-major A (m x n) stored with row stride ld (padded for 128-byte rows)."""
    data: object          # torch tensor (m, ld)
    n: int

    @property
    def m(self) -> int:
        return self.data.shape[0]

    @property
    def ld(self) -> int:
        return self.data.shape[1]

    def c(self) -> IpmMatrix:
        return IpmMatrix(self.m, self.n, self.ld, 0, _dtype_code(self.data), self.data.data_ptr())

    @staticmethod
    def from_numpy(A, dtype=None, device: int = 0) -> "Matrix":
        torch = _torch()
        dtype = dtype or torch.float64
        m, n = A.shape
        esz = torch.empty((), dtype=dtype).element_size()
        align = 128 // esz
        ld = ((n + align - 1) // align) * align
        host = torch.zeros((m, ld), dtype=torch.float64)
        host[:, :n] = torch.from_numpy(A)
        return Matrix(host.to(dtype).to(f"cuda:{device}").contiguous(), n)


@dataclass
class SparseMatrix:
    """Sparse A (m x n) in device memory: CSR (val, row_ptr, col_idx) and a CSC mirror
    (csc_val, col_ptr, row_idx) of the same nonzeros."""
    m: int
    n: int
    val: object           # torch (nnz,) storage dtype, row order
    row_ptr: object       # torch int64 (m + 1,)
    col_idx: object       # torch int32 (nnz,)
    csc_val: object       # torch (nnz,) storage dtype, column order
    col_ptr: object       # torch int64 (n + 1,)
    row_idx: object       # torch int32 (nnz,)

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    def c(self) -> IpmMatrix:
        return IpmMatrix(self.m, self.n, 0, IPM_CSR, _dtype_code(self.val), self.val.data_ptr(), self.nnz,
                         self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.csc_val.data_ptr(),
                         self.col_ptr.data_ptr(), self.row_idx.data_ptr())

    @staticmethod
    def from_scipy(A, dtype=None, device: int = 0) -> "SparseMatrix":
        """A: any scipy.sparse matrix; its values are rounded to ``dtype`` (default float64)."""
        import numpy as np
        torch = _torch()
        dtype = dtype or torch.float64
        dev = f"cuda:{device}"
        r = A.tocsr()
        r.sum_duplicates()
        cc = r.tocsc()
        cc.sort_indices()
        to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).to(dev)
        return SparseMatrix(r.shape[0], r.shape[1], to(r.data, torch.float64).to(dtype), to(r.indptr, torch.int64),
                            to(r.indices, torch.int32), to(cc.data, torch.float64).to(dtype),
                            to(cc.indptr, torch.int64), to(cc.indices, torch.int32))


@dataclass
class Problem:
    A: object             # Matrix or SparseMatrix
    b: object
    c: object

    def c_struct(self) -> IpmProblem:
        return IpmProblem(self.A.c(), self.b.data_ptr(), self.c.data_ptr())

    @staticmethod
    def from_lp(lp, dtype=None, device: int = 0) -> "Problem":
        torch = _torch()
        dev = f"cuda:{device}"
        if hasattr(lp.A, "tocsr"):
            A = SparseMatrix.from_scipy(lp.A, dtype=dtype, device=device)
        else:
            A = Matrix.from_numpy(lp.A, dtype=dtype, device=device)
        b = torch.from_numpy(lp.b).to(dev)
        c = torch.from_numpy(lp.c).to(dev)
        return Problem(A, b, c)


@dataclass
class State:
    x: object
    y: object
    s: object
    k: int = 0
    mu0: float = -1.0
    r0norm: float = -1.0

    @staticmethod
    def initial(m: int, n: int, device: int = 0) -> "State":
        torch = _torch()
        dev = f"cuda:{device}"
        return State(torch.ones(n, dtype=torch.float64, device=dev), torch.zeros(m, dtype=torch.float64, device=dev),
                     torch.ones(n, dtype=torch.float64, device=dev))


@dataclass
class Params:
    w: int
    s: int = 2
    seed: int = 0
    sigma: float = 0.5
    gamma: float = 0.9
    theta: float = 0.9999
    tol_pcg: float = 1e-10
    gap_tol: float = 1e-8
    min_step: float = 1e-14
    stag_ratio: float = 0.99
    maxit_pcg: int = 500
    stag_window: int = 10
    max_redraws: int = 3
    vcorr: int = 1
    precision: int = IPM_PLAIN     # IPM_PLAIN, IPM_MIXED or IPM_MIXED_F32ACC
    warm_start: int = IPM_WARM_NONE
    inner_tol: float = 1e-4
    max_refine: int = 12
    max_shifts: int = 3
    feasible: int = 0              # 1: Algorithm 2 from a strictly feasible state
    solver: int = 0                # 0: CG; 1: Chebyshev after a CG probe
    sketch: int = 0                # 0: sparse embedding; 1: Gaussian W

    def c(self) -> IpmParams:
        return IpmParams(self.sigma, self.gamma, self.theta, self.tol_pcg, self.gap_tol, self.min_step,
                         self.stag_ratio, self.w, self.s, self.maxit_pcg, self.stag_window, self.max_redraws,
                         self.vcorr, self.precision, self.warm_start, self.inner_tol, self.max_refine,
                         self.max_shifts, self.feasible, self.solver, self.sketch, 0,
                         self.seed & ((1 << 64) - 1))


def ipm_normal_matvec(ctx: Context, A: Matrix, d2, v):
    """q = A diag(d2) A^T v (one pass over A)."""
    torch = _torch()
    _need_dev(d2, "d2", torch.float64)
    _need_dev(v, "v", torch.float64)
    q = torch.empty(A.m, dtype=torch.float64, device=v.device)
    Ac = A.c()
    ctx.check(ctx.lib.ipm_normal_matvec(ctx.h, ctypes.byref(Ac), _ptr(d2), _ptr(v), _ptr(q)))
    return q


def ipm_normal_matvec_noalloc(ctx: Context, A, d2, v, q):
    """q = A diag(d2) A^T v into the caller's q, with the library allocating nothing (its partial
    sums in the static scratch array)."""
    torch = _torch()
    _need_dev(d2, "d2", torch.float64)
    _need_dev(v, "v", torch.float64)
    _need_dev(q, "q", torch.float64)
    if q.numel() != A.m or v.numel() != A.m or d2.numel() != A.n:
        raise ValueError("need v, q of length m and d2 of length n")
    Ac = A.c()
    ctx.check(ctx.lib.ipm_normal_matvec_noalloc(ctx.h, ctypes.byref(Ac), _ptr(d2), _ptr(v), _ptr(q)))
    return q


def ipm_stream_read(ctx: Context, x, out=None):
    """FP64 sum of the contiguous FP64 tensor x in one streaming pass (bandwidth probe); returns
    a one-element device tensor (or fills `out`)."""
    torch = _torch()
    _need_dev(x, "x", torch.float64)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    ctx.check(ctx.lib.ipm_stream_read(ctx.h, _ptr(x), x.numel(), _ptr(out)))
    return out


def ipm_stream_copy(ctx: Context, src, dst, nbytes: Optional[int] = None):
    """dst's first nbytes bytes (default: all of src) = src's, in one streaming pass (bandwidth
    probe); both contiguous device tensors."""
    _need_dev(src, "src")
    _need_dev(dst, "dst")
    size = src.numel() * src.element_size()
    nbytes = size if nbytes is None else int(nbytes)
    if nbytes > size or nbytes > dst.numel() * dst.element_size():
        raise ValueError("nbytes exceeds a buffer")
    ctx.check(ctx.lib.ipm_stream_copy(ctx.h, _ptr(src), _ptr(dst), nbytes))
    return dst


def ipm_sketch(ctx: Context, A: Matrix, d, seed: int, k: int, w: int, s: int, out_dtype=None):
    """B = A diag(d) W (m x w) for the hash-defined sparse embedding W of iteration k."""
    torch = _torch()
    out_dtype = out_dtype or torch.float64
    _need_dev(d, "d", torch.float64)
    B = torch.empty((A.m, w), dtype=out_dtype, device=d.device)
    Ac = A.c()
    ctx.check(ctx.lib.ipm_sketch(ctx.h, ctypes.byref(Ac), _ptr(d), seed & ((1 << 64) - 1), k, w, s,
                                 _dtype_code(B), _ptr(B)))
    return B


def ipm_sketch_gaussian(ctx: Context, A, d, seed: int, k: int, w: int):
    """B = A diag(d) W (FP64, m x w) for the Gaussian W of iteration k."""
    torch = _torch()
    _need_dev(d, "d", torch.float64)
    B = torch.empty((A.m, w), dtype=torch.float64, device=d.device)
    Ac = A.c()
    ctx.check(ctx.lib.ipm_sketch_gaussian(ctx.h, ctypes.byref(Ac), _ptr(d), seed & ((1 << 64) - 1), k, w, _ptr(B)))
    return B


def ipm_precond_factor(ctx: Context, B, want_L: bool = True):
    """(L, Linv) with B B^T = L L^T; Linv = L^{-1} (lower triangle, zero above)."""
    torch = _torch()
    _need_dev(B, "B")
    m, w = B.shape
    L = torch.empty((m, m), dtype=torch.float64, device=B.device) if want_L else None
    Linv = torch.empty((m, m), dtype=torch.float64, device=B.device)
    bad = ctypes.c_int64(-1)
    ctx.check(ctx.lib.ipm_precond_factor(ctx.h, m, w, _dtype_code(B), _ptr(B), _ptr(L), _ptr(Linv),
                                         ctypes.byref(bad)))
    return L, Linv


def ipm_pcg_solve(ctx: Context, A: Matrix, d2, Linv, p, params: Params, dy0=None):
    """CG with preconditioner Q = L L^T; returns (dy, info dict)."""
    torch = _torch()
    for t, nm in ((d2, "d2"), (Linv, "Linv"), (p, "p")):
        _need_dev(t, nm, torch.float64)
    dy = torch.zeros_like(p) if dy0 is None else dy0.clone()
    info = IpmPcgInfo()
    Ac = A.c()
    prm = params.c()
    rc = ctx.lib.ipm_pcg_solve(ctx.h, ctypes.byref(Ac), _ptr(d2), _ptr(Linv), _ptr(p), _ptr(dy),
                               0 if dy0 is None else 1, ctypes.byref(prm), ctypes.byref(info))
    ctx.check(rc)
    return dy, {"iters": info.iters, "status": info.status, "warm_used": info.warm_used,
                "rounds": info.rounds, "relres": info.relres, "rho_star": info.rho_star}


def ipm_step(ctx: Context, prob: Problem, st: State, params: Params) -> dict:
    """One iteration of Algorithm 3; updates st in place; returns the step info."""
    return _step(ctx, prob, st, params, None)


def ipm_step_warm(ctx: Context, prob: Problem, st: State, params: Params, dy0) -> dict:
    """ipm_step whose CG solve starts from the M-norm-optimal combination of the candidate
    vectors dy0 (device FP64, shape (m,) or (ncand, m) with ncand 1 or 2); params.warm_start
    must be IPM_WARM_GIVEN for them to be used."""
    torch = _torch()
    _need_dev(dy0, "dy0", torch.float64)
    return _step(ctx, prob, st, params, dy0)


def ipm_last_dy(ctx: Context, m: int, device: int = 0, out=None):
    """The dy accepted by the last successful step on ctx (into ``out`` if given)."""
    torch = _torch()
    if out is None:
        out = torch.empty(m, dtype=torch.float64, device=f"cuda:{device}")
    _need_dev(out, "out", torch.float64)
    ctx.check(ctx.lib.ipm_last_dy(ctx.h, m, _ptr(out)))
    return out


def _step(ctx: Context, prob: Problem, st: State, params: Params, dy0) -> dict:
    pc = prob.c_struct()
    sc = IpmState(st.x.data_ptr(), st.y.data_ptr(), st.s.data_ptr(), st.k, st.mu0, st.r0norm)
    prm = params.c()
    info = IpmStepInfo()
    if dy0 is None:
        rc = ctx.lib.ipm_step(ctx.h, ctypes.byref(pc), ctypes.byref(sc), ctypes.byref(prm), ctypes.byref(info))
    else:
        ncand = 1 if dy0.dim() == 1 else dy0.shape[0]
        rc = ctx.lib.ipm_step_warm(ctx.h, ctypes.byref(pc), ctypes.byref(sc), ctypes.byref(prm), _ptr(dy0),
                                   ncand, ctypes.byref(info))
    st.k, st.mu0, st.r0norm = sc.k, sc.mu0, sc.r0norm
    d = info.as_dict()
    d["rc"] = rc
    ctx.check(rc)
    return d


@dataclass
class SolveResult:
    state: State
    infos: list
    converged: bool
    status: int
    iterations: int = 0
    extra: dict = field(default_factory=dict)


def solve(ctx: Context, prob: Problem, params: Params, maxit: int = 200, st: Optional[State] = None,
          callback=None, net=None, kmax: int = 200) -> SolveResult:
    """Algorithm 3 from x = s = 1, y = 0 until the stop test holds or maxit iterations.

    With a warm-start network ``net`` (learned.Mlp), every iteration after the first starts its
    CG solve from the M-norm-optimal combination of the previous direction and the network's
    prediction (ipm_mlp_predict, then ipm_step_warm with both as candidates)."""
    from dataclasses import replace
    dev = prob.b.device.index or 0
    st = st or State.initial(prob.A.m, prob.A.n, dev)
    infos = []
    prm_warm = replace(params, warm_start=IPM_WARM_GIVEN) if net is not None else None
    cand = None
    if net is not None:
        from .learned import mlp_predict_into
        torch = _torch()
        cand = torch.empty((2, prob.A.m), dtype=torch.float64, device=f"cuda:{dev}")   # [previous dy; network]
    have_prev = False
    for _ in range(maxit + 1):
        if net is not None and have_prev:
            mlp_predict_into(ctx, net, cand[0], st.x, st.s, st.k, kmax, cand[1])
            info = ipm_step_warm(ctx, prob, st, prm_warm, cand)
        else:
            info = ipm_step(ctx, prob, st, params)
        if net is not None and info["rc"] != IPM_CONVERGED:
            ipm_last_dy(ctx, prob.A.m, dev, out=cand[0])
            have_prev = True
        infos.append(info)
        if callback is not None:
            callback(st, info)
        if info["rc"] == IPM_CONVERGED:
            return SolveResult(st, infos, True, IPM_CONVERGED, st.k)
    return SolveResult(st, infos, False, IPM_OK, st.k)
