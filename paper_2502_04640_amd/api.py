"""ctypes binding of libxm (argument marshalling only).

Every function here forwards torch device pointers, sizes and the current HIP
stream to the C ABI declared in include/xm.h; no step of the computation runs
in Python.  Tensors must live on the ROCm device (torch "cuda" device type).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

XM_OK, XM_EINVAL, XM_ENOMEM, XM_EHIP, XM_EGRAPH, XM_ENOCONV = 0, -1, -2, -3, -4, -5
XM_F64, XM_F32, XM_BF16 = 0, 1, 2
XM_KEEP_F32, XM_KEEP_BF16 = 1 << 1, 1 << 2
XM_NOALLOC_SCRATCH_BYTES = 128 << 20   # XM_NOALLOC_SCRATCH_MIB in include/xm.h
_DT = {"f64": XM_F64, "f32": XM_F32, "bf16": XM_BF16}
_STATUS = {XM_EINVAL: "XM_EINVAL", XM_ENOMEM: "XM_ENOMEM", XM_EHIP: "XM_EHIP", XM_EGRAPH: "XM_EGRAPH",
           XM_ENOCONV: "XM_ENOCONV"}


class XMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _ProblemInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("n_obs", ctypes.c_int64), ("n_in", ctypes.c_int64),
                ("nnz_blocks", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("ld", ctypes.c_int32),
                ("copies", ctypes.c_int32), ("qbar", ctypes.c_double), ("build_ms", ctypes.c_double),
                ("scale_reg", ctypes.c_double)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("r0", ctypes.c_int32), ("r_max", ctypes.c_int32), ("lift", ctypes.c_double),
                ("compute", ctypes.c_int32),
                ("grad_tol", ctypes.c_double), ("cert_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("max_inner", ctypes.c_int32), ("delta0", ctypes.c_double), ("lanczos_max", ctypes.c_int32),
                ("lanczos_tol", ctypes.c_double), ("precondition", ctypes.c_int32), ("verbose", ctypes.c_int32)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("certified", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("stair_steps", ctypes.c_int32), ("spmm_count", ctypes.c_int32),
                ("lanczos_iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("cost", ctypes.c_double),
                ("grad_norm", ctypes.c_double), ("lambda_min", ctypes.c_double), ("primal", ctypes.c_double),
                ("dual", ctypes.c_double), ("solve_ms", ctypes.c_double), ("cert_ms", ctypes.c_double)]


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class _Cert(ctypes.Structure):
    _fields_ = [("lambda_min", ctypes.c_double), ("ritz_residual", ctypes.c_double),
                ("lambda_bound", ctypes.c_double), ("primal", ctypes.c_double),
                ("dual", ctypes.c_double), ("qbar", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("defl_min", ctypes.c_double), ("defl_cross", ctypes.c_double), ("rho_hat", ctypes.c_double),
                ("eta", ctypes.c_double), ("certified", ctypes.c_int32), ("iters", ctypes.c_int32)]


class _AdjInfo(ctypes.Structure):
    _fields_ = [("cg_iters", ctypes.c_int32), ("cg_residual", ctypes.c_double), ("cost", ctypes.c_double)]


class _SpmmStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 9), ("total_ms", ctypes.c_double * 9),
                ("bytes_per_launch", ctypes.c_double * 9)]


def library_path() -> str:
    return os.environ.get("XM_LIBRARY", os.path.join(HERE, "libxm.so"))


def load_library() -> ctypes.CDLL:
    """Load libxm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"libxm.so not found at {path}: build it with "
                          "`python -m paper_2502_04640_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, V, I32, I64, U32, D = (ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_uint32, ctypes.c_double)
    lib.xm_build_Q.argtypes = [I32, I32, I64, V, V, V, ctypes.c_int, V, ctypes.c_int, U32, V,
                               ctypes.POINTER(ctypes.c_void_p)]
    lib.xm_build_Q.restype = ctypes.c_int
    lib.xm_build_Q_masked.argtypes = [I32, I32, I64, V, V, V, ctypes.c_int, V, ctypes.c_int, V, U32, V,
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.xm_build_Q_masked.restype = ctypes.c_int
    lib.xm_set_scale_reg.argtypes = [P, D]
    lib.xm_set_scale_reg.restype = ctypes.c_int
    lib.xm_residuals.argtypes = [P, V, V, I32, V, V, V]
    lib.xm_residuals.restype = ctypes.c_int
    lib.xm_drop_largest.argtypes = [V, I64, D, V, ctypes.POINTER(ctypes.c_int64), V]
    lib.xm_drop_largest.restype = ctypes.c_int
    lib.xm_guard_frames.argtypes = [I32, I32, I64, V, V, I32, V, ctypes.POINTER(ctypes.c_int64), V]
    lib.xm_guard_frames.restype = ctypes.c_int
    lib.xm_align_similarity.argtypes = [I64, V, V, V, ctypes.POINTER(ctypes.c_double), V]
    lib.xm_align_similarity.restype = ctypes.c_int
    lib.xm_free.argtypes = [P]
    lib.xm_free.restype = None
    lib.xm_get_info.argtypes = [P, ctypes.POINTER(_ProblemInfo)]
    lib.xm_get_info.restype = ctypes.c_int
    lib.xm_get_Q_rows.argtypes = [P, I32, I32, V, V]
    lib.xm_get_Q_rows.restype = ctypes.c_int
    lib.xm_spmm.argtypes = [P, ctypes.c_int, V, I32, V, V]
    lib.xm_spmm.restype = ctypes.c_int
    lib.xm_default_opts.argtypes = [ctypes.POINTER(_SolveOpts)]
    lib.xm_default_opts.restype = None
    lib.xm_bm_solve.argtypes = [P, ctypes.POINTER(_SolveOpts), V, I32, V, ctypes.POINTER(_SolveInfo), V]
    lib.xm_bm_solve.restype = ctypes.c_int
    lib.xm_certify.argtypes = [P, V, I32, D, I32, V, ctypes.POINTER(_Cert), V]
    lib.xm_certify.restype = ctypes.c_int
    lib.xm_round.argtypes = [P, V, I32, V, V, ctypes.POINTER(ctypes.c_double), V]
    lib.xm_round.restype = ctypes.c_int
    lib.xm_recover_tp.argtypes = [P, V, V, V, V, V]
    lib.xm_recover_tp.restype = ctypes.c_int
    lib.xm_adjoint.argtypes = [P, V, V, V, V, D, V, V, ctypes.c_int, D, I32, ctypes.POINTER(_AdjInfo), V]
    lib.xm_adjoint.restype = ctypes.c_int
    lib.xm_build_stats.argtypes = [P, ctypes.POINTER(_KernelStat), I32, ctypes.POINTER(ctypes.c_int32)]
    lib.xm_build_stats.restype = ctypes.c_int
    lib.xm_set_product_kind.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.xm_set_product_kind.restype = ctypes.c_int
    lib.xm_get_product_kind.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.xm_get_product_kind.restype = ctypes.c_int
    lib.xm_set_spmm_kind.argtypes = [P, ctypes.c_int, ctypes.c_int]
    lib.xm_set_spmm_kind.restype = ctypes.c_int
    lib.xm_spmm_timing.argtypes = [P, I32]
    lib.xm_spmm_timing.restype = ctypes.c_int
    lib.xm_spmm_stats.argtypes = [P, ctypes.POINTER(_SpmmStats), I32]
    lib.xm_spmm_stats.restype = ctypes.c_int
    lib.xm_memory_info.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.xm_memory_info.restype = ctypes.c_int
    lib.xm_memory_trim.argtypes = []
    lib.xm_memory_trim.restype = ctypes.c_int64
    lib.xm_spmm_noalloc.argtypes = [P, ctypes.c_int, V, I32, V, V]
    lib.xm_spmm_noalloc.restype = ctypes.c_int
    lib.xm_spmm_noalloc_bytes.argtypes = [P, ctypes.c_int, I32, ctypes.POINTER(ctypes.c_int64)]
    lib.xm_spmm_noalloc_bytes.restype = ctypes.c_int
    lib.xm_last_error.argtypes = []
    lib.xm_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(code: int, allow=()):
    if code != XM_OK and code not in allow:
        raise XMError(code, load_library().xm_last_error().decode())
    return code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dev_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return t.contiguous()


@dataclasses.dataclass
class SolveOptions:
    r0: int = 5
    r_max: int = 7
    lift: float = 1.0             # 0 with r0 = 3: the paper's U^0 = [I, ..., I]
    compute: str = "f64"          # "f64" | "f32" | "bf16"
    grad_tol: float = 0.0         # <= 0: library default
    cert_tol: float = 0.0
    max_outer: int = 0
    max_inner: int = 0
    delta0: float = 0.0
    lanczos_max: int = 0
    lanczos_tol: float = 0.0
    precondition: bool = True
    verbose: bool = False

    def to_c(self) -> _SolveOpts:
        o = _SolveOpts()
        load_library().xm_default_opts(ctypes.byref(o))
        o.r0, o.r_max, o.lift, o.compute = self.r0, self.r_max, self.lift, _DT[self.compute]
        o.grad_tol, o.cert_tol = self.grad_tol, self.cert_tol
        o.max_outer, o.max_inner, o.delta0 = self.max_outer, self.max_inner, self.delta0
        o.lanczos_max, o.lanczos_tol, o.verbose = self.lanczos_max, self.lanczos_tol, int(self.verbose)
        o.precondition = int(self.precondition)
        return o


class Problem:
    """A device-resident data matrix Q built by xm_build_Q (and its handle)."""

    def __init__(self, handle: int, N: int, M: int):
        self._h = ctypes.c_void_p(handle)
        self.N, self.M = N, M
        self.n3 = 3 * N

    def close(self):
        if self._h and self._h.value:
            load_library().xm_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = _ProblemInfo()
        _check(load_library().xm_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _ProblemInfo._fields_}

    def Q_rows(self, row0: int, nrows: int) -> torch.Tensor:
        out = torch.empty((nrows, self.n3), dtype=torch.float64, device="cuda")
        _check(load_library().xm_get_Q_rows(self._h, row0, nrows, _ptr(out), _stream()))
        return out

    def spmm(self, Y: torch.Tensor, dtype: str = "f64") -> torch.Tensor:
        Y = _dev_tensor(Y, torch.float64, "Y")
        out = torch.empty_like(Y)
        _check(load_library().xm_spmm(self._h, _DT[dtype], _ptr(Y), Y.shape[0], _ptr(out), _stream()))
        return out

    def spmm_noalloc(self, Y: torch.Tensor, out: torch.Tensor, dtype: str = "f64") -> torch.Tensor:
        """xm_spmm_noalloc: Y Q into the caller's `out` (same shape as Y), enqueued
        on the current stream with temporaries from the library's fixed scratch."""
        Y = _dev_tensor(Y, torch.float64, "Y")
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
        out = _dev_tensor(out, torch.float64, "out")
        if out.shape != Y.shape:
            raise ValueError("out must have the shape of Y")
        _check(load_library().xm_spmm_noalloc(self._h, _DT[dtype], _ptr(Y), Y.shape[0], _ptr(out), _stream()))
        return out

    def spmm_noalloc_bytes(self, r: int, dtype: str = "f64") -> int:
        n = ctypes.c_int64(0)
        _check(load_library().xm_spmm_noalloc_bytes(self._h, _DT[dtype], r, ctypes.byref(n)))
        return n.value

    def build_stats(self) -> dict:
        """Device time and algorithmic bytes / flops of the main assembly kernels."""
        arr = (_KernelStat * 8)()
        n = ctypes.c_int32(0)
        _check(load_library().xm_build_stats(self._h, arr, 8, ctypes.byref(n)))
        return {arr[k].name.decode(): {"launches": arr[k].launches, "total_ms": arr[k].total_ms,
                                       "bytes": arr[k].bytes, "flops": arr[k].flops} for k in range(min(n.value, 8))}

    def set_spmm_kind(self, dtype: str, kind: str, role: str | None = None):
        """Product kernel for the stored Q of `dtype`: "upper" (reads the upper
        triangle only), "full" (reads all of Q) or, for "f64" and "f32",
        "factored" (from the elimination factors of Q, without reading Q)."""
        k = {"full": 0, "upper": 1, "factored": 2}[kind]
        if role is None:
            _check(load_library().xm_set_spmm_kind(self._h, _DT[dtype], k))
        else:
            _check(load_library().xm_set_product_kind(self._h, {"residual": 0, "curvature": 1}[role], _DT[dtype], k))

    def spmm_kind(self, dtype: str, role: str) -> str:
        """Product kernel in use for `dtype` in `role` ("residual" or "curvature")."""
        k = ctypes.c_int()
        _check(load_library().xm_get_product_kind(self._h, {"residual": 0, "curvature": 1}[role], _DT[dtype],
                                                  ctypes.byref(k)))
        return ("full", "upper", "factored")[k.value]

    def spmm_timing(self, enable: bool = True):
        _check(load_library().xm_spmm_timing(self._h, int(enable)))

    def spmm_stats(self, reset: bool = True) -> dict:
        st = _SpmmStats()
        _check(load_library().xm_spmm_stats(self._h, ctypes.byref(st), int(reset)))
        out = {}
        for name, k in list(_DT.items()) + [("f64_factored", 3), ("f32_factored", 4), ("f64_ginv", 5),
                                            ("f32_ginv", 6), ("f64_fact_rows", 7), ("f32_fact_rows", 8)]:
            out[name] = {"launches": st.launches[k], "total_ms": st.total_ms[k],
                         "bytes_per_launch": st.bytes_per_launch[k]}
        return out

    def solve(self, opts: Optional[SolveOptions] = None, Y0: Optional[torch.Tensor] = None):
        """Riemannian staircase.  Returns (Y [r][3N] float64, info dict)."""
        opts = opts or SolveOptions()
        o = opts.to_c()
        Y_out = torch.empty((opts.r_max, self.n3), dtype=torch.float64, device="cuda")
        info = _SolveInfo()
        r_in = 0
        if Y0 is not None:
            Y0 = _dev_tensor(Y0, torch.float64, "Y0")
            r_in = Y0.shape[0]
        code = load_library().xm_bm_solve(self._h, ctypes.byref(o), _ptr(Y0), r_in, _ptr(Y_out),
                                          ctypes.byref(info), _stream())
        _check(code, allow=(XM_ENOCONV,))
        d = {f: getattr(info, f) for f, _ in _SolveInfo._fields_}
        d["status"] = code
        return Y_out[: info.r].contiguous(), d

    def certify(self, Y: torch.Tensor, tol: float = 0.0, max_iter: int = 0, want_vector: bool = False):
        Y = _dev_tensor(Y, torch.float64, "Y")
        v = torch.empty(self.n3, dtype=torch.float64, device="cuda") if want_vector else None
        c = _Cert()
        _check(load_library().xm_certify(self._h, _ptr(Y), Y.shape[0], tol, max_iter, _ptr(v), ctypes.byref(c),
                                         _stream()))
        d = {f: getattr(c, f) for f, _ in _Cert._fields_}
        if want_vector:
            d["v_min"] = v
        return d

    def round(self, Y: torch.Tensor):
        """Rounded anchored rotations [N,3,3], scales [N] and rho_hat."""
        Y = _dev_tensor(Y, torch.float64, "Y")
        R = torch.empty((self.N, 3, 3), dtype=torch.float64, device="cuda")
        s = torch.empty(self.N, dtype=torch.float64, device="cuda")
        rho = ctypes.c_double(0.0)
        _check(load_library().xm_round(self._h, _ptr(Y), Y.shape[0], _ptr(R), _ptr(s), ctypes.byref(rho),
                                       _stream()))
        return R, s, rho.value


    def recover_tp(self, R: torch.Tensor, s: torch.Tensor):
        """Translations [N,3] and landmarks [M,3] of an anchored rank-3 solution (eq. tpstar)."""
        R = _dev_tensor(R, torch.float64, "R")
        s = _dev_tensor(s, torch.float64, "s")
        t = torch.empty((self.N, 3), dtype=torch.float64, device="cuda")
        pts = torch.empty((self.M, 3), dtype=torch.float64, device="cuda")
        _check(load_library().xm_recover_tp(self._h, _ptr(R), _ptr(s), _ptr(t), _ptr(pts), _stream()))
        return t, pts

    def set_scale_reg(self, lam: float):
        """xm_set_scale_reg: the objective gains lam sum_{k>=1} (s_k^2 - 1)^2."""
        _check(load_library().xm_set_scale_reg(self._h, float(lam)))

    def residuals(self, R: torch.Tensor, s: torch.Tensor, frame_units: bool = True):
        """xm_residuals: (e [n,3], score [n]) at (R, s), caller's observation order."""
        R = _dev_tensor(R, torch.float64, "R")
        s = _dev_tensor(s, torch.float64, "s")
        n = self.info()["n_in"]
        e = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        score = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(load_library().xm_residuals(self._h, _ptr(R), _ptr(s), 1 if frame_units else 0, _ptr(e), _ptr(score),
                                           _stream()))
        return e, score

    def adjoint(self, R, s, gR=None, gs=None, gcost: float = 0.0, dtype=torch.float64, cg_tol: float = 0.0,
                cg_max: int = 0):
        """Gradients (dl/du [n,3], dl/dw [n], info) of a loss l(R, s, f*) with the given partials."""
        R = _dev_tensor(R, torch.float64, "R")
        s = _dev_tensor(s, torch.float64, "s")
        gR = None if gR is None else _dev_tensor(gR.to(torch.float64), torch.float64, "gR")
        gs = None if gs is None else _dev_tensor(gs.to(torch.float64), torch.float64, "gs")
        n = self.info()["n_in"]
        gu = torch.empty((n, 3), dtype=dtype, device="cuda")
        gw = torch.empty(n, dtype=dtype, device="cuda")
        gdt = XM_F64 if dtype == torch.float64 else XM_F32
        inf = _AdjInfo()
        _check(load_library().xm_adjoint(self._h, _ptr(R), _ptr(s), _ptr(gR), _ptr(gs), float(gcost), _ptr(gu),
                                         _ptr(gw), gdt, cg_tol, cg_max, ctypes.byref(inf), _stream()))
        return gu, gw, {f: getattr(inf, f) for f, _ in _AdjInfo._fields_}


def memory_info() -> dict:
    """Bytes of the library's device pool in live and in cached (free) blocks."""
    live, cached = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load_library().xm_memory_info(ctypes.byref(live), ctypes.byref(cached)))
    return {"live": live.value, "cached": cached.value}


def memory_trim() -> int:
    """Return the pool's cached blocks to the runtime; the bytes released."""
    return int(load_library().xm_memory_trim())


class NotTightError(RuntimeError):
    """The solve did not reach a certified optimum at which the relaxation is
    tight, so the implicit-function gradient of the rotations is not defined."""


class XMSolve(torch.autograd.Function):
    """(R [N,3,3], s [N], f*) = certified SBA optimum of (u, w); differentiable in u and w.

    forward: xm_build_Q -> xm_bm_solve -> xm_round (f* is the cost of the
    rounded, anchored solution); backward: xm_adjoint (envelope theorem for f*,
    implicit-function theorem for R and s).  The gradients are those of a tight
    certified optimum, so forward raises NotTightError when the solve is not
    certified, did not converge, or rounding loses more than `eta_tol`
    (eq. suboptimality: the relaxation is not tight there), and backward raises
    XMError when the adjoint's CG does not converge.
    """

    @staticmethod
    def forward(ctx, u, w, frame, landmark, N, M, opts=None, eta_tol=1e-6):
        opts = opts or SolveOptions()
        keep = {"f64": (), "f32": ("f32",), "bf16": ("f32", "bf16")}[opts.compute]
        P = build_Q(N, M, frame, landmark, u, w, keep=keep)
        Y, info = P.solve(opts)
        R, s, rho = P.round(Y)
        eta = (rho - info["cost"]) / (1.0 + abs(rho) + abs(info["cost"]))
        if info["status"] != XM_OK or not info["certified"] or eta > eta_tol:
            P.close()
            raise NotTightError(f"solve status={info['status']} certified={info['certified']} "
                                f"rank={info['r']} eta={eta:.3e} (tol {eta_tol:.1e}): the gradient of the "
                                "optimum is defined at tight certified optima only")
        ctx.problem = P
        ctx.info = dict(info, eta=eta)
        ctx.u_dtype, ctx.w_dtype = u.dtype, w.dtype
        ctx.save_for_backward(R, s)
        return R, s, torch.tensor(rho, dtype=torch.float64, device=R.device)

    @staticmethod
    def backward(ctx, gR, gs, gcost):
        R, s = ctx.saved_tensors
        gc = 0.0 if gcost is None else float(gcost)
        gu, gw, _ = ctx.problem.adjoint(R, s, gR, gs, gc, dtype=torch.float64)
        return gu.to(ctx.u_dtype), gw.to(ctx.w_dtype), None, None, None, None, None, None


def drop_largest(score: torch.Tensor, frac: float = 0.1):
    """xm_drop_largest: (keep mask uint8 [n], number dropped)."""
    score = _dev_tensor(score, torch.float64, "score")
    keep = torch.empty(score.shape[0], dtype=torch.uint8, device="cuda")
    nd = ctypes.c_int64(0)
    _check(load_library().xm_drop_largest(_ptr(score), score.shape[0], float(frac), _ptr(keep), ctypes.byref(nd),
                                          _stream()))
    return keep, nd.value


def guard_frames(N: int, M: int, frame: torch.Tensor, landmark: torch.Tensor, keep: torch.Tensor,
                 min_links: int = 6):
    """xm_guard_frames on a copy of `keep` (uint8 [n]): (guarded keep mask, number restored)."""
    frame = _dev_tensor(frame, torch.int32, "frame")
    landmark = _dev_tensor(landmark, torch.int32, "landmark")
    if landmark.shape != frame.shape or keep.shape != frame.shape:
        raise ValueError("frame, landmark and keep must have one entry per observation")
    out = _dev_tensor(keep, torch.uint8, "keep").clone()
    nr = ctypes.c_int64(0)
    _check(load_library().xm_guard_frames(N, M, frame.shape[0], _ptr(frame), _ptr(landmark), int(min_links),
                                          _ptr(out), ctypes.byref(nr), _stream()))
    return out, nr.value


def align_similarity(P: torch.Tensor, Q: torch.Tensor, w: Optional[torch.Tensor] = None) -> dict:
    """xm_align_similarity: s, R [3,3], t [3] minimising sum w |s R P_i + t - Q_i|^2
    (P, Q [n,3] float64 on the device), and the weighted RMS residual."""
    P = _dev_tensor(P, torch.float64, "P")
    Q = _dev_tensor(Q, torch.float64, "Q")
    if P.dim() != 2 or P.shape[1] != 3 or Q.shape != P.shape:
        raise ValueError("P and Q must both be [n, 3]")
    if w is not None:
        w = _dev_tensor(w, torch.float64, "w")
        if w.shape != (P.shape[0],):
            raise ValueError("w must be [n]")
    out = (ctypes.c_double * 14)()
    _check(load_library().xm_align_similarity(P.shape[0], _ptr(P), _ptr(Q), _ptr(w), out,
                                              _stream()))
    v = list(out)
    return {"s": v[0], "R": torch.tensor(v[1:10], dtype=torch.float64).reshape(3, 3),
            "t": torch.tensor(v[10:13], dtype=torch.float64), "rmse": v[13]}


def xm2(N: int, M: int, frame: torch.Tensor, landmark: torch.Tensor, u: torch.Tensor,
        w: Optional[torch.Tensor] = None, opts: Optional["SolveOptions"] = None, frac: float = 0.1,
        frame_units: bool = True, keep=("f32",), min_links: int = 6):
    """XM^2 (Section "Structure from Motion with XM"): xm_build_Q -> xm_bm_solve
    -> xm_round -> xm_residuals -> xm_drop_largest -> xm_guard_frames ->
    xm_build_Q_masked -> xm_bm_solve (started from the first solution) ->
    xm_round.  Returns a dict with both passes' (R, s, rho_hat, info), the
    scores, the keep mask, the numbers deleted and restored."""
    opts = opts or SolveOptions()
    P1 = build_Q(N, M, frame, landmark, u, w, keep=keep)
    Y1, i1 = P1.solve(opts)
    R1, s1, rho1 = P1.round(Y1)
    _, score = P1.residuals(R1, s1, frame_units)
    P1.close()
    mask, n_drop = drop_largest(score, frac)
    mask, n_rest = guard_frames(N, M, frame, landmark, mask, min_links)
    P2 = build_Q(N, M, frame, landmark, u, w, keep=keep, mask=mask)
    Y2, i2 = P2.solve(opts, Y0=Y1[: i1["r"]])
    R2, s2, rho2 = P2.round(Y2)
    return {"first": (R1, s1, rho1, i1), "second": (R2, s2, rho2, i2), "score": score, "keep": mask,
            "n_dropped": n_drop - n_rest, "n_restored": n_rest, "problem": P2, "Y": Y2}


def build_Q(N: int, M: int, frame: torch.Tensor, landmark: torch.Tensor, u: torch.Tensor,
            w: Optional[torch.Tensor] = None, keep=("f32",), mask: Optional[torch.Tensor] = None) -> Problem:
    """xm_build_Q on device tensors (frame/landmark int32, u [n,3] and w [n] float64 or float32);
    with `mask` (uint8 [n], nonzero = use), xm_build_Q_masked."""
    lib = load_library()
    frame = _dev_tensor(frame, torch.int32, "frame")
    landmark = _dev_tensor(landmark, torch.int32, "landmark")
    if u.dtype not in (torch.float64, torch.float32):
        raise TypeError("u must be float64 or float32")
    u = _dev_tensor(u, u.dtype, "u")
    u_dt = XM_F64 if u.dtype == torch.float64 else XM_F32
    w_dt = XM_F64
    if w is not None:
        if w.dtype not in (torch.float64, torch.float32):
            raise TypeError("w must be float64 or float32")
        w = _dev_tensor(w, w.dtype, "w")
        w_dt = XM_F64 if w.dtype == torch.float64 else XM_F32
    if u.dim() != 2 or u.shape[1] != 3 or u.shape[0] != frame.shape[0] or landmark.shape[0] != frame.shape[0]:
        raise ValueError("shapes: frame [n], landmark [n], u [n, 3]")
    copies = 0
    for k in keep:
        copies |= {"f32": XM_KEEP_F32, "bf16": XM_KEEP_BF16}[k]
    h = ctypes.c_void_p(0)
    if mask is None:
        _check(lib.xm_build_Q(N, M, frame.shape[0], _ptr(frame), _ptr(landmark), _ptr(u), u_dt, _ptr(w), w_dt,
                              copies, _stream(), ctypes.byref(h)))
    else:
        mask = _dev_tensor(mask, torch.uint8, "mask")
        if mask.shape != frame.shape:
            raise ValueError("mask must have one entry per observation")
        _check(lib.xm_build_Q_masked(N, M, frame.shape[0], _ptr(frame), _ptr(landmark), _ptr(u), u_dt, _ptr(w),
                                     w_dt, _ptr(mask), copies, _stream(), ctypes.byref(h)))
    return Problem(h.value, N, M)
