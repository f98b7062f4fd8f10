"""Python binding of liblabpsd, the MI355X (gfx950) LABPSD eigensolver.

Argument marshalling only: every step of the solver runs in the HIP kernels and
host C++ of liblabpsd.so; this module passes pointers and sizes.  PyTorch supplies
device memory and the current HIP stream.  Block vectors on the device are torch
tensors of shape (columns, ld) -- row j of the tensor is column j of the
column-major block the library sees.

The library must be built first (``python paper_1308_2445_amd/build.py``); if it
is missing, importing this package raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
# torch first: the process must hold exactly one HIP runtime, and liblabpsd.so then
# binds to the one torch already loaded (same soname) instead of a second copy
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblabpsd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("liblabpsd.so is not built: run `python paper_1308_2445_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

OK, NOT_CONVERGED, PENDING = 0, 1, 2
EINVAL, ENOMEM, EHIP, ENOTSPD, ERANK, ESTATE = -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
PANELS_FP64, PANELS_FP32, FACTOR_FP32, APPLY_LEVELS = 1, 2, 4, 8
HYBRID, GLOBAL_ONLY, LOCAL_ONLY = 0, 1, 2
REFINE_MINRES, REFINE_ONESTEP = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1

_STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTSPD",
                 -5: "ERANK", -6: "ESTATE"}

#: names of the entries of labpsd_stats.t_step_s / n_launch
STEP_NAMES = ["products_psi", "residual", "global_precond", "local_refine", "products_p", "gram",
              "rayleigh_ritz", "block_update", "cast"]


class LabpsdError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.labpsd_last_error().decode()
        super().__init__("%s: %s (%s)" % (where, _STATUS_NAMES.get(code, code), msg))
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int), ("m0", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("sigma0", ctypes.c_double),
                ("precision", ctypes.c_int), ("refresh_every", ctypes.c_int),
                ("timing", ctypes.c_int), ("reorth_tol", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("minres_iters", ctypes.c_int64),
                ("localized_cols", ctypes.c_int64), ("rank_dropped", ctypes.c_int),
                ("refreshes", ctypes.c_int), ("hp", ctypes.c_double), ("la", ctypes.c_double),
                ("t_solve_s", ctypes.c_double), ("t_step_s", ctypes.c_double * 12),
                ("n_launch", ctypes.c_int64 * 12), ("n_cols", ctypes.c_int64 * 12),
                ("reorths", ctypes.c_int)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("t_step_s", "n_launch", "n_cols")}
        d["t_step_s"] = {STEP_NAMES[i]: self.t_step_s[i] for i in range(len(STEP_NAMES))}
        d["n_launch"] = {STEP_NAMES[i]: int(self.n_launch[i]) for i in range(len(STEP_NAMES))}
        d["cols"] = {STEP_NAMES[i]: int(self.n_cols[i]) for i in range(len(STEP_NAMES))}
        return d


class FactorInfo(ctypes.Structure):
    _fields_ = [("n_supernodes", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("nnz_factor", ctypes.c_int64), ("flops_factor", ctypes.c_double),
                ("t_order_s", ctypes.c_double), ("t_factor_s", ctypes.c_double),
                ("t_upload_s", ctypes.c_double)]


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int
_d = ctypes.c_double

_SIGS = {
    "labpsd_ctx_create": ([_i32, _p, ctypes.POINTER(_p)], _i32),
    "labpsd_ctx_destroy": ([_p], None),
    "labpsd_ctx_set_stream": ([_p, _p], _i32),
    "labpsd_last_error": ([], ctypes.c_char_p),
    "labpsd_version": ([], ctypes.c_char_p),
    "labpsd_problem_create": ([_p, _i64, _i64, _p, _p, _p, _p, _i32, ctypes.POINTER(_p)], _i32),
    "labpsd_problem_update_h": ([_p, _p, _i32], _i32),
    "labpsd_problem_set_nonlocal": ([_p, _i32, _p, _p, _p, _p], _i32),
    "labpsd_problem_create_hermitian": ([_p, _i64, _i64, _p, _p, _p, _p, _p, _p, ctypes.POINTER(_p)], _i32),
    "labpsd_problem_update_h_hermitian": ([_p, _p, _p], _i32),
    "labpsd_solve_hermitian": ([_p, ctypes.POINTER(SolveParams), _p, _p, _i32, _p, _p, _p, _p,
                                ctypes.POINTER(ctypes.c_int), _i32, ctypes.POINTER(Stats)], _i32),
    "labpsd_problem_destroy": ([_p], None),
    "labpsd_problem_n": ([_p], _i64),
    "labpsd_set_global_precond": ([_p, _d, _p, ctypes.c_uint], _i32),
    "labpsd_set_local_precond": ([_p, _d, _d, _d, _i32, _i32], _i32),
    "labpsd_get_factor_info": ([_p, ctypes.POINTER(FactorInfo)], _i32),
    "labpsd_set_refine_method": ([_p, _i32], _i32),
    "labpsd_solve": ([_p, ctypes.POINTER(SolveParams), _p, _p, _i32, _p, _p, _p, _p,
                      ctypes.POINTER(ctypes.c_int), _i32, ctypes.POINTER(Stats)], _i32),
    "labpsd_spmm": ([_p, _p, _i64, _i32, _p, _p, _i64], _i32),
    "labpsd_spmm_shifted": ([_p, _i32, _p, _i64, _i32, _p, _p, _i64], _i32),
    "labpsd_residual": ([_p, _i64, _i32, _p, _p, _i64, _p, _d, _p, _i64, _p, _p], _i32),
    "labpsd_residual_noalloc": ([_p, _i64, _i32, _p, _p, _i64, _p, _d, _p, _i64, _p, _p], _i32),
    "labpsd_precond_apply": ([_p, _i32, _p, _i64, _i32, _p, _i64], _i32),
    "labpsd_local_refine": ([_p, _i32, _p, _i64, _p, _i64, _i32, _p, _p, _d, _i32, _p], _i32),
    "labpsd_gram": ([_p, _i64, _i32, _p, _p, _p, _i64, _p, _p, _i64], _i32),
    "labpsd_rayleigh_ritz": ([_p, _i32, _i32, _p, _p, _i64, _p, _p, _i64, _p], _i32),
    "labpsd_block_update": ([_p, _i64, _i32, _i32, _p, _p, _p, _i64, _p, _i64, _p, _p, _p, _i64],
                            _i32),
    "labpsd_server_create": ([_p, ctypes.c_size_t, _i32, ctypes.POINTER(_p)], _i32),
    "labpsd_server_submit": ([_p, _p, _p, ctypes.POINTER(SolveParams), _p, ctypes.POINTER(ctypes.c_uint64)],
                             _i32),
    "labpsd_server_poll": ([_p, ctypes.c_uint64, _p, _p, ctypes.POINTER(Stats), _p], _i32),
    "labpsd_server_wait": ([_p, ctypes.c_uint64, _p, _p, ctypes.POINTER(Stats), _p], _i32),
    "labpsd_solve_footprint": ([_i64, _i32, _i32, _i32], ctypes.c_size_t),
    "labpsd_server_memory": ([_p, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], _i32),
    "labpsd_server_destroy": ([_p], None),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

#: every C symbol the header declares (checked by the CPU tests)
EXPORTED = sorted(_SIGS)


def _check(rc: int, where: str, allow=(OK,)) -> int:
    if rc not in allow:
        raise LabpsdError(rc, where)
    return rc


def version() -> str:
    return _lib.labpsd_version().decode()


def _ptr(a) -> int | None:
    """Address of a numpy array or torch tensor (None passes NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ld(t) -> int:
    """Leading dimension of a (columns, ld) torch tensor whose rows are contiguous."""
    if t.dim() == 1:
        return t.shape[0]
    if t.shape[0] <= 1:
        return t.shape[1]          # one column: its stride is not meaningful
    assert t.stride(1) == 1, "block tensors must have contiguous rows (shape (cols, ld))"
    return t.stride(0)


class Context:
    """A library context bound to a HIP device and the current torch stream."""

    def __init__(self, device: int = 0):
        import torch
        torch.cuda.set_device(device)
        h = _p()
        _check(_lib.labpsd_ctx_create(device, _stream(), ctypes.byref(h)), "labpsd_ctx_create")
        self.h = h
        self.device = device

    def sync_stream(self):
        _check(_lib.labpsd_ctx_set_stream(self.h, _stream()), "labpsd_ctx_set_stream")

    def close(self):
        if self.h:
            _lib.labpsd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class SolveResult:
    status: int
    lam: object
    X: object
    res_hist: np.ndarray
    stats: dict
    ritz_hist: object = None   # Ritz values at the start of every iteration (iterations x b)

    @property
    def converged(self) -> bool:
        return self.status == OK


class Problem:
    """The pencil (H, S) on one shared CSR pattern, resident on the device."""

    def __init__(self, ctx: Context, n, rowptr, col, h_val, s_val):
        """rowptr int64[n+1], col int32[nnz], h_val / s_val float64[nnz]: numpy arrays (host)
        or torch device tensors (all four on the same side)."""
        self.ctx = ctx
        self.n = int(n)
        if isinstance(rowptr, np.ndarray) or not hasattr(rowptr, "is_cuda"):
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            h_val = np.ascontiguousarray(h_val, dtype=np.float64)
            s_val = np.ascontiguousarray(s_val, dtype=np.float64)
            where = MEM_HOST
        else:
            import torch
            for t, dt in ((rowptr, torch.int64), (col, torch.int32), (h_val, torch.float64),
                          (s_val, torch.float64)):
                assert t.is_cuda and t.dtype == dt and t.is_contiguous()
            where = MEM_DEVICE
        self.nnz = int(col.shape[0])
        h = _p()
        ctx.sync_stream()
        _check(_lib.labpsd_problem_create(ctx.h, self.n, self.nnz, _ptr(rowptr), _ptr(col), _ptr(h_val),
                                          _ptr(s_val), where, ctypes.byref(h)), "labpsd_problem_create")
        self.h = h

    @classmethod
    def from_pencil(cls, ctx: Context, P) -> "Problem":
        """The pencil of a pufe cell, with its nonlocal term when it has one (P.F, P.G); a
        complex (k-point) cell gives a HermitianProblem."""
        if np.iscomplexobj(P.h_val) or np.iscomplexobj(P.s_val):
            return HermitianProblem(ctx, P.n, P.rowptr, P.col, P.h_val, P.s_val)
        pr = cls(ctx, P.n, P.rowptr, P.col, P.h_val, P.s_val)
        if getattr(P, "F", None) is not None:
            pr.set_nonlocal(P.F, P.G)
        return pr

    def update_h(self, h_val):
        """New H values on the same pattern: numpy array or torch device tensor."""
        if isinstance(h_val, np.ndarray) or not hasattr(h_val, "is_cuda"):
            h_val = np.ascontiguousarray(h_val, dtype=np.float64)
            where = MEM_HOST
        else:
            import torch
            assert h_val.is_cuda and h_val.dtype == torch.float64 and h_val.is_contiguous()
            where = MEM_DEVICE
        self.ctx.sync_stream()
        _check(_lib.labpsd_problem_update_h(self.h, _ptr(h_val), where), "labpsd_problem_update_h")

    def set_nonlocal(self, F, G):
        """The nonlocal term H_nl = F G F^T: F an n x k scipy sparse matrix, G k x k."""
        import scipy.sparse as sp
        Fc = sp.csc_matrix(F)
        Fc.sort_indices()
        k = int(Fc.shape[1])
        cp = np.ascontiguousarray(Fc.indptr, dtype=np.int64)
        ri = np.ascontiguousarray(Fc.indices, dtype=np.int32)
        fv = np.ascontiguousarray(Fc.data, dtype=np.float64)
        Gm = np.asfortranarray(np.asarray(G, dtype=np.float64).reshape(k, k))
        self.ctx.sync_stream()
        _check(_lib.labpsd_problem_set_nonlocal(self.h, k, _ptr(cp), _ptr(ri), _ptr(fv), _ptr(Gm)),
               "labpsd_problem_set_nonlocal")

    def set_global_precond(self, eps_bar: float, coords=None, panels: int = 0):
        """panels: PANELS_FP64 | PANELS_FP32 mask of the factor copies to upload (neither: both),
        optionally | FACTOR_FP32 for a numeric factorisation in single precision, | APPLY_LEVELS for
        one launch per elimination-tree level and phase instead of the single-launch sweep."""
        c = None if coords is None else np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
        self.ctx.sync_stream()
        _check(_lib.labpsd_set_global_precond(self.h, float(eps_bar), _ptr(c), int(panels)),
               "labpsd_set_global_precond")

    def set_local_precond(self, tau1=0.1, tau2=0.1, eta=0.25, max_inner=20, mode=HYBRID):
        _check(_lib.labpsd_set_local_precond(self.h, tau1, tau2, eta, max_inner, mode),
               "labpsd_set_local_precond")

    def set_refine_method(self, method: int):
        """REFINE_MINRES (Section 4) or REFINE_ONESTEP (the conclusions' one-step method)."""
        _check(_lib.labpsd_set_refine_method(self.h, int(method)), "labpsd_set_refine_method")

    def factor_info(self) -> dict:
        fi = FactorInfo()
        _check(_lib.labpsd_get_factor_info(self.h, ctypes.byref(fi)), "labpsd_get_factor_info")
        return {f: getattr(fi, f) for f, _ in fi._fields_}

    def solve(self, nev: int, m0: int, X0, *, tol=1e-8, max_outer=200, sigma0=0.0,
              precision=FP64, refresh_every=10, timing=False, E0=None, device_out=False, reorth_tol=0.0,
              seed=0):
        """Run LABPSD from X0 (numpy n x b Fortran array, torch (b, n) device tensor, or None for
        the library's seeded random start).
        reorth_tol: threshold on max |Psi^T S Psi - I| at a refresh (0: 1e-10; negative: always)."""
        import torch
        b = nev + m0
        n = self.n
        self.ctx.sync_stream()
        if X0 is None:
            in_where = MEM_HOST
        elif isinstance(X0, np.ndarray):
            X0 = np.asfortranarray(X0, dtype=np.float64)
            assert X0.shape == (n, b)
            in_where = MEM_HOST
        else:
            assert tuple(X0.shape) == (b, n) and X0.is_contiguous() and X0.dtype == torch.float64
            in_where = MEM_DEVICE
        E0a = None if E0 is None else np.ascontiguousarray(E0, dtype=np.float64)
        prm = SolveParams(nev, m0, tol, max_outer, sigma0, precision, refresh_every, 1 if timing else 0,
                          reorth_tol, seed)
        hist = np.zeros(max_outer * nev + nev)
        rhist = np.zeros((max_outer + 1) * b)
        nh = ctypes.c_int(0)
        st = Stats()
        if device_out:
            lam = torch.empty(nev, dtype=torch.float64, device="cuda")
            X = torch.empty((nev, n), dtype=torch.float64, device="cuda")
            out_where = MEM_DEVICE
            hist_arg = torch.empty(max_outer * nev + nev, dtype=torch.float64, device="cuda")
            rhist_arg = torch.empty((max_outer + 1) * b, dtype=torch.float64, device="cuda")
        else:
            lam = np.zeros(nev)
            X = np.zeros((n, nev), order="F")
            out_where = MEM_HOST
            hist_arg = hist
            rhist_arg = rhist
        rc = _lib.labpsd_solve(self.h, ctypes.byref(prm), _ptr(X0), _ptr(E0a), in_where, _ptr(lam), _ptr(X),
                               _ptr(hist_arg), _ptr(rhist_arg), ctypes.byref(nh), out_where, ctypes.byref(st))
        _check(rc, "labpsd_solve", allow=(OK, NOT_CONVERGED))
        # the history is a host array, or (device_out) a device tensor view
        src = hist_arg if hist_arg is not None else hist
        return SolveResult(status=rc, lam=lam, X=X, res_hist=src[: nh.value * nev].reshape(nh.value, nev),
                           stats=st.as_dict(), ritz_hist=rhist_arg[: nh.value * b].reshape(nh.value, b))

    def close(self):
        if getattr(self, "h", None):
            _lib.labpsd_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HermitianProblem(Problem):
    """A complex Hermitian pencil (a k-point), solved through its real embedding."""

    def __init__(self, ctx: Context, n, rowptr, col, h_val, s_val):
        self.ctx = ctx
        self.n = int(n)
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        h_val = np.asarray(h_val, dtype=np.complex128)
        s_val = np.asarray(s_val, dtype=np.complex128)
        hr, hi = np.ascontiguousarray(h_val.real), np.ascontiguousarray(h_val.imag)
        sr, si = np.ascontiguousarray(s_val.real), np.ascontiguousarray(s_val.imag)
        self.nnz = int(col.shape[0])
        h = _p()
        ctx.sync_stream()
        _check(_lib.labpsd_problem_create_hermitian(ctx.h, self.n, self.nnz, _ptr(rowptr), _ptr(col), _ptr(hr),
                                                    _ptr(hi), _ptr(sr), _ptr(si), ctypes.byref(h)),
               "labpsd_problem_create_hermitian")
        self.h = h

    def update_h(self, h_val):
        h_val = np.asarray(h_val, dtype=np.complex128)
        hr, hi = np.ascontiguousarray(h_val.real), np.ascontiguousarray(h_val.imag)
        self.ctx.sync_stream()
        _check(_lib.labpsd_problem_update_h_hermitian(self.h, _ptr(hr), _ptr(hi)), "labpsd_problem_update_h_hermitian")

    def solve(self, nev: int, m0: int, X0, *, tol=1e-8, max_outer=200, sigma0=0.0, precision=FP64,
              refresh_every=10, timing=False, E0=None, reorth_tol=0.0, seed=0, device_out=False):
        """X0: complex n x (nev + m0) numpy array or None.  Returns complex X (n x nev); the
        histories are those of the embedded real solve (2 nev residuals per iteration)."""
        b = nev + m0
        n = self.n
        self.ctx.sync_stream()
        x0 = None
        if X0 is not None:
            x0 = np.asfortranarray(np.asarray(X0, dtype=np.complex128))
            assert x0.shape == (n, b)
        E0a = None if E0 is None else np.ascontiguousarray(E0, dtype=np.float64)
        prm = SolveParams(nev, m0, tol, max_outer, sigma0, precision, refresh_every, 1 if timing else 0,
                          reorth_tol, seed)
        hist = np.zeros(2 * (max_outer + 1) * nev)
        rhist = np.zeros(2 * (max_outer + 1) * b)
        nh = ctypes.c_int(0)
        st = Stats()
        lam = np.zeros(nev)
        X = np.zeros((n, nev), dtype=np.complex128, order="F")
        rc = _lib.labpsd_solve_hermitian(self.h, ctypes.byref(prm), _ptr(x0), _ptr(E0a), MEM_HOST, _ptr(lam),
                                         _ptr(X), _ptr(hist), _ptr(rhist), ctypes.byref(nh), MEM_HOST,
                                         ctypes.byref(st))
        _check(rc, "labpsd_solve_hermitian", allow=(OK, NOT_CONVERGED))
        return SolveResult(status=rc, lam=lam, X=X, res_hist=hist[: nh.value * 2 * nev].reshape(nh.value, 2 * nev),
                           stats=st.as_dict(), ritz_hist=rhist[: nh.value * 2 * b].reshape(nh.value, 2 * b))


# ------------------------------------------------------------------ hot-path steps
# Device tensors only; blocks are (columns, ld) tensors.

def labpsd_spmm(prob: Problem, X, YH, YS):
    prob.ctx.sync_stream()
    _check(_lib.labpsd_spmm(prob.h, _ptr(X), _ld(X), X.shape[0], _ptr(YH), _ptr(YS), _ld(YH)), "labpsd_spmm")


def labpsd_spmm_shifted(prob: Problem, precision: int, X, shift, Y):
    prob.ctx.sync_stream()
    _check(_lib.labpsd_spmm_shifted(prob.h, precision, _ptr(X), _ld(X), X.shape[0], _ptr(shift), _ptr(Y),
                                    _ld(Y)), "labpsd_spmm_shifted")


def labpsd_residual(ctx: Context, n: int, m: int, PsiH, PsiS, E, sigma0: float, R, res, rnorm):
    ctx.sync_stream()
    _check(_lib.labpsd_residual(ctx.h, n, m, _ptr(PsiH), _ptr(PsiS), _ld(PsiH), _ptr(E), sigma0, _ptr(R),
                                _ld(R), _ptr(res), _ptr(rnorm)), "labpsd_residual")


def labpsd_residual_noalloc(ctx: Context, n: int, m: int, PsiH, PsiS, E, sigma0: float, R, res, rnorm):
    ctx.sync_stream()
    _check(_lib.labpsd_residual_noalloc(ctx.h, n, m, _ptr(PsiH), _ptr(PsiS), _ld(PsiH), _ptr(E), sigma0,
                                        _ptr(R), _ld(R), _ptr(res), _ptr(rnorm)), "labpsd_residual_noalloc")


def labpsd_precond_apply(prob: Problem, precision: int, R, P):
    prob.ctx.sync_stream()
    _check(_lib.labpsd_precond_apply(prob.h, precision, _ptr(R), _ld(R), R.shape[0], _ptr(P), _ld(P)),
           "labpsd_precond_apply")


def labpsd_local_refine(prob: Problem, precision: int, R, P, cols, shift, eta: float, max_inner: int, its):
    prob.ctx.sync_stream()
    _check(_lib.labpsd_local_refine(prob.h, precision, _ptr(R), _ld(R), _ptr(P), _ld(P), cols.shape[0],
                                    _ptr(cols), _ptr(shift), eta, max_inner, _ptr(its)), "labpsd_local_refine")


def labpsd_gram(ctx: Context, n: int, k: int, Z, ZH, ZS, HR, SR):
    ctx.sync_stream()
    _check(_lib.labpsd_gram(ctx.h, n, k, _ptr(Z), _ptr(ZH), _ptr(ZS), _ld(Z), _ptr(HR), _ptr(SR), _ld(HR)),
           "labpsd_gram")


def labpsd_rayleigh_ritz(ctx: Context, k: int, nwant: int, HR, SR, gamma, W, info):
    ctx.sync_stream()
    _check(_lib.labpsd_rayleigh_ritz(ctx.h, k, nwant, _ptr(HR), _ptr(SR), _ld(HR), _ptr(gamma), _ptr(W),
                                     _ld(W), _ptr(info)), "labpsd_rayleigh_ritz")


def labpsd_block_update(ctx: Context, n: int, k: int, b: int, Z, ZH, ZS, W, Psi, PsiH, PsiS):
    ctx.sync_stream()
    _check(_lib.labpsd_block_update(ctx.h, n, k, b, _ptr(Z), _ptr(ZH), _ptr(ZS), _ld(Z), _ptr(W), _ld(W),
                                    _ptr(Psi), _ptr(PsiH), _ptr(PsiS), _ld(Psi)), "labpsd_block_update")


# ------------------------------------------------------------------ serving

@dataclasses.dataclass
class Served:
    status: int
    lam: np.ndarray
    X: np.ndarray
    stats: dict
    submitted: float
    started: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.submitted

    @property
    def converged(self) -> bool:
        return self.status == OK


def solve_footprint(n: int, nev: int, m0: int, precision: int = FP64) -> int:
    return int(_lib.labpsd_solve_footprint(n, nev, m0, precision))


class Server:
    """Continuous-batching request loop over resident systems (labpsd_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        h = _p()
        _check(_lib.labpsd_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)),
               "labpsd_server_create")
        self.h = h
        self.ctx = ctx
        self._shape = {}

    def submit(self, system: Problem, nev: int, m0: int, *, X0=None, h_val=None, tol=1e-8, max_outer=200,
               sigma0=0.0, precision=FP64, refresh_every=10) -> int:
        prm = SolveParams(nev, m0, tol, max_outer, sigma0, precision, refresh_every, 0)
        x = None if X0 is None else np.asfortranarray(X0, dtype=np.float64)
        if x is not None:
            assert x.shape == (system.n, nev + m0)
        hv = None if h_val is None else np.ascontiguousarray(h_val, dtype=np.float64)
        rid = ctypes.c_uint64(0)
        _check(_lib.labpsd_server_submit(self.h, system.h, _ptr(hv), ctypes.byref(prm), _ptr(x),
                                         ctypes.byref(rid)), "labpsd_server_submit")
        self._shape[rid.value] = (system.n, nev)
        return rid.value

    def _collect(self, rid: int, block: bool):
        n, nev = self._shape[rid]
        lam = np.zeros(nev)
        X = np.zeros((n, nev), order="F")
        st = Stats()
        times = np.zeros(3)
        fn = _lib.labpsd_server_wait if block else _lib.labpsd_server_poll
        rc = fn(self.h, rid, _ptr(lam), _ptr(X), ctypes.byref(st), _ptr(times))
        if rc == PENDING:
            return None
        del self._shape[rid]
        _check(rc, "labpsd_server_wait", allow=(OK, NOT_CONVERGED))
        return Served(status=rc, lam=lam, X=X, stats=st.as_dict(), submitted=times[0], started=times[1],
                      finished=times[2])

    def poll(self, rid: int):
        return self._collect(rid, False)

    def wait(self, rid: int) -> Served:
        return self._collect(rid, True)

    def memory(self) -> dict:
        """Device bytes the server holds now and at most so far (slot workspaces and
        resident blocks, as charged against the budget)."""
        held, peak = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.labpsd_server_memory(self.h, ctypes.byref(held), ctypes.byref(peak)), "labpsd_server_memory")
        return {"held": held.value, "peak": peak.value}

    def close(self):
        if getattr(self, "h", None):
            _lib.labpsd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
