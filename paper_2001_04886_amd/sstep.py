"""Python binding of libsstep.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors to device pointers and the current HIP stream, and fills the C
structs of ``include/sstep.h``.  It raises if the library is missing or fails
to load -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsstep.so")

OK, NOT_CONVERGED, ERR_ARG, ERR_BREAKDOWN, ERR_NONFINITE, ERR_HIP, ERR_NOMEM = 0, 1, -1, -2, -3, -4, -5
MONOMIAL, CHEBYSHEV, NEWTON = 0, 1, 2
FP64, MIXED = 0, 1
METHOD_OMIN, METHOD_GMRES = 0, 1
PRECOND_NONE, PRECOND_ILU0 = 0, 1
ORTH_CHOL, ORTH_MGS = 0, 1
K_MPK, K_GRAM, K_UPDATE, K_RESID, K_SCALAR, K_VEC, K_NCLASS = 0, 1, 2, 3, 4, 5, 6
KERNEL_CLASSES = ("mpk", "gram", "update", "resid", "scalar", "vec")

# every symbol declared in include/sstep.h
EXPORTS = (
    "sstep_default_options", "sstep_status_string", "sstep_workspace_bytes",
    "sstep_gmres_solve", "sstep_gmres_solve_noalloc", "sstep_omin_solve", "sstep_stencil_apply",
    "sstep_kernel_mpk", "sstep_kernel_gram", "sstep_kernel_update",
    "sstep_batch_workspace_bytes", "sstep_batch_plan_create", "sstep_batch_plan_execute",
    "sstep_batch_plan_destroy", "sstep_gmres_solve_batched",
    "sstep_cnn_param_count", "sstep_cnn_workspace_bytes", "sstep_cnn_forward",
    "sstep_cnn_gradient", "sstep_cnn_adam", "sstep_cnn_train_step", "sstep_x0_predict",
    "sstep_grid_pool", "sstep_x0_coarse_workspace_bytes", "sstep_x0_predict_coarse",
    "sstep_precond_workspace_bytes", "sstep_ilu0_factor", "sstep_ilu0_solve", "sstep_ilu0_mul",
)


class StencilC(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("c", C.c_double * 7), ("coef", C.c_void_p)]


class OptionsC(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("precision", C.c_int32), ("basis", C.c_int32),
                ("profile", C.c_int32), ("sigma", C.c_double), ("inner_tol", C.c_double),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p), ("batch_threads", C.c_int32),
                ("batch_wgs_per_cu", C.c_int32), ("batch_graph", C.c_int32),
                ("batch_team", C.c_int32), ("precond", C.c_int32), ("orth", C.c_int32),
                ("graph", C.c_int32), ("batch_gram_cols", C.c_int32)]


class InfoC(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cycles", C.c_int32),
                ("matvecs", C.c_int32), ("rel_resid", C.c_double), ("rel_resid_est", C.c_double),
                ("sigma", C.c_double), ("cheb_centre", C.c_double),
                ("cheb_half_width", C.c_double), ("ms_total", C.c_double),
                ("launches", C.c_int64 * K_NCLASS), ("ms", C.c_double * K_NCLASS),
                ("bytes", C.c_double * K_NCLASS)]


_lib = None


def load(path: str | None = None):
    """Load libsstep.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is missing: run __graft_entry__.build() first")
    # device memory and streams come from torch: its HIP runtime must be the
    # one the library binds to, so it is loaded first (the library loaded
    # first would pull in a second runtime that does not know torch's memory)
    import torch  # noqa: F401
    lib = C.CDLL(p)
    vp, dp, i32, i64 = C.c_void_p, C.c_double, C.c_int, C.c_int64
    sp, op_, ip = C.POINTER(StencilC), C.POINTER(OptionsC), C.POINTER(InfoC)
    lib.sstep_default_options.argtypes = [op_]
    lib.sstep_default_options.restype = None
    lib.sstep_status_string.argtypes = [i32]
    lib.sstep_status_string.restype = C.c_char_p
    lib.sstep_workspace_bytes.argtypes = [sp, i32, i32, i32, i32]
    lib.sstep_workspace_bytes.restype = C.c_size_t
    lib.sstep_gmres_solve.argtypes = [sp, vp, vp, i32, i32, dp, op_, ip]
    lib.sstep_gmres_solve.restype = i32
    lib.sstep_gmres_solve_noalloc.argtypes = [sp, vp, vp, i32, i32, dp, op_, ip]
    lib.sstep_gmres_solve_noalloc.restype = i32
    lib.sstep_omin_solve.argtypes = [sp, vp, vp, i32, i32, dp, op_, ip]
    lib.sstep_omin_solve.restype = i32
    lib.sstep_stencil_apply.argtypes = [sp, vp, vp, vp]
    lib.sstep_stencil_apply.restype = i32
    lib.sstep_kernel_mpk.argtypes = [sp, vp, i64, i32, i32, dp, dp, dp, dp, vp]
    lib.sstep_kernel_mpk.restype = i32
    lib.sstep_kernel_gram.argtypes = [vp, i64, i32, vp, i64, i32, i64, vp, vp]
    lib.sstep_kernel_gram.restype = i32
    lib.sstep_kernel_update.argtypes = [vp, i64, i32, vp, i64, i32, vp, i64, vp]
    lib.sstep_kernel_update.restype = i32
    lib.sstep_batch_workspace_bytes.argtypes = [i32, sp, i32, i32, op_]
    lib.sstep_batch_workspace_bytes.restype = C.c_size_t
    lib.sstep_batch_plan_create.argtypes = [C.POINTER(C.c_void_p), i32, sp, C.POINTER(vp),
                                            C.POINTER(vp), i32, i32, dp, op_]
    lib.sstep_batch_plan_create.restype = i32
    lib.sstep_batch_plan_execute.argtypes = [vp, ip]
    lib.sstep_batch_plan_execute.restype = i32
    lib.sstep_batch_plan_destroy.argtypes = [vp]
    lib.sstep_batch_plan_destroy.restype = None
    lib.sstep_gmres_solve_batched.argtypes = [i32, sp, C.POINTER(vp), C.POINTER(vp), i32, i32,
                                              dp, op_, ip]
    lib.sstep_gmres_solve_batched.restype = i32
    lib.sstep_cnn_param_count.argtypes = []
    lib.sstep_cnn_param_count.restype = C.c_size_t
    lib.sstep_cnn_workspace_bytes.argtypes = [i32, i32, i32, i32]
    lib.sstep_cnn_workspace_bytes.restype = C.c_size_t
    lib.sstep_cnn_forward.argtypes = [vp, dp, i32, i32, i32, vp, vp, vp, vp, op_]
    lib.sstep_cnn_forward.restype = i32
    lib.sstep_cnn_gradient.argtypes = [vp, dp, i32, i32, i32, vp, vp, vp, vp,
                                       C.POINTER(C.c_double), op_]
    lib.sstep_cnn_gradient.restype = i32
    lib.sstep_cnn_adam.argtypes = [vp, vp, vp, vp, i32, C.c_float, op_]
    lib.sstep_cnn_adam.restype = i32
    lib.sstep_cnn_train_step.argtypes = [vp, vp, vp, i32, C.c_float, dp, i32, i32, i32, vp, vp,
                                         vp, C.POINTER(C.c_double), op_]
    lib.sstep_cnn_train_step.restype = i32
    lib.sstep_x0_predict.argtypes = [vp, dp, sp, vp, vp, vp, i32, C.POINTER(C.c_int), op_]
    lib.sstep_x0_predict.restype = i32
    lib.sstep_grid_pool.argtypes = [vp, vp, i32, i32, i32, i32, vp]
    lib.sstep_grid_pool.restype = i32
    lib.sstep_x0_coarse_workspace_bytes.argtypes = [i32, i32, i32]
    lib.sstep_x0_coarse_workspace_bytes.restype = C.c_size_t
    lib.sstep_x0_predict_coarse.argtypes = [vp, dp, i32, i32, sp, vp, vp, vp, i32,
                                            C.POINTER(C.c_int), op_]
    lib.sstep_x0_predict_coarse.restype = i32
    lib.sstep_precond_workspace_bytes.argtypes = [sp, i32]
    lib.sstep_precond_workspace_bytes.restype = C.c_size_t
    lib.sstep_ilu0_factor.argtypes = [sp, vp, vp]
    lib.sstep_ilu0_factor.restype = i32
    lib.sstep_ilu0_solve.argtypes = [sp, vp, vp, vp, vp]
    lib.sstep_ilu0_solve.restype = i32
    lib.sstep_ilu0_mul.argtypes = [sp, vp, vp, vp, vp]
    lib.sstep_ilu0_mul.restype = i32
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return load().sstep_status_string(int(st)).decode()


class SstepError(RuntimeError):
    pass


def _check(st: int, what: str):
    if st < 0:
        raise SstepError(f"{what}: {status_string(st)} ({st})")
    return st


@dataclass
class Stencil:
    """Stencil operator descriptor (include/sstep.h sstep_stencil).  ``coef``,
    if given, is a CUDA float64 tensor [7, N] that must outlive the calls."""
    ndim: int
    nx: int
    ny: int
    nz: int = 1
    c: tuple = (0.0,) * 7
    coef: object = None

    @classmethod
    def from_problem(cls, prob, coef_device=None):
        return cls(prob.ndim, prob.nx, prob.ny, prob.nz, tuple(float(v) for v in prob.c),
                   coef_device)

    @property
    def N(self) -> int:
        return self.nx * self.ny * (self.nz if self.ndim == 3 else 1)

    def c_struct(self) -> StencilC:
        s = StencilC()
        s.ndim, s.nx, s.ny, s.nz = self.ndim, self.nx, self.ny, self.nz if self.ndim == 3 else 1
        for q in range(7):
            s.c[q] = float(self.c[q])
        s.coef = _ptr(self.coef) if self.coef is not None else None
        return s


@dataclass
class Info:
    status: int
    iters: int
    cycles: int
    matvecs: int
    rel_resid: float
    rel_resid_est: float
    sigma: float
    cheb_centre: float
    cheb_half_width: float
    ms_total: float
    launches: dict
    ms: dict
    bytes: dict

    @classmethod
    def from_c(cls, i: InfoC):
        return cls(i.status, i.iters, i.cycles, i.matvecs, i.rel_resid, i.rel_resid_est, i.sigma,
                   i.cheb_centre, i.cheb_half_width, i.ms_total,
                   {k: int(i.launches[n]) for n, k in enumerate(KERNEL_CLASSES)},
                   {k: float(i.ms[n]) for n, k in enumerate(KERNEL_CLASSES)},
                   {k: float(i.bytes[n]) for n, k in enumerate(KERNEL_CLASSES)})


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"tensor lives on {t.device}, the current device is "
                         f"cuda:{torch.cuda.current_device()}")
    if t.dim() > 0 and t.stride(-1) != 1:
        raise ValueError("tensor rows must be contiguous")
    return t.data_ptr()


def _f64(t, n, name):
    """Device address of a dense float64 array of at least n elements (the C
    side reads and writes n elements from it)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.numel() < n:
        raise ValueError(f"{name} must be a float64 tensor with >= {n} elements")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _ptr(t)


def _rows(t, nrows, n, name):
    """Device address of nrows float64 rows of n elements, rows t.stride(0)
    apart (a block of columns of the tall-skinny matrices)."""
    import torch
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.dim() != 2
            or t.shape[0] < nrows or t.shape[1] < n or t.stride(1) != 1
            or (nrows > 1 and t.stride(0) < n)):
        raise ValueError(f"{name} must be a float64 (>= {nrows}, >= {n}) tensor with unit "
                         f"column stride and row stride >= {n}")
    return _ptr(t)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def options(max_iters=0, precision=FP64, basis=MONOMIAL, profile=False, sigma=0.0, inner_tol=0.0,
            workspace=None, stream=None, batch_threads=0, batch_wgs_per_cu=0,
            batch_graph=False, batch_team=0, precond=PRECOND_NONE,
            orth=ORTH_CHOL, graph=False, batch_gram_cols=0) -> OptionsC:
    o = OptionsC()
    load().sstep_default_options(C.byref(o))
    o.max_iters = int(max_iters)
    o.precision = int(precision)
    o.basis = int(basis)
    o.profile = 1 if profile else 0
    o.sigma = float(sigma)
    o.inner_tol = float(inner_tol)
    if workspace is not None:
        o.workspace = _ptr(workspace)
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.stream = _stream(stream)
    o.batch_threads = int(batch_threads)
    o.batch_wgs_per_cu = int(batch_wgs_per_cu)
    o.batch_graph = 1 if batch_graph else 0
    o.batch_team = int(batch_team)
    o.precond = int(precond)
    o.orth = int(orth)
    o.graph = 1 if graph else 0
    o.batch_gram_cols = int(batch_gram_cols)
    return o


def workspace_bytes(A: Stencil, method: int, s: int, k_or_m: int, precision: int = FP64) -> int:
    sc = A.c_struct()
    return int(load().sstep_workspace_bytes(C.byref(sc), method, s, k_or_m, precision))


def allocate_workspace(A: Stencil, method: int, s: int, k_or_m: int, precision: int = FP64,
                       device="cuda", precond: int = PRECOND_NONE):
    """A caller-owned workspace tensor (uint8) large enough for the solver
    (and for its preconditioner, if precond is set)."""
    import torch
    nb = workspace_bytes(A, method, s, k_or_m, precision)
    if nb == 0:
        raise SstepError("invalid arguments for workspace sizing")
    if precond != PRECOND_NONE:
        pb = precond_workspace_bytes(A, precond)
        if pb == 0:
            raise SstepError("preconditioner not supported for this operator")
        nb += pb
    return torch.empty(nb + 256, dtype=torch.uint8, device=device)[: nb]


def gmres_solve(A: Stencil, f, x, s: int, m: int, tol: float, **kw) -> Info:
    """s-step GMRES(m) (Sec. 4, Alg. 4.2); x (in: x0, out: solution) updated in place."""
    sc = A.c_struct()
    info = InfoC()
    fp, xp = _f64(f, A.N, "f"), _f64(x, A.N, "x")
    o = options(**kw)
    load().sstep_gmres_solve(C.byref(sc), fp, xp, s, m, tol,
                             C.byref(o), C.byref(info))
    return Info.from_c(info)


NOALLOC_MAX_WORKSPACE = 134217728  # bytes, SSTEP_NOALLOC_MAX_WORKSPACE


def gmres_solve_noalloc(A: Stencil, f, x, s: int, m: int, tol: float, **kw) -> Info:
    """sstep_gmres_solve on the library's static per-GPU workspace (no
    allocation); x updated in place."""
    sc = A.c_struct()
    info = InfoC()
    fp, xp = _f64(f, A.N, "f"), _f64(x, A.N, "x")
    o = options(**kw)
    load().sstep_gmres_solve_noalloc(C.byref(sc), fp, xp, s, m, tol,
                                     C.byref(o), C.byref(info))
    return Info.from_c(info)


def omin_solve(A: Stencil, f, x, s: int, k: int, tol: float, **kw) -> Info:
    """s-step Orthomin(k) (Sec. 3, Alg. 3.1); x updated in place."""
    sc = A.c_struct()
    info = InfoC()
    fp, xp = _f64(f, A.N, "f"), _f64(x, A.N, "x")
    o = options(**kw)
    load().sstep_omin_solve(C.byref(sc), fp, xp, s, k, tol,
                            C.byref(o), C.byref(info))
    return Info.from_c(info)


def stencil_apply(A: Stencil, x, y, stream=None) -> None:
    """y = A x."""
    sc = A.c_struct()
    _check(load().sstep_stencil_apply(C.byref(sc), _f64(x, A.N, "x"), _f64(y, A.N, "y"),
                                      _stream(stream)), "stencil_apply")


def kernel_mpk(A: Stencil, Y, s: int, basis=MONOMIAL, in_scale=1.0, sigma=1.0, cheb_c=0.0,
               cheb_d=1.0, stream=None) -> None:
    """Matrix powers of Y[0] into Y[1..s]; Y is a (s+1, ld) float64 tensor."""
    sc = A.c_struct()
    if Y.dim() != 2 or Y.shape[0] < s + 1:
        raise ValueError("Y must be (s+1, ld)")
    _check(load().sstep_kernel_mpk(C.byref(sc), _rows(Y, s + 1, A.N, "Y"), Y.stride(0), s, basis,
                                   in_scale, sigma, cheb_c, cheb_d, _stream(stream)), "kernel_mpk")


def kernel_gram(X, Z, G=None, stream=None):
    """G = X^T Z (X: (ncx, ld), Z: (ncz, ld) float64; rows are columns of the
    tall-skinny blocks).  Returns G (ncx, ncz) on the device."""
    import torch
    ncx, ncz, N = X.shape[0], Z.shape[0], X.shape[1]
    if G is None:
        G = torch.empty((ncx, ncz), dtype=torch.float64, device=X.device)
    _check(load().sstep_kernel_gram(_rows(X, ncx, N, "X"), X.stride(0), ncx, _rows(Z, ncz, N, "Z"),
                                    Z.stride(0), ncz, N, _f64(G, ncx * ncz, "G"), _stream(stream)),
           "kernel_gram")
    return G


def kernel_update(X, Y, M, stream=None) -> None:
    """Y[l] += sum_c X[c] M[c, l] (X: (ncx, ld), Y: (ncy, ld), M: (ncx, ncy) float64, device)."""
    ncx, ncy, N = X.shape[0], Y.shape[0], Y.shape[1]
    xp = _rows(X, ncx, N, "X") if ncx else None
    mp = _f64(M, ncx * ncy, "M") if ncx else None
    _check(load().sstep_kernel_update(xp, X.stride(0) if ncx else N, ncx, _rows(Y, ncy, N, "Y"),
                                      Y.stride(0), ncy, mp, N, _stream(stream)), "kernel_update")


class BatchPlan:
    """Batched s-step GMRES(m) over many independent systems in one persistent
    launch (captured in a hipGraph when graph=True).  stencils: list of
    Stencil; fs, xs: lists of CUDA float64 tensors (x is overwritten with the
    solution at every execute(); reset it to the initial guess first)."""

    def __init__(self, stencils, fs, xs, s, m, tol, threads=0, wgs_per_cu=0, graph=True,
                 max_iters=0, workspace=None, team=0, gram_cols=0):
        n = len(stencils)
        if not (len(fs) == len(xs) == n):
            raise ValueError("stencils, fs and xs must have equal lengths")
        self.n = n
        self._A = (StencilC * n)(*[a.c_struct() for a in stencils])
        self._f = (C.c_void_p * n)(*[_f64(f, a.N, "f") for f, a in zip(fs, stencils)])
        self._x = (C.c_void_p * n)(*[_f64(x, a.N, "x") for x, a in zip(xs, stencils)])
        self._keep = (list(fs), list(xs), workspace)
        o = options(max_iters=max_iters, workspace=workspace, batch_threads=threads,
                    batch_wgs_per_cu=wgs_per_cu, batch_graph=graph, batch_team=team,
                    batch_gram_cols=gram_cols)
        self._plan = C.c_void_p()
        _check(load().sstep_batch_plan_create(C.byref(self._plan), n, self._A, self._f, self._x,
                                              s, m, tol, C.byref(o)), "batch_plan_create")

    def execute(self):
        infos = (InfoC * self.n)()
        st = load().sstep_batch_plan_execute(self._plan, infos)
        if st in (ERR_ARG, ERR_HIP, ERR_NOMEM):   # whole-batch failures
            _check(st, "batch_plan_execute")
        # per-system outcomes (including per-system errors) are in the infos
        return st, [Info.from_c(infos[i]) for i in range(self.n)]

    def close(self):
        if self._plan:
            load().sstep_batch_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(stencils, s, m, wgs_per_cu=0, team=0) -> int:
    n = len(stencils)
    arr = (StencilC * n)(*[a.c_struct() for a in stencils])
    opt = OptionsC()
    load().sstep_default_options(C.byref(opt))
    opt.batch_wgs_per_cu = int(wgs_per_cu)
    opt.batch_team = int(team)
    return int(load().sstep_batch_workspace_bytes(n, arr, s, m, C.byref(opt)))


# ---------------------------------------------------------------------------
# learned initial guess (include/sstep.h, sstep_cnn_* and sstep_x0_predict)
# ---------------------------------------------------------------------------

def _f32(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.numel() < n:
        raise ValueError(f"{name} must be a float32 tensor with >= {n} elements")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _ptr(t)


def _bhw(t):
    """(batch, ny, nx) of a [B][ny][nx] or [ny][nx] tensor."""
    if t.dim() == 2:
        return 1, t.shape[0], t.shape[1]
    if t.dim() == 3:
        return t.shape[0], t.shape[1], t.shape[2]
    raise ValueError("expected a [B][ny][nx] or [ny][nx] tensor")


def cnn_param_count() -> int:
    return int(load().sstep_cnn_param_count())


def cnn_workspace_bytes(batch: int, nx: int, ny: int, training: bool) -> int:
    return int(load().sstep_cnn_workspace_bytes(batch, nx, ny, 1 if training else 0))


def cnn_forward(params, out_scale, logk, f, out=None, x0=None, workspace=None, stream=None):
    """Network output (float32, optional) and scaled guess x0 (float64, optional)."""
    B, ny, nx = _bhw(logk)
    n = B * ny * nx
    o = options(workspace=workspace, stream=stream)
    _check(load().sstep_cnn_forward(
        _f32(params, cnn_param_count(), "params"), float(out_scale), B, nx, ny,
        _f32(logk, n, "logk"), _f64(f, n, "f"), _f32(out, n, "out") if out is not None else None,
        _f64(x0, n, "x0") if x0 is not None else None, C.byref(o)), "cnn_forward")


def cnn_gradient(params, out_scale, logk, f, x, grad, workspace=None, stream=None) -> float:
    """Loss and its parameter gradient (into grad, float32) for targets x."""
    B, ny, nx = _bhw(logk)
    n = B * ny * nx
    loss = C.c_double(0.0)
    o = options(workspace=workspace, stream=stream)
    _check(load().sstep_cnn_gradient(
        _f32(params, cnn_param_count(), "params"), float(out_scale), B, nx, ny,
        _f32(logk, n, "logk"), _f64(f, n, "f"), _f64(x, n, "x"),
        _f32(grad, cnn_param_count(), "grad"), C.byref(loss), C.byref(o)), "cnn_gradient")
    return loss.value


def cnn_adam(params, m, v, grad, step: int, lr: float, stream=None) -> None:
    P = cnn_param_count()
    o = options(stream=stream)
    _check(load().sstep_cnn_adam(_f32(params, P, "params"), _f32(m, P, "m"), _f32(v, P, "v"),
                                 _f32(grad, P, "grad"), int(step), float(lr), C.byref(o)),
           "cnn_adam")


def cnn_train_step(params, m, v, step: int, lr: float, out_scale, logk, f, x, workspace=None,
                   stream=None) -> float:
    """One Adam step on a batch; returns the batch loss before the step."""
    B, ny, nx = _bhw(logk)
    n = B * ny * nx
    P = cnn_param_count()
    loss = C.c_double(0.0)
    o = options(workspace=workspace, stream=stream)
    _check(load().sstep_cnn_train_step(
        _f32(params, P, "params"), _f32(m, P, "m"), _f32(v, P, "v"), int(step), float(lr),
        float(out_scale), B, nx, ny, _f32(logk, n, "logk"), _f64(f, n, "f"), _f64(x, n, "x"),
        C.byref(loss), C.byref(o)), "cnn_train_step")
    return loss.value


def x0_predict(params, out_scale, A: Stencil, logk, f, x0, use_fallback=True, workspace=None,
               stream=None) -> bool:
    """Fill x0 with the network's guess for A x = f; returns True when the
    fallback rule replaced it by zero."""
    sc = A.c_struct()
    used = C.c_int(0)
    o = options(workspace=workspace, stream=stream)
    _check(load().sstep_x0_predict(
        _f32(params, cnn_param_count(), "params"), float(out_scale), C.byref(sc),
        _f32(logk, A.N, "logk"), _f64(f, A.N, "f"), _f64(x0, A.N, "x0"),
        1 if use_fallback else 0, C.byref(used), C.byref(o)), "x0_predict")
    return bool(used.value)


def grid_pool(x, factor: int, out=None, stream=None):
    """Block averages over factor x factor cells of x (float64 [B][ny][nx] or
    [ny][nx]) -> [B][ny/factor][nx/factor] (or 2-D), on the device."""
    import torch
    B, ny, nx = _bhw(x)
    shape = (B, ny // factor, nx // factor) if x.dim() == 3 else (ny // factor, nx // factor)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=x.device)
    nc = B * (ny // factor) * (nx // factor)
    _check(load().sstep_grid_pool(_f64(x, B * ny * nx, "x"), _f64(out, nc, "out"), B, nx, ny,
                                  int(factor), _stream(stream)), "grid_pool")
    return out


def x0_coarse_workspace_bytes(nx: int, ny: int, factor: int) -> int:
    return int(load().sstep_x0_coarse_workspace_bytes(int(nx), int(ny), int(factor)))


def x0_predict_coarse(params, out_scale, factor: int, sweeps: int, A: Stencil, logk, f, x0,
                      use_fallback=True, workspace=None, stream=None) -> bool:
    """Fill x0 with the coarse-grid network guess (block-averaged inputs,
    bilinear interpolation, damped Jacobi sweeps) for A x = f; returns True
    when the fallback rule replaced it by zero."""
    sc = A.c_struct()
    used = C.c_int(0)
    o = options(workspace=workspace, stream=stream)
    _check(load().sstep_x0_predict_coarse(
        _f32(params, cnn_param_count(), "params"), float(out_scale), int(factor), int(sweeps),
        C.byref(sc), _f32(logk, A.N, "logk"), _f64(f, A.N, "f"), _f64(x0, A.N, "x0"),
        1 if use_fallback else 0, C.byref(used), C.byref(o)), "x0_predict_coarse")
    return bool(used.value)


# ---------------------------------------------------------------------------
# ILU(0) right preconditioning (Sec. 5)
# ---------------------------------------------------------------------------

def precond_workspace_bytes(A: Stencil, precond: int = PRECOND_ILU0) -> int:
    sc = A.c_struct()
    return int(load().sstep_precond_workspace_bytes(C.byref(sc), int(precond)))


def ilu0_factor(A: Stencil, d=None, stream=None):
    """Pivots of the ILU(0) factors of A: a float64 CUDA tensor [2N] (pivots,
    then their reciprocals).  Raises on a zero pivot."""
    import torch
    if d is None:
        d = torch.empty(2 * A.N, dtype=torch.float64, device="cuda")
    sc = A.c_struct()
    _check(load().sstep_ilu0_factor(C.byref(sc), _f64(d, 2 * A.N, "d"), _stream(stream)),
           "ilu0_factor")
    return d


def ilu0_solve(A: Stencil, d, r, z=None, stream=None):
    """z = M^{-1} r with M = L U the ILU(0) factors."""
    import torch
    if z is None:
        z = torch.empty(A.N, dtype=torch.float64, device="cuda")
    sc = A.c_struct()
    _check(load().sstep_ilu0_solve(C.byref(sc), _f64(d, 2 * A.N, "d"), _f64(r, A.N, "r"),
                                   _f64(z, A.N, "z"), _stream(stream)), "ilu0_solve")
    return z


def ilu0_mul(A: Stencil, d, x, u=None, stream=None):
    """u = M x with M = L U the ILU(0) factors."""
    import torch
    if u is None:
        u = torch.empty(A.N, dtype=torch.float64, device="cuda")
    sc = A.c_struct()
    _check(load().sstep_ilu0_mul(C.byref(sc), _f64(d, 2 * A.N, "d"), _f64(x, A.N, "x"),
                                 _f64(u, A.N, "u"), _stream(stream)), "ilu0_mul")
    return u

