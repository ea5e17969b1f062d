"""Plain FP64 CPU oracle for s-step Orthomin(k) and s-step GMRES(m).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  It never
imports the GPU library and the GPU library never imports it.

The arithmetic lives in ``sstep_oracle.c`` (plain single-threaded C, FP64,
sums in index order); this module only marshals numpy arrays through ctypes.
Each wrapper names the section / algorithm of Chronopoulos & Kim (arXiv
2001.04886) that the C routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sstep_oracle.c")
_LIB = os.environ.get("SSTEP_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

MONOMIAL = 0
CHEBYSHEV = 1
NEWTON = 2

OK, NOT_CONVERGED, ERR_ARG, ERR_BREAKDOWN, ERR_NONFINITE, ERR_NOMEM = 0, 1, -1, -2, -3, -5


_FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-fPIC", "-shared"]
LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction).
    Its OpenMP pragmas are ignored: one thread, sums in index order."""
    cmd = ["gcc", *_FLAGS, "-Wno-unknown-pragmas", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_omp() -> str:
    """The same source compiled with -fopenmp (timing build for the CPU
    baseline): N-length loops on all host cores, inner products summed in
    fixed blocks.  Load it in a separate process (SSTEP_ORACLE_LIB)."""
    cmd = ["gcc", *_FLAGS, "-fopenmp", "-o", LIB_OMP + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_OMP + ".tmp", LIB_OMP)
    return LIB_OMP


class _Stencil(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("c", C.c_double * 7), ("coef", C.POINTER(C.c_double)),
                ("ilu", C.POINTER(C.c_double))]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("cycles", C.c_int),
                ("matvecs", C.c_int), ("rel_resid", C.c_double),
                ("rel_resid_est", C.c_double), ("nhist", C.c_int)]


class _CycleDump(C.Structure):
    _fields_ = [("V", C.POINTER(C.c_double)), ("G", C.POINTER(C.c_double)),
                ("D", C.POINTER(C.c_double)), ("ncols", C.c_int), ("blocks", C.c_int)]


class _OminDump(C.Structure):
    _fields_ = [("P", C.POINTER(C.c_double)), ("AP", C.POINTER(C.c_double)),
                ("r", C.POINTER(C.c_double)), ("nblocks", C.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if "SSTEP_ORACLE_LIB" not in os.environ and (
            not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build()
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    sp = C.POINTER(_Stencil)
    rp = C.POINTER(_Result)
    lib.orc_size.restype = C.c_longlong
    lib.orc_size.argtypes = [sp]
    lib.orc_apply.restype = None
    lib.orc_apply.argtypes = [sp, dp, dp]
    lib.orc_sigma.restype = C.c_double
    lib.orc_sigma.argtypes = [sp]
    lib.orc_cheb_interval.restype = None
    lib.orc_cheb_interval.argtypes = [sp, dp, dp]
    lib.orc_mpk.restype = None
    lib.orc_mpk.argtypes = [sp, dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, dp]
    lib.orc_gmres.restype = C.c_int
    lib.orc_gmres.argtypes = [sp, dp, dp, C.c_int, C.c_double, C.c_int, rp, dp, C.c_int, dp, dp]
    lib.orc_omin.restype = C.c_int
    lib.orc_omin.argtypes = [sp, dp, dp, C.c_int, C.c_double, C.c_int, rp, dp, C.c_int]
    lib.orc_somin.restype = C.c_int
    lib.orc_somin.argtypes = [sp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, rp,
                              dp, C.c_int, C.POINTER(_OminDump)]
    lib.orc_newton_shifts.restype = None
    lib.orc_newton_shifts.argtypes = [C.c_int, C.c_double, C.c_double, dp]
    lib.orc_somin_ex.restype = C.c_int
    lib.orc_somin_ex.argtypes = [sp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                 C.c_int, rp, dp, C.c_int, C.POINTER(_OminDump)]
    lib.orc_sgmres.restype = C.c_int
    lib.orc_sgmres.argtypes = [sp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, rp,
                               dp, C.c_int, C.POINTER(_CycleDump)]
    lib.orc_ilu0_factor.restype = C.c_int
    lib.orc_ilu0_factor.argtypes = [sp, dp]
    lib.orc_ilu0_solve.restype = None
    lib.orc_ilu0_solve.argtypes = [sp, dp, dp, dp]
    lib.orc_ilu0_mul.restype = None
    lib.orc_ilu0_mul.argtypes = [sp, dp, dp, dp]
    lib.orc_somin_ilu0.restype = C.c_int
    lib.orc_somin_ilu0.argtypes = [sp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int, rp, dp,
                                   C.c_int]
    lib.orc_sgmres_ilu0.restype = C.c_int
    lib.orc_sgmres_ilu0.argtypes = [sp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int, rp, dp,
                                    C.c_int]
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Result:
    status: int
    iters: int
    cycles: int
    matvecs: int
    rel_resid: float
    rel_resid_est: float
    hist: np.ndarray


class Operator:
    """Stencil operator (same field meaning as the GPU library's descriptor):
    ndim, nx, ny, nz, seven coefficients (centre, -x, +x, -y, +y, -z, +z) or a
    [7][N] per-point coefficient array."""

    def __init__(self, ndim, nx, ny, nz=1, c=None, coef=None):
        self.ndim, self.nx, self.ny, self.nz = int(ndim), int(nx), int(ny), int(nz if ndim == 3 else 1)
        self.c = np.zeros(7) if c is None else np.asarray(c, dtype=np.float64).copy()
        self.coef = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64)
        self._s = _Stencil()
        self._s.ndim, self._s.nx, self._s.ny, self._s.nz = self.ndim, self.nx, self.ny, self.nz
        for q in range(7):
            self._s.c[q] = float(self.c[q])
        self._s.coef = _dp(self.coef) if self.coef is not None else None

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def ref(self):
        return C.byref(self._s)


def apply(A: Operator, x: np.ndarray) -> np.ndarray:
    """y = A x (Sec. 1 / Sec. 5 finite-difference operator)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.N)
    lib.orc_apply(A.ref, _dp(x), _dp(y))
    return y


def sigma(A: Operator) -> float:
    return _load().orc_sigma(A.ref)


def cheb_interval(A: Operator):
    c, d = C.c_double(), C.c_double()
    _load().orc_cheb_interval(A.ref, C.byref(c), C.byref(d))
    return c.value, d.value


def newton_shifts(s: int, centre: float, half_width: float) -> np.ndarray:
    """Leja-ordered Chebyshev points of the interval: the Newton-basis shifts."""
    th = np.empty(s)
    _load().orc_newton_shifts(s, centre, half_width, _dp(th))
    return th


def mpk(A: Operator, y0: np.ndarray, s: int, basis: int = MONOMIAL, params=None) -> np.ndarray:
    """Matrix powers [y_0 .. y_s] of y0 (Sec. 3-4), shape (s+1, N).  params =
    (sigma, centre, half_width) overrides the scaling and interval derived
    from A (used when A is a window cut out of a larger grid)."""
    lib = _load()
    if params is not None:
        sg, cc, cd = (float(v) for v in params)
    else:
        sg = sigma(A)
        cc, cd = cheb_interval(A) if basis != MONOMIAL else (0.0, 1.0)
    Y = np.empty((s + 1, A.N))
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    lib.orc_mpk(A.ref, _dp(y0), s, basis, sg, cc, cd, _dp(Y))
    return Y


def _res(r: _Result, hist):
    return Result(r.status, r.iters, r.cycles, r.matvecs, r.rel_resid, r.rel_resid_est,
                  hist[: r.nhist].copy())


def gmres(A, f, x0, M, tol, max_steps=0, dump=False, hist_cap=100000):
    """Restarted GMRES(M) (Sec. 2, Alg. 2.2).  Returns (x, Result[, Q, H])."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = _Result()
    hist = np.zeros(hist_cap)
    Q = np.zeros((M + 1, A.N)) if dump else None
    H = np.zeros((M, M + 1)) if dump else None
    lib.orc_gmres(A.ref, _dp(f), _dp(x), M, tol, max_steps, C.byref(res), _dp(hist), hist_cap,
                  _dp(Q), _dp(H))
    out = (x, _res(res, hist))
    if dump:
        out = out + (Q, H.T.copy())  # H column-major (ld M+1) -> (M+1, M)
    return out


def omin(A, f, x0, k, tol, max_iters=0, hist_cap=100000):
    """Omin(k) / GCR (Sec. 2, Alg. 2.1).  Returns (x, Result)."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = _Result()
    hist = np.zeros(hist_cap)
    lib.orc_omin(A.ref, _dp(f), _dp(x), k, tol, max_iters, C.byref(res), _dp(hist), hist_cap)
    return x, _res(res, hist)


def somin(A, f, x0, s, k, tol, max_iters=0, basis=MONOMIAL, dump=False, hist_cap=100000,
          mgs=False):
    """s-step Orthomin(k) (Sec. 3, Alg. 3.1).  Returns (x, Result[, P, AP, r]).
    mgs: the larger-s variant of Sec. 3 (A^T A-orthogonal direction blocks by
    modified Gram-Schmidt, diagonal Scalar1/Scalar2)."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = _Result()
    hist = np.zeros(hist_cap)
    d = None
    if dump:
        P = np.zeros((k * s, A.N))
        AP = np.zeros((k * s, A.N))
        r = np.zeros(A.N)
        d = _OminDump(_dp(P), _dp(AP), _dp(r), 0)
    lib.orc_somin_ex(A.ref, _dp(f), _dp(x), s, k, tol, max_iters, basis, 1 if mgs else 0,
                     C.byref(res), _dp(hist), hist_cap, C.byref(d) if d is not None else None)
    out = (x, _res(res, hist))
    if dump:
        nb = d.nblocks
        out = out + (P[: nb * s].copy(), AP[: nb * s].copy(), r)
    return out


def sgmres(A, f, x0, s, m, tol, max_blocks=0, basis=MONOMIAL, dump=False, hist_cap=100000):
    """Restarted s-step GMRES(m) (Sec. 4, Alg. 4.1-4.2).  Returns (x, Result[, dump])
    where dump = dict(V=(ncols+1, N) basis U_k, G=(ncols+1, ncols) Hessenberg,
    D=(ncols+1, ncols+1) U^T U, ncols, blocks) for the first cycle."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = _Result()
    hist = np.zeros(hist_cap)
    K = m * s
    d = None
    if dump:
        V = np.zeros((K + 1, A.N))
        G = np.zeros((K, K + 1))
        D = np.zeros((K + 1, K + 1))
        d = _CycleDump(_dp(V), _dp(G), _dp(D), 0, 0)
    lib.orc_sgmres(A.ref, _dp(f), _dp(x), s, m, tol, max_blocks, basis, C.byref(res), _dp(hist),
                   hist_cap, C.byref(d) if d is not None else None)
    out = (x, _res(res, hist))
    if dump:
        nc = d.ncols
        out = out + (dict(V=V[: nc + 1].copy(), G=G.T[: nc + 1, :nc].copy(),
                          D=D.T[: nc + 1, : nc + 1].copy(), ncols=nc, blocks=d.blocks),)
    return out


# ---------------------------------------------------------------------------
# ILU(0) right preconditioning (Sec. 5)
# ---------------------------------------------------------------------------

def ilu0_factor(A: Operator) -> np.ndarray:
    """Incomplete LU with A's five-point pattern (Sec. 5), shape (5, N): rows
    are the slots south, west (unit lower factor L), centre, east, north (U).
    Raises on a zero pivot or a 3-D operator."""
    LU = np.empty((5, A.N))
    st = _load().orc_ilu0_factor(A.ref, _dp(LU))
    if st != OK:
        raise ValueError(f"ILU(0) factorisation failed (status {st})")
    return LU


def ilu0_solve(A: Operator, LU: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = (L U)^{-1} r."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(A.N)
    _load().orc_ilu0_solve(A.ref, _dp(np.ascontiguousarray(LU)), _dp(r), _dp(z))
    return z


def ilu0_mul(A: Operator, LU: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = L U x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.N)
    _load().orc_ilu0_mul(A.ref, _dp(np.ascontiguousarray(LU)), _dp(x), _dp(y))
    return y


def apply_precond(A: Operator, LU: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A (L U)^{-1} x, the right-preconditioned operator of Sec. 5."""
    LU = np.ascontiguousarray(LU)
    s = _Stencil()
    C.pointer(s)[0] = A._s
    s.ilu = _dp(LU)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.N)
    _load().orc_apply(C.byref(s), _dp(x), _dp(y))
    return y


def somin_ilu0(A, f, x0, s, k, tol, max_iters=0, hist_cap=100000):
    """s-step Orthomin(k) on the ILU(0) right-preconditioned system (Sec. 3
    and Sec. 5).  Returns (x, Result); residuals are true residuals."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = _Result()
    hist = np.zeros(hist_cap)
    lib.orc_somin_ilu0(A.ref, _dp(f), _dp(x), s, k, tol, max_iters, C.byref(res), _dp(hist),
                       hist_cap)
    return x, _res(res, hist)


def sgmres_ilu0(A, f, x0, s, m, tol, max_blocks=0, hist_cap=100000):
    """s-step GMRES(m) on the ILU(0) right-preconditioned system (Sec. 4 and
    Sec. 5).  Returns (x, Result); residuals are true residuals."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = _Result()
    hist = np.zeros(hist_cap)
    lib.orc_sgmres_ilu0(A.ref, _dp(f), _dp(x), s, m, tol, max_blocks, C.byref(res), _dp(hist),
                        hist_cap)
    return x, _res(res, hist)
