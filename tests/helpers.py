"""Test-side helpers: dense reference constructions built from library
routines (numpy), used to pin the oracle to definitions rather than to itself."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2001_04886_amd import problems as PB


def operator(prob: PB.Problem) -> O.Operator:
    return O.Operator(prob.ndim, prob.nx, prob.ny, prob.nz, c=prob.c, coef=prob.coef)


def dense(A: O.Operator) -> np.ndarray:
    """Dense matrix of the oracle operator, column j = A e_j."""
    N = A.N
    M = np.zeros((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[:] = 0.0
        e[j] = 1.0
        M[:, j] = O.apply(A, e)
    return M


def krylov_min_residual(Ad: np.ndarray, r0: np.ndarray, dim: int) -> np.ndarray:
    """z = argmin_{z in K_dim(A, r0)} ||r0 - A z||_2 (the defining property of
    the GMRES / GCR iterate, Sec. 2 eq. (3)).  The Krylov space is spanned by
    an orthonormal basis obtained with two passes of Gram-Schmidt per vector
    (numerically robust), and the small problem is solved by numpy lstsq."""
    n = len(r0)
    Q = np.zeros((n, dim))
    v = r0 / np.linalg.norm(r0)
    for j in range(dim):
        Q[:, j] = v
        w = Ad @ v
        for _ in range(2):
            w = w - Q[:, : j + 1] @ (Q[:, : j + 1].T @ w)
        nw = np.linalg.norm(w)
        if nw < 1e-13 * np.linalg.norm(Ad, 2):
            Q = Q[:, : j + 1]
            break
        v = w / nw
    y, *_ = np.linalg.lstsq(Ad @ Q, r0, rcond=None)
    return Q @ y


def tridiag_eig(b: float, a: float, c: float, n: int, j: int):
    """Closed-form eigenpair j (1..n) of the n x n tridiagonal Toeplitz matrix
    with sub-diagonal b, diagonal a, super-diagonal c (b c > 0):
    lambda = a + 2 sgn(c) sqrt(b c) cos(j pi/(n+1)), v_i = (b/c)^{i/2} sin(i j pi/(n+1))."""
    th = j * np.pi / (n + 1)
    lam = a + 2.0 * np.sign(c) * np.sqrt(b * c) * np.cos(th)
    i = np.arange(1, n + 1)
    v = (b / c) ** (i / 2.0) * np.sin(i * th)
    return lam, v


def stencil_eigpair(prob: PB.Problem, js):
    """Closed-form eigenpair of a constant-coefficient stencil: the operator is
    a Kronecker sum of per-axis tridiagonal Toeplitz matrices (the centre
    coefficient split as -(c_- + c_+) per axis plus the remainder on axis x)."""
    c = prob.c
    ns = [prob.nx, prob.ny] + ([prob.nz] if prob.ndim == 3 else [])
    diag_axes = [-(c[1 + 2 * d] + c[2 + 2 * d]) for d in range(len(ns))]
    rest = c[0] - sum(diag_axes)
    lam = rest
    vec = None
    for d, n in enumerate(ns):
        l, v = tridiag_eig(c[1 + 2 * d], diag_axes[d], c[2 + 2 * d], n, js[d])
        lam += l
        # x fastest: vec[p] with p = i + nx*(j + ny*l)
        vec = v if vec is None else np.kron(v, vec)
    return lam, vec


def window(shape, point, R):
    """The grid of shape (nx, ny, nz) clipped to the box of radius R around
    point (i, j, l): its dims, the flat indices of its points (x fastest) and
    the position of the point inside it.  A stencil value of level <= R at the
    point depends only on points of this window, and the clipped sides keep
    the grid's own Dirichlet boundary."""
    lo = [max(0, v - R) for v in point]
    hi = [min(n - 1, v + R) for n, v in zip(shape, point)]
    ax = [np.arange(a, b + 1, dtype=np.int64) for a, b in zip(lo, hi)]
    nx, ny = shape[0], shape[1]
    flat = (ax[2][:, None, None] * nx * ny + ax[1][None, :, None] * nx + ax[0][None, None, :]).ravel()
    dims = [len(a) for a in ax]
    i, j, l = point
    ctr = (l - lo[2]) * dims[0] * dims[1] + (j - lo[1]) * dims[0] + (i - lo[0])
    return dims, flat, ctr
