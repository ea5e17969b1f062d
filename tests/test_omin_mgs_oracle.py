"""The larger-s variant of s-step Orthomin (Sec. 3, after Alg. 3.1): every
new direction block is made A^T A-orthogonal by modified Gram-Schmidt, so the
Scalar1 and Scalar2 systems become diagonal.  The oracle's variant is pinned
to that statement (W of every stored block diagonal), to A P = AP, to the
minimum-residual property of the first s-step iteration (Sec. 2 eq. (3)),
to sparse LU, to the plain variant's iterates where both are well
conditioned (the two span the same spaces), and to the paper's claim that it
admits a larger s."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_2001_04886_amd import problems as PB
from helpers import dense, krylov_min_residual, operator
from test_paper_problem import sparse_from_coef


def paper(n):
    pr = PB.paper_problem(n)
    return pr, operator(pr), PB.paper_rhs(n), PB.paper_x0(pr.N)


@pytest.mark.parametrize("s,k", [(4, 2), (8, 1), (12, 2)])
def test_blocks_are_ata_orthogonal(s, k):
    pr, A, g, x0 = paper(24)
    _, r, P, AP, _ = O.somin(A, g, x0, s, k, 0.0, max_iters=6, dump=True, mgs=True)
    assert r.iters == 6
    for b in range(AP.shape[0] // s):
        Ab, Pb = AP[b * s:(b + 1) * s], P[b * s:(b + 1) * s]
        W = Ab @ Ab.T
        d = np.sqrt(np.maximum(np.diag(W), 1e-300))
        off = W / np.outer(d, d) - np.diag(np.diag(W) > 0)
        # one pass of MGS leaves cosines of order eps * cond(AR) (no
        # reorthogonalisation): 1e-12 at s <= 8, 1e-10 at s = 12 here
        assert np.max(np.abs(off)) <= (1e-12 if s <= 8 else 1e-9), np.max(np.abs(off))
        # the same combinations were applied to P: A P = AP, up to the
        # rounding the recurrences accumulate (the plain variant drifts to
        # 7e-5 here at s = 12, this one to 4e-9)
        APb = np.stack([O.apply(A, p) for p in Pb])
        bound = 1e-9 if s <= 8 else 1e-7
        assert np.linalg.norm(APb - Ab) <= bound * max(np.linalg.norm(Ab), 1e-300)


@pytest.mark.parametrize("s", [2, 3, 5])
def test_first_iteration_is_the_s_step_minimum_residual(s):
    pr, A, g, x0 = paper(7)
    x, r = O.somin(A, g, x0, s, 2, 0.0, max_iters=1, mgs=True)
    Ad = dense(A)
    r0 = g - Ad @ x0
    xr = x0 + krylov_min_residual(Ad, r0, s)
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("s,k", [(2, 2), (3, 1), (4, 3)])
def test_same_iterates_as_the_plain_variant_when_well_conditioned(s, k):
    pr, A, g, x0 = paper(16)
    xa, ra = O.somin(A, g, x0, s, k, 0.0, max_iters=12)
    xb, rb = O.somin(A, g, x0, s, k, 0.0, max_iters=12, mgs=True)
    assert ra.iters == rb.iters == 12
    assert np.linalg.norm(xa - xb) <= 1e-8 * np.linalg.norm(xa)


@pytest.mark.parametrize("s", [8, 12, 16])
def test_reaches_sparse_lu_solution_at_large_s(s):
    n = 24
    pr, A, g, x0 = paper(n)
    ref = spla.spsolve(sparse_from_coef(n, pr.coef).tocsc(), g)
    x, r = O.somin(A, g, x0, s, 1, 1e-11, max_iters=5000, mgs=True)
    assert r.status == O.OK and r.rel_resid <= 1e-11
    assert np.linalg.norm(x - ref) <= 1e-7 * np.linalg.norm(ref)


def test_larger_s_takes_fewer_iterations_than_the_plain_variant():
    # the paper: with the A^T A-orthogonal blocks a larger s can be chosen
    pr, A, g, x0 = paper(64)
    tol = 1e-6 / np.linalg.norm(g)
    for s in (12, 16):
        _, plain = O.somin(A, g, x0, s, 1, tol, max_iters=20000)
        _, mgs = O.somin(A, g, x0, s, 1, tol, max_iters=20000, mgs=True)
        assert mgs.status == O.OK and mgs.iters < 0.8 * plain.iters, (s, mgs.iters, plain.iters)


def test_dependent_column_is_dropped():
    # a block whose Krylov vectors are dependent (A = identity: A r = r)
    A = O.Operator(2, 5, 4, c=[1.0, 0, 0, 0, 0, 0, 0])
    g = np.linspace(1.0, 2.0, 20)
    x, r = O.somin(A, g, np.zeros(20), 4, 1, 1e-12, max_iters=5, mgs=True)
    assert r.status == O.OK and r.iters == 1
    np.testing.assert_allclose(x, g, rtol=1e-13)


@pytest.mark.parametrize("delta,kept", [(1e-9, [True, False, False, False]),
                                        (1e-3, [True, True, True, False])])
def test_nearly_dependent_columns_are_dropped(delta, kept):
    # A = diag(1 + delta d): consecutive Krylov columns differ by O(delta), so
    # after A^T A-orthogonalisation column q keeps about delta^(2q) of its
    # squared A-norm.  Columns below the drop threshold (1e-14 of the value
    # before orthogonalisation) must be exactly zero in both P and AP, the
    # others kept: delta = 1e-9 leaves only column 0; delta = 1e-3 keeps
    # columns 1 (~1e-6) and 2 (~1e-12) and drops column 3 (~1e-18).
    nx, ny, s = 6, 5, 4
    N = nx * ny
    coef = np.zeros((7, N))
    coef[0] = 1.0 + delta * np.linspace(-1.0, 1.0, N)
    A = O.Operator(2, nx, ny, coef=coef)
    g = np.cos(np.arange(N))
    x, r, P, AP, _ = O.somin(A, g, np.zeros(N), s, 1, 0.0, max_iters=1, dump=True, mgs=True)
    for q in range(s):
        if kept[q]:
            assert np.linalg.norm(AP[q]) > 0.0 and np.linalg.norm(P[q]) > 0.0, q
        else:
            assert not AP[q].any() and not P[q].any(), q
    # the kept directions still satisfy A P = AP
    np.testing.assert_allclose(O.apply(A, P[0]), AP[0], rtol=1e-13)
