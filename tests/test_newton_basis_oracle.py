"""Newton basis with Leja-ordered shifts (the larger-s stabilisation of the
s-step methods, alongside the Chebyshev option): the oracle's shifts are
pinned to the closed-form Chebyshev points and to the Leja rule by brute
force, its matrix powers to the Newton recurrence on the dense matrix, its
s-GMRES to the Krylov minimum-residual property (Sec. 2 eq. (3)) and to the
monomial basis where both are well conditioned, and its behaviour at large s
to fewer blocks than the monomial basis."""
import numpy as np
import pytest

import oracle as O
from paper_2001_04886_amd import problems as PB
from helpers import dense, krylov_min_residual, operator


@pytest.mark.parametrize("s,c,d", [(1, 3.0, 2.0), (4, 2.0, 1.0), (7, -0.5, 3.0), (16, 8.0, 7.5),
                                   (6, 0.0, 1.0)])
def test_shifts_are_leja_ordered_chebyshev_points(s, c, d):
    th = O.newton_shifts(s, c, d)
    pts = c + d * np.cos((2 * np.arange(s) + 1) * np.pi / (2 * s))
    np.testing.assert_allclose(np.sort(th), np.sort(pts), rtol=0, atol=1e-14 * (abs(c) + d))
    assert abs(th[0]) == pytest.approx(np.max(np.abs(pts)), rel=1e-15)
    for n in range(1, s):
        rest = [p for p in pts if np.min(np.abs(p - th[:n])) > 1e-12 * d]
        best = max(np.prod(np.abs(p - th[:n])) for p in rest)
        assert np.prod(np.abs(th[n] - th[:n])) >= best * (1 - 1e-12)


@pytest.mark.parametrize("ndim,n,s", [(2, 9, 5), (3, 5, 8)])
def test_powers_follow_the_newton_recurrence(ndim, n, s):
    pr = PB.convdiff(ndim, n, 30.0)
    A = operator(pr)
    Ad = dense(A)
    c, d = O.cheb_interval(A)
    th = O.newton_shifts(s, c, d)
    y0 = np.sin(np.arange(pr.N) * 0.61)
    Y = O.mpk(A, y0, s, basis=O.NEWTON)
    for j in range(s):
        ref = (Ad @ Y[j] - th[j] * Y[j]) / d
        assert np.linalg.norm(Y[j + 1] - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("s,m", [(2, 3), (4, 2), (5, 1)])
def test_first_cycle_is_the_krylov_minimum_residual(s, m):
    pr = PB.convdiff(2, 7, 25.0)
    A = operator(pr)
    Ad = dense(A)
    rng = np.random.default_rng(4)
    f, x0 = rng.standard_normal(pr.N), rng.standard_normal(pr.N)
    x, r = O.sgmres(A, f, x0, s, m, 0.0, max_blocks=m, basis=O.NEWTON)
    xr = x0 + krylov_min_residual(Ad, f - Ad @ x0, s * m)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


@pytest.mark.parametrize("method", ["gmres", "omin"])
def test_same_iterates_as_monomial_when_well_conditioned(method):
    pr = PB.convdiff(2, 16, 10.0)
    A = operator(pr)
    f = np.cos(np.arange(pr.N) * 0.3)
    run = O.sgmres if method == "gmres" else O.somin
    kw = dict(max_blocks=6) if method == "gmres" else dict(max_iters=6)
    xa, ra = run(A, f, np.zeros(pr.N), 3, 2, 0.0, **kw)
    xb, rb = run(A, f, np.zeros(pr.N), 3, 2, 0.0, basis=O.NEWTON, **kw)
    assert ra.iters == rb.iters
    assert np.linalg.norm(xa - xb) <= 1e-9 * np.linalg.norm(xa)


def test_large_s_needs_fewer_blocks_than_monomial():
    pr = PB.convdiff(2, 48, 20.0)
    A = operator(pr)
    f = np.random.default_rng(0).standard_normal(pr.N)
    _, mono = O.sgmres(A, f, np.zeros(pr.N), 12, 4, 1e-10, max_blocks=20000)
    _, newt = O.sgmres(A, f, np.zeros(pr.N), 12, 4, 1e-10, max_blocks=20000, basis=O.NEWTON)
    assert newt.status == O.OK and mono.status == O.OK
    assert newt.iters < 0.7 * mono.iters and newt.cycles < mono.cycles, (newt.iters, mono.iters)
