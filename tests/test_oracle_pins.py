"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix
(closed forms, definitions solved by numpy, the paper's equivalence
statements).  CPU only."""
import numpy as np
import pytest

import oracle as O
from paper_2001_04886_amd import problems as PB
from helpers import dense, krylov_min_residual, operator, stencil_eigpair, window


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------------
# inputs
# --------------------------------------------------------------------------

def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0 yields 0xE220A8397B1DCDAF as its first output
    # (Steele, Lea & Flood; the reference output used by xoshiro seeding).
    assert int(PB.splitmix64(np.array([0], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_x_true_range_and_independence():
    a = PB.x_true(0, 100000)
    b = PB.x_true(1, 100000)
    assert a.min() >= -1.0 and a.max() < 1.0
    assert abs(a.mean()) < 0.01 and abs(a.std() - 1 / np.sqrt(3)) < 0.01
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01
    # counter-based: a slice equals the same slice of the whole
    np.testing.assert_array_equal(PB.uniform01(3, 10, offset=500), PB.uniform01(3, 510)[500:])


# --------------------------------------------------------------------------
# operator (Sec. 1 / Sec. 5 discretisation)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ndim,shape,gamma", [(2, (7, 5), 10.0), (2, (6, 9), 0.0),
                                               (3, (6, 7, 5), 10.0), (2, (16, 16), 20.0)])
def test_operator_closed_form_eigenpairs(ndim, shape, gamma):
    # real closed-form eigenpairs exist while the cell Peclet number gamma h / 2 < 1
    prob = PB.convdiff(ndim, shape[0], gamma, ny=shape[1], nz=shape[2] if ndim == 3 else None)
    A = operator(prob)
    rng = np.random.default_rng(1)
    for _ in range(5):
        js = [int(rng.integers(1, n + 1)) for n in shape[:ndim]]
        lam, v = stencil_eigpair(prob, js)
        Av = O.apply(A, v)
        assert rel(Av, lam * v) < 1e-12, (js, rel(Av, lam * v))


def test_operator_convdiff_eigenvalue_formula():
    # per-axis eigenvalues of the convection-diffusion matrix,
    # (2 - 2 sqrt(1 - (gamma h/2)^2) cos(j pi h)) / h^2, summed over axes
    n, gamma = 9, 10.0
    h = 1.0 / (n + 1)
    prob = PB.convdiff(2, n, gamma)
    lam, _ = stencil_eigpair(prob, [2, 5])
    ax = lambda j: (2 - 2 * np.sqrt(1 - (gamma * h / 2) ** 2) * np.cos(j * np.pi * h)) / h**2
    assert abs(lam - (ax(2) + ax(5))) < 1e-10 * abs(lam)


@pytest.mark.parametrize("ndim", [2, 3])
def test_operator_second_order_consistency(ndim):
    # A u_h approximates -Lap u + gamma * sum u_xd for a smooth u with zero
    # boundary values; the error must fall by ~4x when h halves.
    gamma = 10.0
    errs = []
    for n in ([16, 32] if ndim == 3 else [32, 64]):
        prob = PB.convdiff(ndim, n, gamma)
        A = operator(prob)
        h = 1.0 / (n + 1)
        g = np.arange(1, n + 1) * h
        if ndim == 2:
            Y, X = np.meshgrid(g, g, indexing="ij")
            u = np.sin(np.pi * X) * np.sin(np.pi * Y)
            Lu = 2 * np.pi**2 * u + gamma * np.pi * (np.cos(np.pi * X) * np.sin(np.pi * Y)
                                                     + np.sin(np.pi * X) * np.cos(np.pi * Y))
        else:
            Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
            sx, sy, sz = np.sin(np.pi * X), np.sin(np.pi * Y), np.sin(np.pi * Z)
            u = sx * sy * sz
            Lu = 3 * np.pi**2 * u + gamma * np.pi * (np.cos(np.pi * X) * sy * sz
                                                     + sx * np.cos(np.pi * Y) * sz
                                                     + sx * sy * np.cos(np.pi * Z))
        errs.append(np.abs(O.apply(A, u.ravel()) - Lu.ravel()).max())
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, errs


def test_operator_variable_coefficients_reduce_to_constant():
    prob = PB.convdiff(3, 5, 20.0, ny=4, nz=3)
    coef = np.repeat(prob.c[:, None], prob.N, axis=1)
    A1, A2 = operator(prob), O.Operator(3, 5, 4, 3, coef=coef)
    x = PB.x_true(2, prob.N)
    np.testing.assert_array_equal(O.apply(A1, x), O.apply(A2, x))


def test_diffusion_operator_symmetric_positive_definite():
    logk = PB.grf(12, 0.1, seed=3)
    A = O.Operator(2, 12, 12, coef=PB.diffusion_coef(logk))
    M = dense(A)
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_sigma_is_power_of_two_gershgorin_bound():
    for prob in [PB.convdiff(2, 64, 10.0), PB.convdiff(3, 256, 50.0), PB.convdiff(2, 7, 0.0)]:
        A = operator(prob)
        s = O.sigma(A)
        bound = np.abs(prob.c[: 2 * prob.ndim + 1]).sum()
        assert bound <= s < 2 * bound
        assert np.log2(s) == int(np.log2(s))


def test_chebyshev_interval_is_symmetric_part_spectrum():
    prob = PB.convdiff(2, 7, 30.0, ny=5)
    A = operator(prob)
    M = dense(A)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    c, d = O.cheb_interval(A)
    assert abs((c - d) - ev.min()) < 1e-9 * ev.max()
    assert abs((c + d) - ev.max()) < 1e-9 * ev.max()


def test_mpk_monomial_and_chebyshev_closed_forms():
    prob = PB.convdiff(2, 8, 10.0, ny=6)
    A = operator(prob)
    M = dense(A)
    s = 6
    y0 = PB.x_true(4, prob.N)
    sg = O.sigma(A)
    Y = O.mpk(A, y0, s, O.MONOMIAL)
    for j in range(s + 1):
        ref = np.linalg.matrix_power(M / sg, j) @ y0
        assert rel(Y[j], ref) < 1e-13
    # Chebyshev on an eigenvector v: y_j = T_j((lambda - c)/d) v, T_j the
    # Chebyshev polynomial of the first kind (numpy's Chebyshev class).
    lam, v = stencil_eigpair(prob, [3, 2])
    c, d = O.cheb_interval(A)
    Yc = O.mpk(A, v, s, O.CHEBYSHEV)
    t = (lam - c) / d
    for j in range(s + 1):
        Tj = np.polynomial.chebyshev.Chebyshev.basis(j)(t)
        assert rel(Yc[j], Tj * v) < 1e-11
    # both bases span the same Krylov space
    Ym = O.mpk(A, y0, s, O.MONOMIAL)
    Yc = O.mpk(A, y0, s, O.CHEBYSHEV)
    Qm, _ = np.linalg.qr(Ym.T)
    assert np.linalg.norm(Yc.T - Qm @ (Qm.T @ Yc.T)) < 1e-9 * np.linalg.norm(Yc)


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
def test_mpk_is_local_window_reproduces_grid(basis):
    # level j of the matrix powers at a point depends only on the points
    # within j grid steps (a (2j+1)-point-wide box, the 7-point stencil
    # applied j times); the grid clipped to that box, with the full grid's
    # scaling and interval, gives the same value bit for bit, at the domain
    # edge as well (clipped sides are the grid's own Dirichlet boundary)
    nx, ny, nz, s = 14, 11, 9, 4
    prob = PB.convdiff(3, nx, 50.0, ny=ny, nz=nz)
    A = operator(prob)
    y0 = PB.x_true(9, prob.N)
    sg = O.sigma(A)
    cc, cd = O.cheb_interval(A)
    Y = O.mpk(A, y0, s, basis)
    y1 = O.apply(A, y0)
    rng = np.random.default_rng(3)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny // 2, nz - 1), (nx - 2, 1, 4)]
    pts += [tuple(int(rng.integers(0, n)) for n in (nx, ny, nz)) for _ in range(20)]
    for pt in pts:
        p = pt[0] + nx * pt[1] + nx * ny * pt[2]
        dims, flat, ctr = window((nx, ny, nz), pt, s)
        W = O.Operator(3, *dims, c=prob.c)
        Yw = O.mpk(W, y0[flat], s, basis, params=(sg, cc, cd))
        assert np.array_equal(Yw[:, ctr], Y[:, p]), pt
        d1, f1, c1 = window((nx, ny, nz), pt, 1)
        assert O.apply(O.Operator(3, *d1, c=prob.c), y0[f1])[c1] == y1[p], pt
    # a window one step too narrow does not reproduce the last level (the
    # check above is not vacuous)
    pt = (7, 5, 4)
    dims, flat, ctr = window((nx, ny, nz), pt, s - 1)
    Yw = O.mpk(O.Operator(3, *dims, c=prob.c), y0[flat], s, basis, params=(sg, cc, cd))
    p = pt[0] + nx * pt[1] + nx * ny * pt[2]
    assert Yw[s - 1, ctr] == Y[s - 1, p] and Yw[s, ctr] != Y[s, p]


# --------------------------------------------------------------------------
# standard GMRES(M) (Sec. 2, Alg. 2.2, eqs. (2)-(3))
# --------------------------------------------------------------------------

def _tiny(gamma=10.0, nx=6, ny=5, seed=0):
    prob = PB.convdiff(2, nx, gamma, ny=ny, seed=seed)
    A = operator(prob)
    M = dense(A)
    xt = prob.x_true()
    f = M @ xt
    return prob, A, M, f


@pytest.mark.parametrize("Mk", [1, 3, 8, 12])
def test_gmres_one_cycle_is_krylov_minimiser(Mk):
    prob, A, M, f = _tiny()
    x0 = 0.1 * PB.x_true(9, prob.N)
    x, res = O.gmres(A, f, x0, Mk, 0.0, max_steps=Mk)
    z = krylov_min_residual(M, f - M @ x0, Mk)
    assert rel(x, x0 + z) < 1e-10


def test_gmres_full_krylov_is_exact():
    prob, A, M, f = _tiny(nx=5, ny=4)
    x, res = O.gmres(A, f, np.zeros(prob.N), prob.N, 1e-14)
    assert rel(x, np.linalg.solve(M, f)) < 1e-10
    assert res.status == O.OK


def test_gmres_arnoldi_relation_and_orthonormality():
    prob, A, M, f = _tiny()
    Mk = 10
    x, res, Q, H = O.gmres(A, f, np.zeros(prob.N), Mk, 0.0, max_steps=Mk, dump=True)
    assert np.abs(Q @ Q.T - np.eye(Mk + 1)).max() < 1e-12
    AQ = (M @ Q[:Mk].T)
    assert np.linalg.norm(AQ - Q.T @ H) < 1e-12 * np.linalg.norm(M, 2)
    assert np.allclose(np.tril(H, -2), 0.0)


def test_gmres_residuals_monotone():
    prob = PB.convdiff(2, 24, 20.0)
    A = operator(prob)
    f = O.apply(A, prob.x_true())
    x, res = O.gmres(A, f, np.zeros(prob.N), 15, 1e-10)
    assert res.status == O.OK and res.rel_resid <= 1e-10
    h = res.hist
    # the least-squares residual never grows inside a cycle; after a restart
    # it starts from the true residual of the previous iterate
    assert np.all(np.diff(h) <= 1e-12 * h[0])


# --------------------------------------------------------------------------
# Omin(k) / GCR (Sec. 2, Alg. 2.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("iters", [1, 2, 5, 9])
def test_gcr_iterate_is_krylov_minimiser(iters):
    prob, A, M, f = _tiny()
    x, res = O.omin(A, f, np.zeros(prob.N), 1000, 0.0, max_iters=iters)
    z = krylov_min_residual(M, f, iters)
    assert rel(x, z) < 1e-9


@pytest.mark.parametrize("iters", [2, 5, 8])
def test_omin1_equals_gcr_for_symmetric_matrix(iters):
    # for symmetric A the Orthomin(1) recurrence keeps all directions
    # A^T A-orthogonal, so it equals GCR (the minimiser over K_i)
    prob, A, M, f = _tiny(gamma=0.0)
    x, res = O.omin(A, f, np.zeros(prob.N), 1, 0.0, max_iters=iters)
    z = krylov_min_residual(M, f, iters)
    assert rel(x, z) < 1e-9


def test_omin_truncated_converges_monotone():
    prob = PB.convdiff(2, 16, 10.0)
    A = operator(prob)
    f = O.apply(A, prob.x_true())
    x, res = O.omin(A, f, np.zeros(prob.N), 4, 1e-10)
    assert res.status == O.OK and res.rel_resid <= 1e-10
    assert np.all(np.diff(res.hist) <= 1e-14)


# --------------------------------------------------------------------------
# s-step Orthomin(k) (Sec. 3, Alg. 3.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 3])
def test_somin_s1_is_omin(k):
    # with s = 1 the s-step method reduces to Omin(k) (Sec. 3)
    prob, A, M, f = _tiny(gamma=25.0, nx=9, ny=7)
    for iters in [1, 4, 10]:
        x1, _ = O.omin(A, f, np.zeros(prob.N), k, 0.0, max_iters=iters)
        x2, _ = O.somin(A, f, np.zeros(prob.N), 1, k, 0.0, max_iters=iters)
        assert rel(x2, x1) < 1e-11


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
@pytest.mark.parametrize("s", [2, 4])
def test_somin_first_iteration_is_s_step_mr(basis, s):
    # the first iteration minimises over span{r, Ar, .., A^{s-1} r} (s-MR = GMRES(s))
    prob, A, M, f = _tiny(gamma=10.0)
    x0 = 0.3 * PB.x_true(5, prob.N)
    x, _ = O.somin(A, f, x0, s, 3, 0.0, max_iters=1, basis=basis)
    z = krylov_min_residual(M, f - M @ x0, s)
    assert rel(x, x0 + z) < 1e-10


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_s_step_gcr_is_krylov_minimiser(basis, iters):
    # s-GCR (no truncation) after i iterations equals GMRES after i*s steps
    prob, A, M, f = _tiny(gamma=10.0, nx=8, ny=7)
    s = 3
    x, _ = O.somin(A, f, np.zeros(prob.N), s, 100, 0.0, max_iters=iters, basis=basis)
    z = krylov_min_residual(M, f, s * iters)
    assert rel(x, z) < 1e-8


@pytest.mark.parametrize("iters", [2, 3, 4])
def test_somin1_equals_s_gcr_for_symmetric_matrix(iters):
    # s-Omin(1) coincides with s-GCR for symmetric A (Sec. 3)
    prob, A, M, f = _tiny(gamma=0.0, nx=8, ny=7)
    s = 2
    x, _ = O.somin(A, f, np.zeros(prob.N), s, 1, 0.0, max_iters=iters)
    z = krylov_min_residual(M, f, s * iters)
    assert rel(x, z) < 1e-8


def test_somin_window_is_AtA_orthogonal_and_residual_minimal():
    prob = PB.convdiff(2, 12, 30.0, ny=10)
    A = operator(prob)
    f = O.apply(A, prob.x_true())
    s, k = 3, 3
    x, res, P, AP, r = O.somin(A, f, np.zeros(prob.N), s, k, 0.0, max_iters=7, dump=True)
    nb = AP.shape[0] // s
    assert nb == k
    nrm = np.linalg.norm(AP, axis=1)
    G = (AP @ AP.T) / np.outer(nrm, nrm)
    for a in range(nb):
        for b in range(nb):
            if a != b:
                blk = G[a * s:(a + 1) * s, b * s:(b + 1) * s]
                assert np.abs(blk).max() < 1e-8, (a, b, np.abs(blk).max())
    # r_{i+1} is orthogonal to the images of the last block (residual minimised)
    last = AP[(nb - 1) * s:]
    assert np.abs(last @ r).max() < 1e-10 * np.linalg.norm(r) * nrm.max()
    # Pk -> APk consistency: AP = A P
    for q in range(P.shape[0]):
        assert rel(O.apply(A, P[q]), AP[q]) < 1e-9


def test_somin_eigenvector_rhs_exact_in_one_iteration():
    prob = PB.convdiff(2, 10, 10.0, ny=8)
    A = operator(prob)
    lam, v = stencil_eigpair(prob, [2, 3])
    x, res = O.somin(A, v, np.zeros(prob.N), 4, 2, 1e-12)
    assert res.status == O.OK and res.iters == 1
    assert rel(x, v / lam) < 1e-12


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
def test_somin_small_workload_converges(basis):
    prob = PB.small_2d(0)
    A = operator(prob)
    f = O.apply(A, prob.x_true())
    x, res = O.somin(A, f, np.zeros(prob.N), 4, 4, 1e-8, basis=basis)
    assert res.status == O.OK and res.rel_resid <= 1e-8
    assert 30 <= res.iters <= 90, res.iters
    assert np.all(np.diff(res.hist) <= 1e-14)


# --------------------------------------------------------------------------
# s-step GMRES(m) (Sec. 4, Alg. 4.1-4.2, eqs. (4)-(8), Remark 4.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("basis,s,m,tolx", [(O.MONOMIAL, 1, 8, 1e-10), (O.MONOMIAL, 2, 5, 1e-10),
                                            (O.MONOMIAL, 4, 3, 1e-10), (O.CHEBYSHEV, 4, 3, 1e-10),
                                            (O.CHEBYSHEV, 6, 2, 1e-10),
                                            # the configured block sizes: monomial s = 8 (a
                                            # 9-column power basis, conditioning ~1e8: measured
                                            # 4e-8 here), Chebyshev and Newton s = 8 and 12
                                            # (measured <= 3e-14)
                                            (O.MONOMIAL, 8, 3, 1e-6), (O.MONOMIAL, 8, 2, 1e-6),
                                            (O.CHEBYSHEV, 8, 3, 1e-10), (O.CHEBYSHEV, 12, 2, 1e-10),
                                            (O.NEWTON, 8, 3, 1e-10), (O.NEWTON, 12, 2, 1e-10)])
def test_sgmres_cycle_is_gmres_ms_minimiser(basis, s, m, tolx):
    # Remark 4.1: one cycle of s-GMRES(m) gives the GMRES(ms) iterate
    prob, A, M, f = _tiny(gamma=10.0, nx=9, ny=8)
    x0 = 0.2 * PB.x_true(11, prob.N)
    x, res = O.sgmres(A, f, x0, s, m, 0.0, max_blocks=m, basis=basis)
    z = krylov_min_residual(M, f - M @ x0, s * m)
    assert rel(x, x0 + z) < tolx
    xg, _ = O.gmres(A, f, x0, s * m, 0.0, max_steps=s * m)
    assert rel(x, xg) < tolx


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
def test_sgmres_arnoldi_relation_block_orthogonality_and_D(basis):
    prob = PB.convdiff(2, 10, 20.0, ny=9)
    A = operator(prob)
    M = dense(A)
    f = M @ prob.x_true()
    s, m = 3, 5
    x, res, d = O.sgmres(A, f, np.zeros(prob.N), s, m, 0.0, max_blocks=m, basis=basis, dump=True)
    nc = d["ncols"]
    assert nc == s * m
    U = d["V"].T          # N x (nc+1)
    V = U[:, :nc]
    G = d["G"]            # (nc+1) x nc
    # eq. (5): A V_k = U_k Gbar_k
    assert np.linalg.norm(M @ V - U @ G) < 1e-12 * np.linalg.norm(M, 2) * np.linalg.norm(V)
    # Gbar is upper Hessenberg
    assert np.allclose(np.tril(G, -2), 0.0)
    # blocks mutually orthogonal (not inside a block), next vector normalised
    for i in range(m):
        for j in range(m):
            if i != j:
                Bi, Bj = V[:, i * s:(i + 1) * s], V[:, j * s:(j + 1) * s]
                assert np.abs(Bi.T @ Bj).max() < 1e-10 * np.linalg.norm(Bi) * np.linalg.norm(Bj)
    assert abs(np.linalg.norm(U[:, nc]) - 1.0) < 1e-13
    # D = U^T U is block diagonal with the W_k blocks (eq. (7))
    D = d["D"]
    assert np.linalg.norm(U.T @ U - D) < 1e-10 * np.linalg.norm(D)


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
@pytest.mark.parametrize("nx,ny,s,m", [(4, 3, 4, 3), (5, 3, 5, 3), (6, 4, 4, 6)])
def test_sgmres_full_krylov_exact_on_distinct_spectrum(basis, nx, ny, s, m):
    # non-square grids have N distinct eigenvalues, so K_N = R^N and one cycle
    # with ms = N returns the exact solution
    prob = PB.convdiff(2, nx, 10.0, ny=ny, seed=2)
    A = operator(prob)
    M = dense(A)
    f = M @ prob.x_true()
    x, res = O.sgmres(A, f, np.zeros(prob.N), s, m, 1e-13, basis=basis)
    assert res.status == O.OK
    assert rel(x, np.linalg.solve(M, f)) < 1e-9


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
def test_sgmres_eigenvector_rhs_lucky_breakdown(basis):
    prob = PB.convdiff(2, 10, 10.0, ny=8)
    A = operator(prob)
    lam, v = stencil_eigpair(prob, [4, 1])
    x, res = O.sgmres(A, v, np.zeros(prob.N), 4, 5, 1e-12, basis=basis)
    assert res.status == O.OK and res.iters == 1 and res.cycles == 1
    assert rel(x, v / lam) < 1e-12


def test_sgmres_square_grid_rank_truncation():
    # square grids have paired eigenvalues, so the Krylov space saturates below
    # N and a block's Gram matrix turns singular: the block is truncated
    prob = PB.convdiff(2, 4, 10.0, seed=3)
    A = operator(prob)
    M = dense(A)
    f = M @ prob.x_true()
    x, res = O.sgmres(A, f, np.zeros(prob.N), 4, 4, 1e-12)
    assert res.status == O.OK and np.all(np.isfinite(x))
    assert rel(x, np.linalg.solve(M, f)) < 1e-9


@pytest.mark.parametrize("basis", [O.MONOMIAL, O.CHEBYSHEV])
def test_sgmres_small_workload(basis):
    prob = PB.small_2d(0)
    A = operator(prob)
    f = O.apply(A, prob.x_true())
    x, res = O.sgmres(A, f, np.zeros(prob.N), 4, 20, 1e-8, basis=basis)
    assert res.status == O.OK and res.rel_resid <= 1e-8
    assert res.cycles <= 4 and res.iters <= 80, (res.cycles, res.iters)
    # least-squares residual estimate never increases inside a cycle
    h = res.hist
    starts = [0] + [i for i in range(1, len(h)) if i % 20 == 0]
    for a, b in zip(starts, starts[1:] + [len(h)]):
        assert np.all(np.diff(h[a:b]) <= 1e-12)


def test_sgmres_restarts_reduce_true_residual():
    prob = PB.convdiff(2, 32, 10.0)
    A = operator(prob)
    f = O.apply(A, prob.x_true())
    x = np.zeros(prob.N)
    last = 1.0
    for _ in range(3):
        x, res = O.sgmres(A, f, x, 4, 5, 0.0, max_blocks=5)
        assert res.rel_resid <= last
        last = res.rel_resid
    assert last < 1e-2


# --------------------------------------------------------------------------
# failure handling
# --------------------------------------------------------------------------

def test_bad_arguments_and_nonfinite_inputs():
    prob, A, M, f = _tiny()
    x0 = np.zeros(prob.N)
    assert O.sgmres(A, f, x0, 0, 4, 1e-8)[1].status == O.ERR_ARG
    assert O.sgmres(A, f, x0, 4, 0, 1e-8)[1].status == O.ERR_ARG
    assert O.somin(A, f, x0, 17, 2, 1e-8)[1].status == O.ERR_ARG
    assert O.somin(A, f, x0, 2, 2, -1.0)[1].status == O.ERR_ARG
    fb = f.copy()
    fb[3] = np.nan
    assert O.sgmres(A, fb, x0, 2, 4, 1e-8)[1].status == O.ERR_NONFINITE
    assert O.somin(A, fb, x0, 2, 2, 1e-8)[1].status == O.ERR_NONFINITE
    x, res = O.sgmres(A, f, x0, 2, 2, 0.0, max_blocks=3)
    assert res.status == O.NOT_CONVERGED and res.iters == 3
