"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle
and against definitions computed with numpy, on seeded inputs.

Tolerances.  Kernels: rounding-level (a few ulp of the operand scale).
Solvers run for the same number of blocks / iterations as the oracle
(tol = 0, capped) so the iterates are comparable; the bar is
||x - x_oracle|| / ||x_oracle|| <= 1e-8 (the rounding-order difference
between the two implementations measured here is ~1e-12)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2001_04886_amd import problems as PB
from paper_2001_04886_amd import sstep as S
from helpers import operator, stencil_eigpair

pytestmark = pytest.mark.gpu

DEV = "cuda"


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problem_pair(prob):
    return operator(prob), S.Stencil.from_problem(prob)


# --------------------------------------------------------------------------
# kernels
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ndim,shape,gamma", [(2, (64, 64), 10.0), (2, (37, 23), 50.0),
                                               (2, (300, 5), 1.0), (3, (13, 11, 7), 50.0),
                                               (3, (257, 3, 2), 5.0), (2, (1, 1), 0.0)])
def test_stencil_apply_matches_oracle(ndim, shape, gamma):
    prob = PB.convdiff(ndim, shape[0], gamma, ny=shape[1], nz=shape[2] if ndim == 3 else None)
    Ao, Ag = problem_pair(prob)
    x = PB.x_true(5, prob.N)
    y = torch.empty(prob.N, dtype=torch.float64, device=DEV)
    S.stencil_apply(Ag, dev(x), y)
    yo = O.apply(Ao, x)
    scale = np.abs(prob.c).sum()
    assert np.abs(host(y) - yo).max() <= 4e-16 * scale * 8


def test_stencil_apply_variable_coefficients():
    logk = PB.grf(40, 0.1, seed=1)
    coef = PB.diffusion_coef(logk)
    Ao = O.Operator(2, 40, 40, coef=coef)
    cd = dev(coef)
    Ag = S.Stencil(2, 40, 40, 1, (0.0,) * 7, cd)
    x = PB.x_true(2, 1600)
    y = torch.empty(1600, dtype=torch.float64, device=DEV)
    S.stencil_apply(Ag, dev(x), y)
    yo = O.apply(Ao, x)
    assert np.abs(host(y) - yo).max() <= 1e-14 * np.abs(coef).sum(0).max()


@pytest.mark.parametrize("basis", [S.MONOMIAL, S.CHEBYSHEV])
@pytest.mark.parametrize("ndim,shape,s", [(2, (33, 17), 4), (3, (9, 10, 11), 8), (2, (64, 64), 12),
                                          (3, (40, 35, 70), 8), (2, (300, 7), 5), (3, (17, 33, 9), 12),
                                          (2, (1000, 50), 16), (3, (5, 4, 3), 1), (2, (2, 300), 3),
                                          (3, (70, 3, 200), 6)])
def test_matrix_powers_match_oracle(basis, ndim, shape, s):
    prob = PB.convdiff(ndim, shape[0], 20.0, ny=shape[1], nz=shape[2] if ndim == 3 else None)
    Ao, Ag = problem_pair(prob)
    w = PB.x_true(7, prob.N)
    scale = 0.37
    ld = (prob.N + 63) // 64 * 64
    Y = torch.zeros((s + 1, ld), dtype=torch.float64, device=DEV)
    Y[0, : prob.N] = dev(w)
    sg = O.sigma(Ao)
    cc, cd = O.cheb_interval(Ao)
    S.kernel_mpk(Ag, Y, s, basis, scale, sg, cc, cd)
    Yo = O.mpk(Ao, w * scale, s, basis)
    Yg = host(Y)[:, : prob.N]
    for j in range(1, s + 1):
        assert rel(Yg[j], Yo[j]) < 1e-13 * (j + 1), j


@pytest.mark.parametrize("N,ncx,ncz", [(1, 1, 1), (1000, 7, 3), (4097, 40, 8), (65536 + 513, 64, 9),
                                       (300001, 17, 16), (1024 * 1024 + 5, 40, 8),
                                       # every Z width class, chunks shorter than one step,
                                       # ragged column groups of the shared-Z kernel
                                       (127, 3, 8), (130, 5, 4), (5000, 20, 2), (70001, 33, 12),
                                       (123457, 18, 13), (262147, 50, 16)])
def test_block_gram_matches_numpy(N, ncx, ncz):
    rng = np.random.default_rng(N)
    ld = (N + 63) // 64 * 64
    X = torch.zeros((ncx, ld), dtype=torch.float64, device=DEV)
    Z = torch.zeros((ncz, ld), dtype=torch.float64, device=DEV)
    Xh = rng.standard_normal((ncx, N))
    Zh = rng.standard_normal((ncz, N))
    X[:, :N] = dev(Xh)
    Z[:, :N] = dev(Zh)
    G = host(S.kernel_gram(X[:, :N], Z[:, :N]))
    ref = Xh @ Zh.T
    bound = 1e-15 * np.sqrt(N) * 8 * np.outer(np.linalg.norm(Xh, axis=1), np.linalg.norm(Zh, axis=1))
    assert np.all(np.abs(G - ref) <= bound + 1e-300)
    # deterministic: same bits on a second call
    G2 = host(S.kernel_gram(X[:, :N], Z[:, :N]))
    assert np.array_equal(G, G2)


@pytest.mark.parametrize("N,nc", [(1, 1), (5, 2), (1000, 3), (4097, 5), (65536 + 513, 9),
                                  (300001, 4), (1024 * 1024 + 5, 9), (2 << 20, 7), (77777, 13)])
def test_block_self_gram_matches_numpy(N, nc):
    # X^T X of one block (the one-pass symmetric kernel for <= 9 columns, the
    # general block Gram beyond): symmetric to the bit, within the summation bound
    rng = np.random.default_rng(N + 7 * nc)
    ld = (N + 63) // 64 * 64
    X = torch.zeros((nc, ld), dtype=torch.float64, device=DEV)
    Xh = rng.standard_normal((nc, N))
    X[:, :N] = dev(Xh)
    G = host(S.kernel_gram(X[:, :N], X[:, :N]))
    ref = Xh @ Xh.T
    nrm = np.linalg.norm(Xh, axis=1)
    assert np.all(np.abs(G - ref) <= 1e-15 * np.sqrt(N) * 8 * np.outer(nrm, nrm) + 1e-300)
    assert np.array_equal(G, G.T)
    assert np.array_equal(G, host(S.kernel_gram(X[:, :N], X[:, :N])))


@pytest.mark.parametrize("N,ncx,ncy", [(1, 1, 1), (999, 0, 3), (4097, 40, 8), (100003, 13, 16),
                                       (1 << 20, 64, 1), (511, 5, 1), (512, 6, 9), (513, 7, 2),
                                       (2047, 128, 5), (2049, 130, 16), (100003, 201, 8)])
def test_block_update_matches_numpy(N, ncx, ncy):
    rng = np.random.default_rng(N + ncx)
    ld = (N + 63) // 64 * 64
    Xh = rng.standard_normal((max(ncx, 1), N))
    Yh = rng.standard_normal((ncy, N))
    Mh = rng.standard_normal((max(ncx, 1), ncy))
    X = torch.zeros((max(ncx, 1), ld), dtype=torch.float64, device=DEV)
    Y = torch.zeros((ncy, ld), dtype=torch.float64, device=DEV)
    X[:, :N] = dev(Xh)
    Y[:, :N] = dev(Yh)
    S.kernel_update(X[:ncx, :N], Y[:, :N], dev(Mh[:ncx]) if ncx else None)
    ref = Yh + (Xh[:ncx].T @ Mh[:ncx]).T if ncx else Yh
    assert np.abs(host(Y)[:, :N] - ref).max() <= 1e-14 * (np.abs(Xh).max() * np.abs(Mh).sum(0).max() + 1)


# --------------------------------------------------------------------------
# solvers vs oracle
# --------------------------------------------------------------------------

def solve_pair(prob, method, s, km, tol, max_iters=0, basis=S.MONOMIAL, x0=None, f=None):
    Ao, Ag = problem_pair(prob)
    if f is None:
        f = O.apply(Ao, prob.x_true())
    x0 = np.zeros(prob.N) if x0 is None else x0
    xd = dev(x0.copy())
    if method == "gmres":
        info = S.gmres_solve(Ag, dev(f), xd, s, km, tol, max_iters=max_iters, basis=basis)
        xo, res = O.sgmres(Ao, f, x0, s, km, tol, max_blocks=max_iters, basis=basis)
    else:
        info = S.omin_solve(Ag, dev(f), xd, s, km, tol, max_iters=max_iters, basis=basis)
        xo, res = O.somin(Ao, f, x0, s, km, tol, max_iters=max_iters, basis=basis)
    return host(xd), info, xo, res


@pytest.mark.parametrize("basis", [S.MONOMIAL, S.CHEBYSHEV])
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_sgmres_small_workload_fixed_blocks(seed, basis):
    # 64 x 64, gamma 10, s-GMRES(m=20, s=4), exactly 45 blocks (3 cycles)
    prob = PB.small_2d(seed)
    xg, info, xo, res = solve_pair(prob, "gmres", 4, 20, 0.0, max_iters=45, basis=basis)
    assert info.status == S.NOT_CONVERGED and res.status == O.NOT_CONVERGED
    assert info.iters == res.iters == 45 and info.cycles == res.cycles == 3
    assert rel(xg, xo) <= 1e-8, rel(xg, xo)


@pytest.mark.parametrize("basis", [S.MONOMIAL, S.CHEBYSHEV])
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_somin_small_workload_fixed_iterations(seed, basis):
    prob = PB.small_2d(seed)
    xg, info, xo, res = solve_pair(prob, "omin", 4, 4, 0.0, max_iters=40, basis=basis)
    assert info.iters == res.iters == 40
    assert rel(xg, xo) <= 1e-8, rel(xg, xo)


@pytest.mark.parametrize("method,s,km", [("gmres", 4, 20), ("omin", 4, 4)])
def test_small_workload_converged_tol_1e12(method, s, km):
    prob = PB.small_2d(0)
    xg, info, xo, res = solve_pair(prob, method, s, km, 1e-12)
    assert info.status == S.OK and res.status == O.OK
    assert info.rel_resid <= 1e-12
    assert abs(info.iters - res.iters) <= 1
    assert rel(xg, xo) <= 1e-8
    xt = prob.x_true()
    assert rel(xg, xt) <= 1e-8


@pytest.mark.parametrize("method,s,km", [("gmres", 4, 20), ("omin", 4, 4)])
def test_small_workload_tol_1e8(method, s, km):
    prob = PB.small_2d(1)
    xg, info, xo, res = solve_pair(prob, method, s, km, 1e-8)
    assert info.status == S.OK and info.rel_resid <= 1e-8
    assert info.iters == res.iters
    assert rel(xg, xo) <= 1e-8


@pytest.mark.parametrize("case", ["ragged2d", "tiny3d", "s1", "m1", "s8m5", "s16"])
def test_sgmres_edge_shapes(case):
    prob, s, m, nb = {
        "ragged2d": (PB.convdiff(2, 37, 30.0, ny=23, seed=3), 4, 6, 14),
        "tiny3d": (PB.convdiff(3, 7, 50.0, ny=5, nz=6, seed=4), 3, 5, 9),
        "s1": (PB.convdiff(2, 20, 10.0, seed=5), 1, 12, 30),
        "m1": (PB.convdiff(2, 20, 10.0, seed=6), 4, 1, 7),
        "s8m5": (PB.convdiff(3, 12, 50.0, seed=7), 8, 5, 8),
        "s16": (PB.convdiff(2, 30, 10.0, seed=8), 16, 2, 3),
    }[case]
    basis = S.CHEBYSHEV if s >= 8 else S.MONOMIAL
    xg, info, xo, res = solve_pair(prob, "gmres", s, m, 0.0, max_iters=nb, basis=basis)
    assert info.iters == res.iters == nb and info.cycles == res.cycles
    assert rel(xg, xo) <= 1e-8, rel(xg, xo)


@pytest.mark.parametrize("basis", [S.MONOMIAL, S.CHEBYSHEV])
def test_sgmres_eigenvector_lucky_breakdown(basis):
    prob = PB.convdiff(2, 10, 10.0, ny=8)
    lam, v = stencil_eigpair(prob, [4, 1])
    xg, info, xo, res = solve_pair(prob, "gmres", 4, 5, 1e-12, basis=basis, f=v)
    assert info.status == S.OK and info.iters == 1 and info.cycles == 1
    assert rel(xg, v / lam) <= 1e-12


def test_somin_eigenvector_one_iteration():
    prob = PB.convdiff(2, 10, 10.0, ny=8)
    lam, v = stencil_eigpair(prob, [2, 3])
    xg, info, xo, res = solve_pair(prob, "omin", 4, 2, 1e-12, f=v)
    assert info.status == S.OK and info.iters == 1
    assert rel(xg, v / lam) <= 1e-12


def test_sgmres_square_grid_rank_truncation():
    prob = PB.convdiff(2, 4, 10.0, seed=3)
    xg, info, xo, res = solve_pair(prob, "gmres", 4, 4, 1e-12)
    assert info.status == S.OK and np.all(np.isfinite(xg))
    assert info.iters == res.iters and info.cycles == res.cycles
    assert rel(xg, xo) <= 1e-8


@pytest.mark.parametrize("nx,ny,s,m", [(4, 3, 4, 3), (6, 4, 4, 6)])
def test_sgmres_full_krylov_exact(nx, ny, s, m):
    prob = PB.convdiff(2, nx, 10.0, ny=ny, seed=2)
    xg, info, xo, res = solve_pair(prob, "gmres", s, m, 1e-13)
    assert info.status == S.OK
    assert rel(xg, prob.x_true()) <= 1e-9


def test_omin_window_truncation_and_restart_path():
    # k smaller than the iteration count (ring buffer wraps), ragged grid
    prob = PB.convdiff(2, 29, 40.0, ny=31, seed=9)
    xg, info, xo, res = solve_pair(prob, "omin", 3, 2, 0.0, max_iters=25)
    assert info.iters == res.iters == 25
    assert rel(xg, xo) <= 1e-8


def test_nonzero_initial_guess():
    prob = PB.convdiff(2, 24, 10.0, seed=11)
    x0 = 0.05 * (np.arange(prob.N) % 50)   # the paper's initial guess x(i) = 0.05 mod(i, 50)
    xg, info, xo, res = solve_pair(prob, "gmres", 4, 8, 0.0, max_iters=12, x0=x0)
    assert rel(xg, xo) <= 1e-8
    xg, info, xo, res = solve_pair(prob, "omin", 4, 3, 0.0, max_iters=12, x0=x0)
    assert rel(xg, xo) <= 1e-8


@pytest.mark.parametrize("method,kw", [
    ("gmres", {}), ("gmres", {"precision": S.MIXED}), ("gmres", {"basis": S.NEWTON}),
    ("gmres", {"graph": True}), ("gmres", {"precond": S.PRECOND_ILU0}),
    ("omin", {}), ("omin", {"orth": S.ORTH_MGS}), ("omin", {"precond": S.PRECOND_ILU0})])
def test_initial_guess_already_converged(method, kw):
    # x0 = x_true with f = A x_true (built by the oracle): the initial true
    # residual is at rounding level, so every form stops before its first
    # block / iteration and returns x0 (up to the round trip through the
    # preconditioned unknown u = LU x)
    if "precond" in kw:
        prob = PB.convdiff(2, 37, 30.0, ny=23, seed=12)
    else:
        prob = PB.convdiff(3, 13, 30.0, ny=11, nz=9, seed=12)
    Ao, Ag = problem_pair(prob)
    xt = prob.x_true()
    f = O.apply(Ao, xt)
    x = dev(xt.copy())
    if method == "gmres":
        info = S.gmres_solve(Ag, dev(f), x, 4, 5, 1e-8, **kw)
    else:
        info = S.omin_solve(Ag, dev(f), x, 4, 3, 1e-8, **kw)
    assert info.status == S.OK
    assert info.iters == 0
    assert info.rel_resid <= 1e-12
    assert rel(host(x), xt) <= 1e-12


def test_error_paths():
    prob = PB.convdiff(2, 16, 10.0)
    Ao, Ag = problem_pair(prob)
    f = O.apply(Ao, prob.x_true())
    fb = f.copy()
    fb[17] = np.nan
    x = torch.zeros(prob.N, dtype=torch.float64, device=DEV)
    assert S.gmres_solve(Ag, dev(fb), x, 4, 4, 1e-8).status == S.ERR_NONFINITE
    x.zero_()
    assert S.omin_solve(Ag, dev(fb), x, 4, 4, 1e-8).status == S.ERR_NONFINITE
    x.zero_()
    info = S.gmres_solve(Ag, dev(f), x, 2, 2, 0.0, max_iters=3)
    assert info.status == S.NOT_CONVERGED and info.iters == 3
    # zero right-hand side: x = 0 is exact
    x.zero_()
    info = S.gmres_solve(Ag, torch.zeros_like(x), x, 4, 4, 1e-8)
    assert info.status == S.OK and info.iters == 0
    # a workspace that is too small is rejected
    ws = torch.empty(1024, dtype=torch.uint8, device=DEV)
    assert S.gmres_solve(Ag, dev(f), x, 4, 4, 1e-8, workspace=ws).status == S.ERR_NOMEM


def test_caller_workspace_and_stream():
    prob = PB.convdiff(3, 20, 50.0, seed=1)
    Ao, Ag = problem_pair(prob)
    f = O.apply(Ao, prob.x_true())
    ws = S.allocate_workspace(Ag, S.METHOD_GMRES, 8, 5)
    st = torch.cuda.Stream()
    x = torch.zeros(prob.N, dtype=torch.float64, device=DEV)
    with torch.cuda.stream(st):
        info = S.gmres_solve(Ag, dev(f), x, 8, 5, 1e-10, workspace=ws, basis=S.CHEBYSHEV)
    assert info.status == S.OK and info.rel_resid <= 1e-10
    xo, res = O.sgmres(Ao, f, np.zeros(prob.N), 8, 5, 1e-10, basis=O.CHEBYSHEV)
    assert info.iters == res.iters
    assert rel(host(x), xo) <= 1e-8


# --------------------------------------------------------------------------
# mixed precision: FP32 basis / matrix powers / block updates, FP64 Gram,
# least squares, x and restart residual (iterative refinement by restarts)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ndim,n,s,m,basis", [(3, 24, 4, 10, S.MONOMIAL), (3, 24, 8, 10, S.MONOMIAL),
                                              (3, 24, 12, 6, S.CHEBYSHEV), (2, 64, 4, 20, S.MONOMIAL),
                                              (2, 37, 8, 5, S.CHEBYSHEV)])
def test_mixed_precision_reaches_fp64_accuracy(ndim, n, s, m, basis):
    # parity unpinned by the paper: the mixed result is checked by its true
    # FP64 residual and against the FP64 oracle solved to 1e-12
    prob = PB.convdiff(ndim, n, 50.0 if ndim == 3 else 10.0, seed=3)
    Ao, Ag = problem_pair(prob)
    f = O.apply(Ao, prob.x_true())
    x = torch.zeros(prob.N, dtype=torch.float64, device=DEV)
    info = S.gmres_solve(Ag, dev(f), x, s, m, 1e-10, precision=S.MIXED, basis=basis)
    assert info.status == S.OK, info
    assert info.rel_resid <= 1e-10
    xg = host(x)
    # independent FP64 residual check on the host
    r = f - O.apply(Ao, xg)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-10
    xo, res = O.sgmres(Ao, f, np.zeros(prob.N), s, m, 1e-12, basis=basis)
    assert rel(xg, xo) <= 1e-7, rel(xg, xo)


def test_mixed_precision_workspace_is_half():
    A = S.Stencil(3, 64, 64, 64, (1.0,) * 7)
    assert S.workspace_bytes(A, S.METHOD_GMRES, 8, 10, S.MIXED) < 0.6 * S.workspace_bytes(A, S.METHOD_GMRES, 8, 10)
