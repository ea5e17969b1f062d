"""GPU parity of the Newton basis (Leja-ordered Chebyshev-point shifts of the
spectral interval) through the C ABI against the FP64 oracle: fixed work for
s-GMRES and s-Omin on per-level and fused matrix-powers paths (2-D and 3-D),
converged runs at large s, and mixed precision."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2001_04886_amd import problems as PB
from paper_2001_04886_amd import sstep as S
from helpers import operator
import parity_bounds as PBND

# the measured-spread bound of the same case (Newton, s = 8, m = 2, 2 blocks,
# f_p = cos(0.37 p) + 0.1 on 128^3)
BOUND_128 = [c for c in PBND.CASES if c[0] == "3d128-newton-s8m2-b2-cos"][0][-1]

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [  # (ndim, n, gamma, method, s, k_or_m, blocks)
    (2, 48, 20.0, "gmres", 4, 3, 6),
    (2, 48, 20.0, "omin", 6, 2, 5),
    # fused 2-D matrix powers; s = 4 (at s = 8 the 2048^2 Krylov basis is so
    # ill-conditioned that rounding moves the iterate by 1e-7 for the Newton
    # and Chebyshev bases alike, 6e-4 for the monomial one)
    (2, 2048, 5.0, "gmres", 4, 2, 2),
    (3, 40, 50.0, "gmres", 8, 2, 4),
    # fused 3-D matrix powers; after 16 Krylov steps of this s = 8 basis on
    # 128^3 with the smooth right-hand side, rounding alone moves the oracle's
    # own iterate by 3.5e-7 (tests/test_rounding_spread.py), hence the bound
    # of parity_bounds.CASES for this case instead of 1e-8
    (3, 128, 50.0, "gmres", 8, 2, 2),
    (3, 24, 50.0, "omin", 8, 2, 4),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}d{c[1]}-{c[3]}-s{c[4]}" for c in CASES])
def test_fixed_work(case):
    ndim, n, gamma, method, s, km, nb = case
    print(f"newton fixed work {case}", flush=True)
    pr = PB.convdiff(ndim, n, gamma)
    A = operator(pr)
    Ag = S.Stencil.from_problem(pr)
    f = np.cos(np.arange(pr.N) * 0.37) + 0.1
    xd = torch.zeros(pr.N, dtype=torch.float64, device="cuda")
    fd = torch.from_numpy(f).cuda()
    if method == "gmres":
        info = S.gmres_solve(Ag, fd, xd, s, km, 0.0, max_iters=nb, basis=S.NEWTON)
        xo, res = O.sgmres(A, f, np.zeros(pr.N), s, km, 0.0, max_blocks=nb, basis=O.NEWTON)
    else:
        info = S.omin_solve(Ag, fd, xd, s, km, 0.0, max_iters=nb, basis=S.NEWTON)
        xo, res = O.somin(A, f, np.zeros(pr.N), s, km, 0.0, max_iters=nb, basis=O.NEWTON)
    torch.cuda.synchronize()
    assert info.iters == res.iters == nb
    assert info.cheb_centre == pytest.approx(O.cheb_interval(A)[0], rel=1e-14)
    assert info.rel_resid == pytest.approx(res.rel_resid, rel=1e-9)
    bound = BOUND_128 if n >= 128 and ndim == 3 else PBND.CONTRACT
    assert rel(xd.cpu().numpy(), xo) <= bound, rel(xd.cpu().numpy(), xo)


@pytest.mark.parametrize("s", [12, 16])
def test_converged_large_s(s):
    print(f"newton converged s={s}", flush=True)
    pr = PB.convdiff(2, 64, 20.0)
    A = operator(pr)
    Ag = S.Stencil.from_problem(pr)
    f = np.random.default_rng(s).standard_normal(pr.N)
    xd = torch.zeros(pr.N, dtype=torch.float64, device="cuda")
    info = S.gmres_solve(Ag, torch.from_numpy(f).cuda(), xd, s, 4, 1e-10, basis=S.NEWTON)
    xo, res = O.sgmres(A, f, np.zeros(pr.N), s, 4, 1e-10, max_blocks=20000, basis=O.NEWTON)
    torch.cuda.synchronize()
    assert info.status == S.OK and res.status == O.OK and info.rel_resid <= 1e-10
    assert abs(info.iters - res.iters) <= 1, (info.iters, res.iters)
    assert rel(xd.cpu().numpy(), xo) <= 1e-8


def test_mixed_precision_newton():
    print("newton mixed precision", flush=True)
    pr = PB.convdiff(3, 48, 50.0)
    A = operator(pr)
    Ag = S.Stencil.from_problem(pr)
    f = np.random.default_rng(1).standard_normal(pr.N)
    xd = torch.zeros(pr.N, dtype=torch.float64, device="cuda")
    info = S.gmres_solve(Ag, torch.from_numpy(f).cuda(), xd, 12, 4, 1e-10, basis=S.NEWTON,
                         precision=S.MIXED)
    torch.cuda.synchronize()
    assert info.status == S.OK and info.rel_resid <= 1e-10
    r = f - O.apply(A, xd.cpu().numpy())
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(f)
