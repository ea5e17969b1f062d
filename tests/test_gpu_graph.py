"""s-GMRES with the restart cycle captured in a hipGraph (opt.graph) against
the eager launches of the same library: the same kernels in the same order,
so iterates, counts and residuals must agree bit for bit.  Each solve replays
its graph once per restart cycle with host synchronisations in between, the
last cycle of a capped solve is captured again with fewer blocks, and the
cases cover the fused 3-D matrix powers, per-level 2-D launches, variable
coefficients with ILU(0) right preconditioning and mixed precision."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2001_04886_amd import problems as PB
from paper_2001_04886_amd import sstep as S

pytestmark = pytest.mark.gpu


def solve(A, f, x0, s, m, tol, **kw):
    x = x0.clone()
    info = S.gmres_solve(A, f, x, s, m, tol, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


CASES = [
    ("small2d", dict(s=4, m=20, tol=1e-8)),
    ("cube128", dict(s=8, m=4, tol=1e-8)),
    ("paper64_ilu0", dict(s=2, m=5, tol=1e-10, precond=S.PRECOND_ILU0)),
    ("cube32_mixed", dict(s=8, m=6, tol=1e-10, precision=S.MIXED)),
    ("small2d_capped", dict(s=4, m=6, tol=1e-14, max_iters=15)),
]


def setup(name):
    if name.startswith("small2d"):
        pr = PB.small_2d()
    elif name.startswith("cube128"):
        pr = PB.convdiff(3, 128, 50.0)  # fused matrix-powers launches
    elif name.startswith("cube32"):
        pr = PB.convdiff(3, 32, 50.0)
    else:
        pr = PB.paper_problem(64)
    coef = torch.from_numpy(pr.coef).cuda() if pr.coef is not None else None
    A = S.Stencil.from_problem(pr, coef)
    rng = np.random.default_rng(7)
    f = torch.from_numpy(rng.standard_normal(pr.N)).cuda()
    return A, f, torch.zeros(pr.N, dtype=torch.float64, device="cuda"), coef


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_graph_replay_matches_eager(name, kw):
    print(f"graph replay {name}", flush=True)
    A, f, x0, keep = setup(name)
    kw = dict(kw)
    s, m, tol = kw.pop("s"), kw.pop("m"), kw.pop("tol")
    xe, ie = solve(A, f, x0, s, m, tol, **kw)
    for rep in range(2):
        xg, ig = solve(A, f, x0, s, m, tol, graph=True, **kw)
        assert (ig.status, ig.iters, ig.cycles, ig.matvecs) == (ie.status, ie.iters, ie.cycles,
                                                                ie.matvecs)
        assert ig.rel_resid == ie.rel_resid
        assert np.array_equal(xg, xe)
    assert ie.cycles >= 3
