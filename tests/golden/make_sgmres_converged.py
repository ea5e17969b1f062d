"""Writes sgmres_3d128_s8m40_tol1e-12.txt: the FP64 oracle's converged s-step
GMRES(m = 40, s = 8) solution (monomial basis, Sec. 4, Alg. 4.1-4.2) of the
3-D 7-point convection-diffusion problem on 128^3 (gamma = 50,
f = A x_true, x_true seed 0, x0 = 0) to a true relative residual of 1e-12,
sampled at 8192 seeded points.  The oracle needs about a quarter of an hour
for this solve on one core, too long to repeat inside a GPU test, so the
samples are stored.  Calls only the oracle and the input generators.

    python tests/golden/make_sgmres_converged.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2001_04886_amd import problems as PB  # noqa: E402

N_SIDE, GAMMA, S, M, TOL, NSAMP = 128, 50.0, 8, 40, 1e-12, 8192
OUT = os.path.join(HERE, f"sgmres_3d{N_SIDE}_s{S}m{M}_tol1e-12.txt")


def sample_points(n: int) -> np.ndarray:
    """Seeded sample of grid points: the first and last 64 points and
    uniformly drawn ones (sorted, distinct)."""
    rng = np.random.default_rng(20011)
    idx = np.concatenate([np.arange(64), np.arange(n - 64, n),
                          rng.choice(n, NSAMP - 128, replace=False)])
    return np.unique(idx)


def main():
    prob = PB.convdiff(3, N_SIDE, GAMMA)
    A = O.Operator(3, N_SIDE, N_SIDE, N_SIDE, c=prob.c)
    xt = prob.x_true()
    f = O.apply(A, xt)
    x, res = O.sgmres(A, f, np.zeros(prob.N), S, M, TOL)
    assert res.status == O.OK, res.status
    idx = sample_points(prob.N)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle, s-step GMRES(m=%d, s=%d), monomial basis, 3-D 7-pt "
                 "convection-diffusion %d^3, gamma=%g, f = A x_true (seed 0), x0 = 0, "
                 "tol %g on the true relative residual\n" % (M, S, N_SIDE, GAMMA, TOL))
        fh.write("# written by tests/golden/make_sgmres_converged.py (oracle only)\n")
        fh.write("blocks %d\ncycles %d\nrel_resid %.17e\nnorm_x %.17e\nerr_vs_true %.17e\n"
                 % (res.iters, res.cycles, res.rel_resid, np.linalg.norm(x),
                    np.linalg.norm(x - xt) / np.linalg.norm(xt)))
        fh.write("# point index, x[index]\n")
        for i in idx:
            fh.write("%d %.17e\n" % (i, x[i]))
    print(OUT, res.iters, res.cycles, res.rel_resid)


if __name__ == "__main__":
    main()
