"""Fixed-work GPU parity cases whose iterate bound is set by the rounding
spread of the method itself, and those bounds.

At a fixed amount of work (a given number of s-blocks, tol = 0) the iterate
is the least-squares minimiser over the Krylov space the blocks span
(Remark 4.1).  With the monomial basis at s = 8 that space is represented by
blocks of power vectors whose conditioning grows like the ratio of the
extreme eigenvalues to the eighth power, so rounding alone moves the computed
minimiser far above 1e-8.  ``tests/test_rounding_spread.py`` measures, on the
CPU, how far the FP64 oracle's own iterate moves under two changes that only
reorder or perturb rounding (every matrix-vector product perturbed by one ulp
in a seeded direction; every inner product summed in reverse order) and
checks each bound below against that spread: the bound must leave a margin
of at least 3x over the spread and may not exceed 30x of it (or 1e-8,
whichever is larger).  ``tests/test_gpu_headline_parity.py`` compares the
GPU iterate with the oracle's under the same bounds.

Each case: (id, ndim, n, gamma, method, s, k_or_m, blocks, basis, rhs, bound)
rhs "xt": f = A x_true (x_true seeded U(-1, 1), seed 0); "cos": f_p =
cos(0.37 p) + 0.1, a smooth right-hand side that makes the first block's
columns nearly dependent.  basis 0 monomial, 1 Chebyshev, 2 Newton.
"""

# measured spreads (max of the two rounding changes), 128^3 gamma = 50:
#   monomial s=8, m=40, 2 blocks 2.7e-5, 4 blocks 3.2e-5
#   monomial s=8, m=2, 4 blocks (two restart cycles) 1.9e-6
#   Chebyshev / Newton s=8, m=40, 4 blocks, rhs xt: 4e-14 / 6e-14
#   Newton s=8, m=2, 2 blocks, rhs cos: 3.5e-7
CASES = [
    ("3d128-mono-s8m40-b2", 3, 128, 50.0, "gmres", 8, 40, 2, 0, "xt", 2e-4),
    ("3d128-mono-s8m40-b4", 3, 128, 50.0, "gmres", 8, 40, 4, 0, "xt", 2e-4),
    ("3d128-mono-s8m2-b4-2cycles", 3, 128, 50.0, "gmres", 8, 2, 4, 0, "xt", 1e-5),
    ("3d128-cheb-s8m40-b4", 3, 128, 50.0, "gmres", 8, 40, 4, 1, "xt", 1e-8),
    ("3d128-newton-s8m40-b4", 3, 128, 50.0, "gmres", 8, 40, 4, 2, "xt", 1e-8),
    ("3d128-newton-s8m2-b2-cos", 3, 128, 50.0, "gmres", 8, 2, 2, 2, "cos", 2e-6),
]

CONTRACT = 1e-8  # relative iterate bound wherever rounding allows it


def rhs(kind, prob, apply):
    import numpy as np
    if kind == "xt":
        return apply(prob.x_true())
    return np.cos(np.arange(prob.N) * 0.37) + 0.1
