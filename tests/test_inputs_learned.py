"""Inputs of the learned-initial-guess workload (CPU): the device-side
generators follow the same recipe as the numpy ones, and the grid symmetries
used to augment training data map solved systems to solved systems."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2001_04886_amd import problems as P
from paper_2001_04886_amd.learn import symmetry


def test_coef_torch_equals_numpy():
    lk = P.grf(24, 0.1, 3)
    np.testing.assert_array_equal(P.diffusion_coef_torch(torch.tensor(lk)).numpy(),
                                  P.diffusion_coef(lk))


def test_coef_constant_k_is_laplacian():
    n = 9
    c = P.diffusion_coef(np.zeros((n, n)))
    h2 = (1.0 / (n + 1)) ** 2
    np.testing.assert_allclose(c[0], 4.0 / h2)
    np.testing.assert_allclose(c[1:5], -1.0 / h2)
    assert np.all(c[5:] == 0.0)


def test_grf_torch_statistics():
    g = P.grf_batch_torch(64, 0.1, 5, 16, device="cpu").numpy()
    np.testing.assert_allclose(g.mean(axis=(1, 2)), 0.0, atol=1e-12)
    np.testing.assert_allclose(g.std(axis=(1, 2)), 1.0, rtol=1e-12)
    h = 1.0 / 65
    for lag in (1, 3, 6):
        c = np.mean(g[:, :, :-lag] * g[:, :, lag:])
        assert abs(c - np.exp(-(lag * h) ** 2 / (2 * 0.01))) < 0.08


def test_grf_torch_seeded():
    a = P.grf_batch_torch(32, 0.1, 9, 3, device="cpu")
    b = P.grf_batch_torch(32, 0.1, 9, 3, device="cpu")
    c = P.grf_batch_torch(32, 0.1, 10, 3, device="cpu")
    assert torch.equal(a, b) and not torch.equal(a, c)


@pytest.mark.parametrize("g", range(8))
def test_symmetry_maps_solutions_to_solutions(g):
    # A(R k) (R x) = R (A(k) x) for every grid symmetry R: the augmented
    # (R k, R f, R x) is as solved as the original
    n = 14
    lk = P.grf(n, 0.1, 21)
    x = P.grf(n, 0.1, 22)
    A = O.Operator(2, n, n, 1, np.zeros(7), coef=P.diffusion_coef(lk))
    f = O.apply(A, x.ravel()).reshape(n, n)
    lk_r, x_r, f_r = (symmetry(torch.tensor(t)[None], g)[0].numpy() for t in (lk, x, f))
    A_r = O.Operator(2, n, n, 1, np.zeros(7), coef=P.diffusion_coef(lk_r))
    np.testing.assert_allclose(O.apply(A_r, x_r.ravel()).reshape(n, n), f_r,
                               rtol=1e-12, atol=1e-12 * np.abs(f).max())


def test_symmetry_group_is_distinct():
    t = torch.arange(16.0).reshape(1, 4, 4)
    images = {tuple(symmetry(t, g).ravel().tolist()) for g in range(8)}
    assert len(images) == 8
