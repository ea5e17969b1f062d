"""Pins of the FP64 CPU reference of the learned initial-guess network against
facts other than itself: a library correlation routine, the 1x1 special case,
the adjoint identities of a linear map, central finite differences and
closed forms of the Adam recursion."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn as R


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def dilated(k3, d):
    kd = np.zeros((2 * d + 1, 2 * d + 1))
    kd[::d, ::d] = k3
    return kd


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_fwd_matches_library_correlation(d):
    # a dilated 3x3 cross-correlation with zero padding = scipy's 'same'
    # correlation with the zero-stuffed (2d+1)^2 kernel, summed over inputs
    B, Cin, Cout, H, W = 2, 3, 2, 11, 13
    x, w, b = rnd((B, Cin, H, W), 1), rnd((Cout, Cin, 3, 3), 2), rnd(Cout, 3)
    y = R.conv_fwd(x, w, b, d)
    for bb in range(B):
        for co in range(Cout):
            ref = b[co] + sum(correlate2d(x[bb, ci], dilated(w[co, ci], d), mode="same")
                              for ci in range(Cin))
            np.testing.assert_allclose(y[bb, co], ref, rtol=1e-12, atol=1e-12)


def test_fwd_centre_tap_is_channel_matmul():
    B, Cin, Cout, H, W = 2, 5, 4, 7, 6
    x, b = rnd((B, Cin, H, W), 4), rnd(Cout, 5)
    w = np.zeros((Cout, Cin, 3, 3))
    w[:, :, 1, 1] = rnd((Cout, Cin), 6)
    y = R.conv_fwd(x, w, b, 3)
    ref = np.einsum("oc,bchw->bohw", w[:, :, 1, 1], x) + b[None, :, None, None]
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_fwd_single_off_centre_tap_is_shift():
    # only tap (ty, tx) = (0, 2) set: y(i, j) = x(i - d, j + d), zero outside
    d, H, W = 2, 9, 8
    x = rnd((1, 1, H, W), 7)
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 0, 2] = 1.0
    y = R.conv_fwd(x, w, None, d)[0, 0]
    ref = np.zeros((H, W))
    ref[d:, :W - d] = x[0, 0, :H - d, d:]
    np.testing.assert_array_equal(y, ref)


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_bwd_data_is_adjoint(d):
    B, Cin, Cout, H, W = 2, 3, 4, 10, 12
    x, w, g = rnd((B, Cin, H, W), 8), rnd((Cout, Cin, 3, 3), 9), rnd((B, Cout, H, W), 10)
    lhs = np.sum(R.conv_fwd(x, w, None, d) * g)
    rhs = np.sum(x * R.conv_bwd_data(g, w, d))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_bwd_weight_is_gradient_of_bilinear_form(d):
    # <conv(x, v), g> is linear in v, so it equals <dW(x, g), v>; db = sum g
    B, Cin, Cout, H, W = 2, 3, 4, 10, 9
    x, v, g = rnd((B, Cin, H, W), 11), rnd((Cout, Cin, 3, 3), 12), rnd((B, Cout, H, W), 13)
    dw, db = R.conv_bwd_weight(x, g, d)
    lhs = np.sum(R.conv_fwd(x, v, None, d) * g)
    assert abs(lhs - np.sum(dw * v)) <= 1e-12 * max(1.0, abs(lhs))
    np.testing.assert_allclose(db, g.sum(axis=(0, 2, 3)), rtol=1e-12)


def test_param_layout_size():
    # 2*32*9+32 + 2*(32*32*9+32) + 32*9+1
    assert R.param_count() == 19393
    p = np.arange(R.param_count(), dtype=float)
    np.testing.assert_array_equal(R.pack(R.unpack(p)), p)


def small_net_case(seed=0, B=2, H=12, W=14):
    rng = np.random.default_rng(seed)
    params = np.concatenate([
        np.concatenate([rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci)),
                        0.1 * rng.standard_normal(co)])
        for co, ci, _ in R.layer_shapes()])
    logk = rng.standard_normal((B, H, W))
    f = rng.standard_normal((B, H, W)) * 3.0
    t = rng.standard_normal((B, H, W))
    return params, logk, f, t


def test_network_gradient_matches_central_differences():
    params, logk, f, t = small_net_case()
    _, grad = R.loss_and_grad(params, logk, f, t)
    rng = np.random.default_rng(1)
    # entries from every weight block and every bias block
    idx, o = [], 0
    for co, ci, _ in R.layer_shapes():
        idx += list(o + rng.choice(co * ci * 9, 6, replace=False))
        o += co * ci * 9
        idx += list(o + rng.choice(co, min(co, 2), replace=False))
        o += co
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_and_grad(pp, logk, f, t)[0] - R.loss_and_grad(pm, logk, f, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(grad[i])), (i, fd, grad[i])


def test_input_scaling_equivariance():
    # x0 depends on f only through f / rms(f), rescaled by rms(f): x0(c f) = c x0(f)
    params, logk, f, _ = small_net_case(3)
    x1 = R.predict_x0(params, 0.7, logk, f)
    x2 = R.predict_x0(params, 0.7, logk, 5.0 * f)
    np.testing.assert_allclose(x2, 5.0 * x1, rtol=1e-12, atol=1e-14)


def test_loss_zero_at_own_output():
    params, logk, f, _ = small_net_case(4)
    out, _, _ = R.forward(params, logk, f)
    loss, grad = R.loss_and_grad(params, logk, f, out)
    assert loss == 0.0 and np.all(grad == 0.0)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are g and g^2 at
    # every step, so each step moves by lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, 0.0, -7.0])
    p0 = np.array([1.0, 2.0, -1.0, 0.5, 0.0])
    p, m, v = p0.copy(), np.zeros(5), np.zeros(5)
    T, lr, eps = 7, 1e-2, 1e-8
    for t in range(1, T + 1):
        p, m, v = R.adam_step(p, m, v, g, t, lr=lr, eps=eps)
    np.testing.assert_allclose(p, p0 - T * lr * g / (np.abs(g) + eps), rtol=1e-13, atol=1e-15)


def test_adam_two_steps_closed_form():
    # after gradients g1, g2: mhat = (b1 g1 + g2)/(1 + b1), vhat = (b2 g1^2 + g2^2)/(1 + b2)
    b1, b2, lr, eps = 0.9, 0.999, 1e-3, 1e-8
    g1, g2 = np.array([1.0, -2.0, 0.5]), np.array([-3.0, 0.25, 0.5])
    p0 = np.array([0.1, 0.2, 0.3])
    p, m, v = R.adam_step(p0, np.zeros(3), np.zeros(3), g1, 1, lr, b1, b2, eps)
    p1 = p0 - lr * g1 / (np.abs(g1) + eps)
    np.testing.assert_allclose(p, p1, rtol=1e-14)
    p, m, v = R.adam_step(p, m, v, g2, 2, lr, b1, b2, eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    np.testing.assert_allclose(p, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-13)


# ---------------------------------------------------------------------------
# coarse-grid guess: block averages, bilinear interpolation, Jacobi sweeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("factor", [1, 2, 4, 8])
def test_pool_is_block_mean(factor):
    # against numpy's reshape-and-mean of the same blocks
    B, ny, nx = 2, 8 * 3, 8 * 5
    x = rnd((B, ny, nx), 11)
    ref = x.reshape(B, ny // factor, factor, nx // factor, factor).mean(axis=(2, 4))
    np.testing.assert_allclose(R.pool(x, factor), ref, rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(R.pool(np.full((ny, nx), 2.5), factor), 2.5)


@pytest.mark.parametrize("factor", [2, 4, 8])
def test_upsample_matches_library_bilinear(factor):
    # torch's bilinear interpolation with half-cell centres (align_corners
    # False) is the same map, written independently
    torch = pytest.importorskip("torch")
    xc = rnd((5, 7), 12)
    ref = torch.nn.functional.interpolate(torch.tensor(xc)[None, None], scale_factor=factor,
                                          mode="bilinear", align_corners=False)[0, 0].numpy()
    np.testing.assert_allclose(R.upsample(xc, factor), ref, rtol=1e-13, atol=1e-14)


def test_upsample_reproduces_affine_fields_inside():
    # at fine points whose two coarse neighbours lie inside the coarse grid the
    # interpolant of an affine field is the field itself
    factor, nyc, nxc = 4, 6, 9
    J, I = np.meshgrid(np.arange(nyc), np.arange(nxc), indexing="ij")
    xc = 0.3 + 1.7 * I - 0.9 * J
    x = R.upsample(xc, factor)
    u = (np.arange(nxc * factor) + 0.5) / factor - 0.5
    w = (np.arange(nyc * factor) + 0.5) / factor - 0.5
    inside_x = (u >= 0) & (u <= nxc - 1)
    inside_y = (w >= 0) & (w <= nyc - 1)
    ref = 0.3 + 1.7 * u[None, :] - 0.9 * w[:, None]
    m = inside_y[:, None] & inside_x[None, :]
    np.testing.assert_allclose(x[m], ref[m], rtol=1e-13, atol=1e-13)
    # constants everywhere, the edges included
    np.testing.assert_allclose(R.upsample(np.full((nyc, nxc), -1.25), factor), -1.25, rtol=0, atol=0)


def _diffusion_operator(n, seed):
    import oracle as O
    from paper_2001_04886_amd import problems as P
    logk = P.grf(n, 0.2, seed=seed)
    return O.Operator(2, n, n, coef=P.diffusion_coef(logk)), logk


def test_jacobi_sweep_matches_dense_formula():
    from helpers import dense
    A, _ = _diffusion_operator(6, 3)
    M = dense(A)
    f, x = rnd(36, 13), rnd(36, 14)
    ref = x + 0.8 * (f - M @ x) / np.diag(M)
    np.testing.assert_allclose(R.jacobi(A, f, x, 1), ref, rtol=1e-13, atol=1e-13)
    # the solution is a fixed point
    xs = np.linalg.solve(M, f)
    np.testing.assert_allclose(R.jacobi(A, f, xs, 5), xs, rtol=1e-10, atol=1e-12)


def test_coarse_guess_with_factor_one_is_the_fine_guess():
    # factor 1, no sweeps: the composition reduces to predict_x0 (with log k
    # rounded to float32 as the network input is stored)
    n = 12
    A, logk = _diffusion_operator(n, 4)
    f = rnd((n, n), 15)
    params = 0.1 * rnd(R.param_count(), 16)
    ref = R.predict_x0(params, 0.3, logk.astype(np.float32).astype(np.float64)[None], f[None])[0]
    np.testing.assert_allclose(R.predict_x0_coarse(params, 0.3, 1, 0, A, logk, f), ref.ravel(),
                               rtol=1e-13, atol=1e-13)
