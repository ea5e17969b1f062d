"""Plain FP64 CPU reference of the learned initial-guess network.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this module; it never
imports the GPU library.

The paper's restarted s-step GMRES (Alg 4.2) starts from an arbitrary x0.  The
network that proposes x0 is an extension beyond the paper; its definition is
fixed here, independently of the GPU code:

* input: two channels per grid point, ``log k`` and ``f / rms(f)``
  (rms over the grid of one sample);
* four dilated 3x3 convolutions, channels 2 -> 32 -> 32 -> 32 -> 1,
  dilations 1, 2, 4, 8, zero padding equal to the dilation, ReLU after the
  first three;
* output ``x0 = out * rms(f) * out_scale`` (``out_scale`` is a constant of the
  trained model);
* loss: mean squared difference between ``out`` and the target
  ``x / (rms(f) * out_scale)`` over every point of the batch;
* optimiser: Adam with bias correction.

Parameters are one flat vector, layer by layer: ``W_l`` as
``[Cout][Cin][3][3]`` followed by ``b_l`` as ``[Cout]``.

The convolution loops are in ``cnn_oracle.c`` (direct loops, FP64); the
composition below is plain numpy in FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

CHANNELS = (2, 32, 32, 32, 1)
DILATIONS = (1, 2, 4, 8)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cnn_oracle.c")
_LIB = os.environ.get("SSTEP_CNN_ORACLE_LIB") or os.path.join(_HERE, "libcnn_oracle.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if "SSTEP_CNN_ORACLE_LIB" not in os.environ and (
            not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build()
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    i = C.c_int
    lib.cnn_conv_fwd.restype = None
    lib.cnn_conv_fwd.argtypes = [dp, i, i, i, i, dp, dp, i, i, dp]
    lib.cnn_conv_bwd_data.restype = None
    lib.cnn_conv_bwd_data.argtypes = [dp, i, i, i, i, dp, i, i, dp]
    lib.cnn_conv_bwd_weight.restype = None
    lib.cnn_conv_bwd_weight.argtypes = [dp, dp, i, i, i, i, i, i, dp, dp]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def conv_fwd(x, w, bias, d):
    """x [B][Cin][H][W], w [Cout][Cin][3][3], bias [Cout] or None."""
    x = _c64(x)
    w = _c64(w)
    B, Cin, H, W = x.shape
    Cout = w.shape[0]
    assert w.shape == (Cout, Cin, 3, 3)
    y = np.empty((B, Cout, H, W))
    b = _c64(bias) if bias is not None else None
    _load().cnn_conv_fwd(_dp(x), B, Cin, H, W, _dp(w), _dp(b) if b is not None else None,
                         Cout, int(d), _dp(y))
    return y


def conv_bwd_data(dy, w, d):
    dy = _c64(dy)
    w = _c64(w)
    B, Cout, H, W = dy.shape
    Cin = w.shape[1]
    dx = np.empty((B, Cin, H, W))
    _load().cnn_conv_bwd_data(_dp(dy), B, Cout, H, W, _dp(w), Cin, int(d), _dp(dx))
    return dx


def conv_bwd_weight(x, dy, d):
    x = _c64(x)
    dy = _c64(dy)
    B, Cin, H, W = x.shape
    Cout = dy.shape[1]
    dw = np.empty((Cout, Cin, 3, 3))
    db = np.empty(Cout)
    _load().cnn_conv_bwd_weight(_dp(x), _dp(dy), B, Cin, Cout, H, W, int(d), _dp(dw), _dp(db))
    return dw, db


def layer_shapes():
    """[(Cout, Cin, dilation)] for the four layers."""
    return [(CHANNELS[l + 1], CHANNELS[l], DILATIONS[l]) for l in range(4)]


def param_count() -> int:
    return sum(co * ci * 9 + co for co, ci, _ in layer_shapes())


def unpack(params):
    """Flat parameter vector -> [(W_l, b_l)]."""
    params = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for co, ci, _ in layer_shapes():
        w = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out.append((w, b))
    assert o == params.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def rms(f):
    """Per-sample root mean square over the grid; f [B][H][W]."""
    f = np.asarray(f, dtype=np.float64)
    return np.sqrt(np.mean(f.reshape(f.shape[0], -1) ** 2, axis=1))


def forward(params, logk, f):
    """Returns (out [B][H][W], activations [a0..a4] in NCHW, rms(f) [B])."""
    logk = np.asarray(logk, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    fr = rms(f)
    a = np.stack([logk, f / fr[:, None, None]], axis=1)
    acts = [a]
    for l, ((w, b), (_, _, d)) in enumerate(zip(unpack(params), layer_shapes())):
        z = conv_fwd(a, w, b, d)
        a = np.maximum(z, 0.0) if l < 3 else z
        acts.append(a)
    return a[:, 0], acts, fr


def predict_x0(params, out_scale, logk, f):
    out, _, fr = forward(params, logk, f)
    return out * (fr * out_scale)[:, None, None]


# Coarse-grid guess -----------------------------------------------------------
#
# The network above sees 31 points in each direction.  For the coarse-grid
# guess it runs on block averages of the inputs (factor x factor cells), and
# its guess is carried back to the fine grid by bilinear interpolation and
# smoothed by damped Jacobi sweeps with the fine-grid operator.

def pool(x, factor):
    """Block averages: x [B][ny][nx] (or [ny][nx]) -> [B][ny/factor][nx/factor];
    entry (J, I) is the mean of the factor x factor block with corner
    (factor J, factor I)."""
    x = np.asarray(x, dtype=np.float64)
    two_d = x.ndim == 2
    if two_d:
        x = x[None]
    B, ny, nx = x.shape
    out = np.zeros((B, ny // factor, nx // factor))
    for J in range(ny // factor):
        for I in range(nx // factor):
            blk = x[:, J * factor:(J + 1) * factor, I * factor:(I + 1) * factor]
            out[:, J, I] = blk.sum(axis=(1, 2)) / (factor * factor)
    return out[0] if two_d else out


def upsample(xc, factor):
    """Bilinear interpolation of the coarse field xc [nyc][nxc], whose values
    sit at the centres of factor x factor blocks, onto the fine grid: fine
    index i sits at coarse coordinate (i + 1/2)/factor - 1/2; the two coarse
    neighbours used are clamped into the coarse grid."""
    xc = np.asarray(xc, dtype=np.float64)
    nyc, nxc = xc.shape

    def axis(nc):
        u = (np.arange(nc * factor) + 0.5) / factor - 0.5
        lo = np.floor(u)
        t = u - lo
        lo = lo.astype(np.int64)
        return np.clip(lo, 0, nc - 1), np.clip(lo + 1, 0, nc - 1), t

    ia, ib, tx = axis(nxc)
    ja, jb, ty = axis(nyc)
    rows_a = (1.0 - tx)[None, :] * xc[ja][:, ia] + tx[None, :] * xc[ja][:, ib]
    rows_b = (1.0 - tx)[None, :] * xc[jb][:, ia] + tx[None, :] * xc[jb][:, ib]
    return (1.0 - ty)[:, None] * rows_a + ty[:, None] * rows_b


def jacobi(A, f, x, sweeps, omega=0.8):
    """Damped Jacobi sweeps x <- x + omega (f - A x) / diag(A) on the oracle
    operator A (flat vectors)."""
    import oracle as O
    d = A.coef[0] if A.coef is not None else np.full(A.N, A.c[0])
    x = np.array(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    for _ in range(sweeps):
        x = x + omega * (f - O.apply(A, x)) / d
    return x


def predict_x0_coarse(params, out_scale, factor, sweeps, A, logk, f):
    """Coarse-grid guess for one [ny][nx] sample (flat result): block-averaged
    log k (stored in float32, as the network input is) and f, the network's
    guess on the coarse grid, bilinear interpolation, Jacobi sweeps."""
    logk_c = pool(logk, factor).astype(np.float32).astype(np.float64)
    f_c = pool(f, factor)
    xc = predict_x0(params, out_scale, logk_c[None], f_c[None])[0]
    return jacobi(A, np.asarray(f, dtype=np.float64).ravel(), upsample(xc, factor).ravel(), sweeps)


def target(x, f, out_scale):
    """Normalised regression target x / (rms(f) * out_scale)."""
    return np.asarray(x, dtype=np.float64) / (rms(f) * out_scale)[:, None, None]


def loss_and_grad(params, logk, f, t):
    """Mean squared error of the network output against the normalised target
    t [B][H][W], and its gradient with respect to the flat parameters
    (reverse pass through the four layers, ReLU derivative 1 where the
    activation is positive)."""
    out, acts, _ = forward(params, logk, f)
    t = np.asarray(t, dtype=np.float64)
    nel = out.size
    err = out - t
    loss = float(np.sum(err * err) / nel)
    g = (2.0 / nel) * err[:, None]
    layers = unpack(params)
    grads = [None] * 4
    for l in range(3, -1, -1):
        w, _ = layers[l]
        d = DILATIONS[l]
        dw, db = conv_bwd_weight(acts[l], g, d)
        grads[l] = (dw, db)
        if l > 0:
            g = conv_bwd_data(g, w, d) * (acts[l] > 0.0)
    return loss, pack(grads)


def adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments) at step number ``step`` >= 1.
    Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
