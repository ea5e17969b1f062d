"""Seeded synthetic problem generators (inputs only; no solver arithmetic).

This module is shared by the tests, the benchmark and the oracle checks.  It
builds the *inputs* of a solve -- stencil coefficients of the discretised PDE,
seeded exact solutions, random fields, batched system tables -- and nothing
of the s-step methods themselves.  It imports neither the GPU binding nor the
oracle.

Problems
--------
* Convection-diffusion ``-Lap u + gamma * (u_x + u_y [+ u_z]) = f`` on the unit
  square / cube, Dirichlet 0, 5-point (2-D) or 7-point (3-D) centred
  differences on an ``n``-point-per-axis interior grid, ``h = 1/(n+1)``: the
  same discretisation as the paper's Sec. 5 (five-point Laplacian, central
  first derivatives) with constant coefficients.
* Variable-coefficient diffusion ``-div(k grad u) = f`` (harmonic-mean face
  coefficients) for the learned-initial-guess problem.
* The paper's own test problem (Sec. 5, eq. (9)): variable coefficients in
  conservative form, analytic solution, the paper's initial guess.
* Exact solutions ``x_true[p] = 2 U(seed, p) - 1`` with ``U`` the top 53 bits of
  SplitMix64 applied to the counter ``seed * 2**40 + p`` (a counter-based
  generator, so any slice can be produced independently on any device).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function of state ``z`` (Steele, Lea & Flood 2014):
    z += golden gamma, then two xor-shift-multiply rounds and a final xor-shift.
    Vectorised over a uint64 array; arithmetic wraps mod 2**64."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """U(seed, p) in [0, 1) for p = offset .. offset+n-1, 53-bit resolution."""
    ctr = np.uint64(seed) * np.uint64(1 << 40) + np.arange(offset, offset + n, dtype=np.uint64)
    return (splitmix64(ctr) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def x_true(seed: int, n: int) -> np.ndarray:
    """Seeded exact solution, entries uniform in [-1, 1)."""
    return 2.0 * uniform01(seed, n) - 1.0


def convdiff_coeffs(ndim: int, nx: int, ny: int, nz: int = 1, gamma: float = 0.0):
    """Seven stencil coefficients (centre, -x, +x, -y, +y, -z, +z) of
    -Lap u + gamma * sum_d du/dx_d with h_d = 1/(n_d + 1)."""
    ns = [nx, ny] + ([nz] if ndim == 3 else [])
    c = np.zeros(7)
    for d, n in enumerate(ns):
        h = 1.0 / (n + 1)
        c[0] += 2.0 / h**2
        c[1 + 2 * d] = -1.0 / h**2 - gamma / (2.0 * h)
        c[2 + 2 * d] = -1.0 / h**2 + gamma / (2.0 * h)
    return c


class Problem:
    """A stencil problem: grid, coefficients (constant ``c`` or per-point
    ``coef`` [7][N]), seeded exact solution."""

    def __init__(self, ndim, nx, ny, nz=1, c=None, coef=None, seed=0, name=""):
        self.ndim, self.nx, self.ny = int(ndim), int(nx), int(ny)
        self.nz = int(nz) if ndim == 3 else 1
        self.c = np.zeros(7) if c is None else np.asarray(c, dtype=np.float64)
        self.coef = coef
        self.seed = seed
        self.name = name

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def x_true(self) -> np.ndarray:
        return x_true(self.seed, self.N)


def convdiff(ndim: int, n: int, gamma: float, seed: int = 0, ny: int | None = None,
             nz: int | None = None) -> Problem:
    ny = n if ny is None else ny
    nz = (n if nz is None else nz) if ndim == 3 else 1
    return Problem(ndim, n, ny, nz, c=convdiff_coeffs(ndim, n, ny, nz, gamma), seed=seed,
                   name=f"convdiff{ndim}d_{n}_g{gamma:g}")


# Named workloads -----------------------------------------------------------

def small_2d(seed: int = 0) -> Problem:
    """64 x 64 interior grid, gamma = 10 (N = 4096)."""
    return convdiff(2, 64, 10.0, seed)


def cube_3d(n: int = 256, seed: int = 0, gamma: float = 50.0) -> Problem:
    """n^3 interior grid, 7-point, gamma = 50 (n = 256: N = 16 777 216)."""
    return convdiff(3, n, gamma, seed)


def square_2d_large(n: int = 4096, seed: int = 0, gamma: float = 50.0) -> Problem:
    """n^2 interior grid, 5-point, gamma = 50 (n = 4096: N = 16 777 216)."""
    return convdiff(2, n, gamma, seed)


def batched_table(nsys: int = 512, master_seed: int = 0, nmin: int = 32, nmax: int = 512,
                  gmax: float = 100.0):
    """Per-system (side length n ~ U{nmin..nmax}, gamma ~ U(0, gmax), seed) for
    a batch of independent 2-D convection-diffusion systems, all drawn from the
    counter-based generator with ``master_seed``."""
    u = uniform01(master_seed + 7919, 2 * nsys)
    ns = nmin + np.minimum((u[:nsys] * (nmax - nmin + 1)).astype(np.int64), nmax - nmin)
    gammas = u[nsys:] * gmax
    return [(int(ns[i]), float(gammas[i]), int(master_seed * 100003 + i + 1)) for i in range(nsys)]


# The paper's test problem (Sec. 5, eq. (9)) ----------------------------------
#
#   -(b u_x)_x - (c u_y)_y + (d u)_x + (e u)_y + f u = g  on (0,1)^2, u = 0 on
#   the boundary, b = exp(-xy), c = exp(xy), d = beta (x+y), e = gamma (x+y),
#   f = 1/(1+xy), beta = 1, gamma = 50, with g built from the analytic solution
#   u = x exp(xy) sin(pi x) sin(pi y) (the printed test function repeats
#   sin(pi y); the first factor is read as sin(pi x), which vanishes on the
#   whole boundary as the Dirichlet condition needs).

PAPER_BETA, PAPER_GAMMA = 1.0, 50.0


def _grid2(n: int):
    """Interior points of the unit square, h = 1/(n+1): arrays X, Y of shape
    [n][n] indexed [j][i] (x fastest when flattened, point p = i + n j)."""
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(t, t)
    return X, Y, h


def conservative_coef(n: int, b, c, d, e, f) -> np.ndarray:
    """Per-point [7][N] stencil (centre, -x, +x, -y, +y; 0, 0) on the n x n
    interior grid of -(b u_x)_x - (c u_y)_y + (d u)_x + (e u)_y + f u: the
    diffusion terms as five-point conservative differences with b, c at the
    cell faces (x +- h/2, y +- h/2), the first-order terms as central
    differences of the products d u, e u (d, e at the neighbouring points), f at
    the point.  b..f are functions of (x, y) arrays.  Entries of neighbours
    outside the grid are 0 (Dirichlet 0)."""
    X, Y, h = _grid2(n)

    def ev(fn, x, y):
        return np.broadcast_to(np.asarray(fn(x, y), dtype=np.float64), x.shape)

    h2 = h * h
    bw, be = ev(b, X - h / 2, Y), ev(b, X + h / 2, Y)
    cs, cn = ev(c, X, Y - h / 2), ev(c, X, Y + h / 2)
    west = -bw / h2 - ev(d, X - h, Y) / (2 * h)
    east = -be / h2 + ev(d, X + h, Y) / (2 * h)
    south = -cs / h2 - ev(e, X, Y - h) / (2 * h)
    north = -cn / h2 + ev(e, X, Y + h) / (2 * h)
    west[:, 0] = 0.0
    east[:, -1] = 0.0
    south[0, :] = 0.0
    north[-1, :] = 0.0
    coef = np.zeros((7, n * n))
    coef[0] = ((bw + be + cs + cn) / h2 + ev(f, X, Y)).ravel()
    coef[1], coef[2], coef[3], coef[4] = west.ravel(), east.ravel(), south.ravel(), north.ravel()
    return coef


def paper_functions(beta: float = PAPER_BETA, gamma: float = PAPER_GAMMA):
    """Coefficient functions (b, c, d, e, f) of eq. (9)."""
    return (lambda x, y: np.exp(-x * y), lambda x, y: np.exp(x * y),
            lambda x, y: beta * (x + y), lambda x, y: gamma * (x + y),
            lambda x, y: 1.0 / (1.0 + x * y))


def paper_exact(n: int) -> np.ndarray:
    """u = x exp(xy) sin(pi x) sin(pi y) at the interior grid points."""
    X, Y, _ = _grid2(n)
    return (X * np.exp(X * Y) * np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()


def paper_rhs(n: int, beta: float = PAPER_BETA, gamma: float = PAPER_GAMMA) -> np.ndarray:
    """g = L u of eq. (9) for the analytic u, at the interior grid points.
    With E = exp(xy), sx = sin(pi x), cx = cos(pi x) (sy, cy alike):
      u    = x E sx sy
      u_x  = E sy ((1 + xy) sx + pi x cx)
      u_xx = E sy ((y (2 + xy) - pi^2 x) sx + 2 pi (1 + xy) cx)
      u_y  = x E sx (x sy + pi cy)
      u_yy = x E sx ((x^2 - pi^2) sy + 2 pi x cy)
    and L u = -(b_x u_x + b u_xx) - (c_y u_y + c u_yy) + d_x u + d u_x
              + e_y u + e u_y + f u, with b_x = -y exp(-xy), c_y = x exp(xy),
    d_x = beta, e_y = gamma."""
    X, Y, _ = _grid2(n)
    pi = np.pi
    E = np.exp(X * Y)
    sx, cx, sy, cy = np.sin(pi * X), np.cos(pi * X), np.sin(pi * Y), np.cos(pi * Y)
    u = X * E * sx * sy
    ux = E * sy * ((1 + X * Y) * sx + pi * X * cx)
    uxx = E * sy * ((Y * (2 + X * Y) - pi**2 * X) * sx + 2 * pi * (1 + X * Y) * cx)
    uy = X * E * sx * (X * sy + pi * cy)
    uyy = X * E * sx * ((X**2 - pi**2) * sy + 2 * pi * X * cy)
    b, c = np.exp(-X * Y), E
    bx, cy_ = -Y * np.exp(-X * Y), X * E
    d, e = beta * (X + Y), gamma * (X + Y)
    f = 1.0 / (1.0 + X * Y)
    g = -(bx * ux + b * uxx) - (cy_ * uy + c * uyy) + beta * u + d * ux + gamma * u + e * uy + f * u
    return g.ravel()


def paper_x0(N: int) -> np.ndarray:
    """The paper's initial guess 0.05 * mod(i, 50) over the unknowns numbered
    from 1 (point p = 0, 1, ... holds 0.05 * ((p + 1) mod 50))."""
    return 0.05 * ((np.arange(N, dtype=np.int64) + 1) % 50)


def paper_problem(n: int, beta: float = PAPER_BETA, gamma: float = PAPER_GAMMA) -> Problem:
    """Eq. (9) on an n x n interior grid (variable coefficients [7][N])."""
    return Problem(2, n, n, coef=conservative_coef(n, *paper_functions(beta, gamma)),
                   name=f"paper_eq9_{n}_b{beta:g}_g{gamma:g}")


# Gaussian random fields ----------------------------------------------------

def grf(n: int, length: float, seed: int, pad: int = 2) -> np.ndarray:
    """Unit-variance Gaussian random field on an n x n grid of the unit square
    with covariance exp(-r^2 / (2 length^2)), by spectral synthesis on a
    (pad*n)^2 periodic grid cropped to n x n (the crop avoids wrap-around
    correlation).  Row index = y, column index = x."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = pad * n
    h = 1.0 / (n + 1)
    k = np.fft.fftfreq(m, d=h) * 2.0 * np.pi
    kx, ky = np.meshgrid(k, k, indexing="xy")
    # spectral density of the squared-exponential covariance (2-D)
    spec = np.exp(-0.5 * (kx**2 + ky**2) * length**2)
    noise = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    field = np.fft.ifft2(noise * np.sqrt(spec)).real
    field = field[:n, :n]
    field = (field - field.mean()) / field.std()
    return np.ascontiguousarray(field)


def diffusion_coef(logk: np.ndarray) -> np.ndarray:
    """Per-point [7][N] stencil of -div(k grad u) on an n x n grid, h = 1/(n+1),
    with harmonic-mean face coefficients k_{i+1/2} = 2 k_i k_{i+1}/(k_i + k_{i+1});
    faces on the boundary use the cell's own k (Dirichlet 0 outside)."""
    ny, nx = logk.shape
    k = np.exp(logk)
    h2 = (1.0 / (nx + 1)) ** 2

    def hm(a, b):
        return 2.0 * a * b / (a + b)

    kw = np.empty_like(k); ke = np.empty_like(k); ks = np.empty_like(k); kn = np.empty_like(k)
    kw[:, 1:] = hm(k[:, 1:], k[:, :-1]); kw[:, 0] = k[:, 0]
    ke[:, :-1] = hm(k[:, :-1], k[:, 1:]); ke[:, -1] = k[:, -1]
    ks[1:, :] = hm(k[1:, :], k[:-1, :]); ks[0, :] = k[0, :]
    kn[:-1, :] = hm(k[:-1, :], k[1:, :]); kn[-1, :] = k[-1, :]
    coef = np.zeros((7, nx * ny))
    coef[0] = ((kw + ke + ks + kn) / h2).ravel()
    coef[1] = (-kw / h2).ravel()
    coef[2] = (-ke / h2).ravel()
    coef[3] = (-ks / h2).ravel()
    coef[4] = (-kn / h2).ravel()
    return coef


# ---------------------------------------------------------------------------
# Device-side variants for the learned-initial-guess data (many 256^2 samples):
# the same field and stencil recipes as grf / diffusion_coef, built with torch
# on the GPU so that thousands of samples do not wait on host FFTs.  Noise
# comes from torch's seeded generator, so the fields differ from grf's (numpy
# PCG64) for the same seed; statistics and coefficients follow the same recipe.
# ---------------------------------------------------------------------------

def grf_batch_torch(n: int, length: float, seed: int, count: int, device="cuda", pad: int = 2):
    """count unit-variance squared-exponential Gaussian random fields on an
    n x n grid (spectral synthesis on a (pad*n)^2 periodic grid, cropped);
    float64 tensor [count][n][n], each normalised to mean 0, std 1."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    m = pad * n
    h = 1.0 / (n + 1)
    k = torch.fft.fftfreq(m, d=h, dtype=torch.float64, device=device) * 2.0 * np.pi
    ky, kx = torch.meshgrid(k, k, indexing="ij")
    amp = torch.exp(-0.25 * (kx ** 2 + ky ** 2) * length ** 2)  # sqrt of the spectral density
    out = torch.empty((count, n, n), dtype=torch.float64, device=device)
    chunk = 64
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        re = torch.randn((c1 - c0, m, m), generator=gen, dtype=torch.float64, device=device)
        im = torch.randn((c1 - c0, m, m), generator=gen, dtype=torch.float64, device=device)
        field = torch.fft.ifft2(torch.complex(re, im) * amp).real[:, :n, :n]
        mu = field.mean(dim=(1, 2), keepdim=True)
        sd = field.std(dim=(1, 2), keepdim=True, unbiased=False)
        out[c0:c1] = (field - mu) / sd
    return out


def diffusion_coef_torch(logk):
    """diffusion_coef for one torch field logk [n][n] (any device):
    [7][N] float64 tensor, same face rule and ordering."""
    import torch
    ny, nx = logk.shape
    k = torch.exp(logk.to(torch.float64))
    h2 = (1.0 / (nx + 1)) ** 2

    def hm(a, b):
        return 2.0 * a * b / (a + b)

    kw = torch.empty_like(k); ke = torch.empty_like(k); ks = torch.empty_like(k); kn = torch.empty_like(k)
    kw[:, 1:] = hm(k[:, 1:], k[:, :-1]); kw[:, 0] = k[:, 0]
    ke[:, :-1] = hm(k[:, :-1], k[:, 1:]); ke[:, -1] = k[:, -1]
    ks[1:, :] = hm(k[1:, :], k[:-1, :]); ks[0, :] = k[0, :]
    kn[:-1, :] = hm(k[:-1, :], k[1:, :]); kn[-1, :] = k[-1, :]
    coef = torch.zeros((7, nx * ny), dtype=torch.float64, device=logk.device)
    coef[0] = ((kw + ke + ks + kn) / h2).reshape(-1)
    coef[1] = (-kw / h2).reshape(-1)
    coef[2] = (-ke / h2).reshape(-1)
    coef[3] = (-ks / h2).reshape(-1)
    coef[4] = (-kn / h2).reshape(-1)
    return coef
