// batched.hip -- many independent s-step GMRES(m) solves (Sec. 4, Alg. 4.2)
// in one persistent launch.
//
// The grid holds as many workgroups as can be resident at once.  Each
// workgroup repeatedly takes the next system from a global queue (systems are
// ordered largest first) and runs the whole restarted s-step GMRES for it:
// matrix powers level by level, the Gram of the new block against the stored
// blocks, the block update, the block's own Gram, the FP64 Cholesky /
// Hessenberg / Givens work, the next start vector, the assembly of x and the
// true residual.  A workgroup only ever waits on its own barrier, so the launch
// cannot deadlock whatever the residency; every system solve is bounded by the
// block cap, so every workgroup reaches the end of the queue.
//
// The arithmetic per block is the same as in gmres.hip (normalised start
// vectors with their norms folded into coefficients, one-pass block CGS, a
// direct W_k, equilibrated Cholesky with rank truncation, L-scaled Givens QR).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "dense.hpp"
#include "launch.hpp"
#include "solvers.hpp"

namespace sstep {

struct BatchSys {
    StencilView A;
    const double* f;
    double* x;
    double* ws;        // this system's basis region: (m*s+1) columns of ld doubles
    long long ld;
    double sigma;
    int status, blocks, cycles, pad;
    double rel_resid;
    long long ticks[SSTEP_K_NCLASS];  // wall-clock ticks of the owning workgroup per class
};

// per-workgroup scratch for the small dense state (sized for m*s <= 512)
struct BatchSlot {
    double G[513 * 512];   // Hessenberg, column-major, ld = K+1
    double R[513 * 512];   // rotated L G
    double cs[513], sn[513], rhs[513], y[513];
    double T[512 * 17];    // projection coefficients [row][s+1]
    double C[512 * 16];    // Gram output
    GramFactor Wf[128];
    double nu[129], inv_nu[129];
};

struct BatchArgs {
    BatchSys* sys;
    const int* order;
    int nsys;
    int s, m;
    double tol;
    int max_blocks;
    double rank_tol, lucky_tol;
    BatchSlot* slots;
    int* queue;
};

template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    return t;
}

// Phase timer of the owning workgroup: thread 0 reads the constant-rate wall
// clock after the barrier that closes a phase and charges the interval to one
// kernel class (matrix powers, Gram, update, residual, scalar work, vector).
// The accumulators live in LDS (slot SSTEP_K_NCLASS holds the last reading).
struct PhaseClock {
    long long* acc;  // LDS [SSTEP_K_NCLASS + 1]
    __device__ void start() {
        if (threadIdx.x == 0) {
            for (int c = 0; c < SSTEP_K_NCLASS; ++c) acc[c] = 0;
            acc[SSTEP_K_NCLASS] = wall_clock64();
        }
    }
    __device__ void lap(int cls) {
        if (threadIdx.x == 0) {
            const long long t = wall_clock64();
            acc[cls] += t - acc[SSTEP_K_NCLASS];
            acc[SSTEP_K_NCLASS] = t;
        }
    }
};

typedef double d2v __attribute__((ext_vector_type(2)));
#define SSTEP_GLOBAL __attribute__((address_space(1)))
#define SSTEP_LDS __attribute__((address_space(3)))

// explicit address spaces: the basis, x and f live in global memory, the
// update coefficients in LDS (generic pointers would compile to flat accesses)
__device__ __forceinline__ d2v ld2(const double* p) { return *(const SSTEP_GLOBAL d2v*)p; }
__device__ __forceinline__ void st2(double* p, d2v v) { *(SSTEP_GLOBAL d2v*)p = v; }
__device__ __forceinline__ double ldg(const double* p) { return *(const SSTEP_GLOBAL double*)p; }
__device__ __forceinline__ double lds(const double* p) { return *(const SSTEP_LDS double*)p; }

// Grid coordinates of the points a thread visits (p = tid, tid + NT, ...),
// advanced without divisions.
struct Walker {
    int i, j, l, di, dj, dl, nx, ny;
    __device__ Walker(const StencilView& A, long long p0, int step) {
        nx = A.nx;
        ny = A.ny;
        const long long rest = p0 / nx;
        i = (int)(p0 - rest * nx);
        j = (int)(rest % ny);
        l = (int)(rest / ny);
        const int rows = step / nx;
        di = step - rows * nx;
        dj = rows % ny;
        dl = rows / ny;
    }
    __device__ __forceinline__ void next() {
        i += di;
        j += dj;
        l += dl;
        if (i >= nx) {
            i -= nx;
            ++j;
        }
        if (j >= ny) {
            j -= ny;
            ++l;
        }
    }
};

// One stencil pass over the workgroup's points: out = sc * (A in), or with f
// given r = f - A in into out; returns this thread's share of sum(out^2).
// Neighbours are summed in the order -x, +x, -y, +y, -z, +z, then the centre
// (outside the grid = Dirichlet 0).  The
// operator's scalars are copied to registers first (the descriptor sits in
// LDS), and constant / per-point coefficients get separate loops.
template <int NT>
__device__ double wg_stencil(const StencilView& Ad, const double* in, double* out, double sc,
                             const double* f) {
    const int nx = Ad.nx, ny = Ad.ny, nz = Ad.nz, ndim = Ad.ndim;
    const long long N = Ad.N, sy = nx, sz = (long long)nx * ny;
    const double* coef = Ad.coef;
    double c[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) c[q] = Ad.c[q];
    const SSTEP_GLOBAL double* gin = (const SSTEP_GLOBAL double*)in;
    SSTEP_GLOBAL double* gout = (SSTEP_GLOBAL double*)out;
    const SSTEP_GLOBAL double* gf = (const SSTEP_GLOBAL double*)f;
    const SSTEP_GLOBAL double* gc = (const SSTEP_GLOBAL double*)coef;
    StencilView geom;
    geom.nx = nx;
    geom.ny = ny;
    Walker w(geom, threadIdx.x, NT);
    double sq = 0.0;
    for (long long p = threadIdx.x; p < N; p += NT, w.next()) {
        double cc[7];
        if (coef) {
#pragma unroll
            for (int q = 0; q < 7; ++q) cc[q] = (q < 2 * ndim + 1) ? gc[q * N + p] : 0.0;
        } else {
#pragma unroll
            for (int q = 0; q < 7; ++q) cc[q] = c[q];
        }
        double acc = 0.0;
        if (w.i > 0) acc += cc[1] * gin[p - 1];
        if (w.i < nx - 1) acc += cc[2] * gin[p + 1];
        if (w.j > 0) acc += cc[3] * gin[p - sy];
        if (w.j < ny - 1) acc += cc[4] * gin[p + sy];
        if (ndim == 3) {
            if (w.l > 0) acc += cc[5] * gin[p - sz];
            if (w.l < nz - 1) acc += cc[6] * gin[p + sz];
        }
        acc += cc[0] * gin[p];
        const double v = f ? gf[p] - acc : sc * acc;
        gout[p] = v;
        sq += v * v;
    }
    return sq;
}

// Y[:, l] += sum_{c < nc} V[:, c] M[c * ldm + l] for l < nout <= NMAX (M in LDS);
// returns this thread's share of ||Y[:, 0]||^2 after the update when norm.
// Each thread owns point pairs (16-byte loads); eight columns of V are in
// flight per step; the sum over c runs in column order.  Lanes l >= nout
// compute on clamped (valid) columns and are never stored, so the loops have
// no data-dependent branches.
template <int NT, int NMAX>
__device__ double wg_lincomb(const double* V, long long ld, int nc, const double* M, int ldm,
                             double* Y, long long ldy, int nout, long long N, bool norm) {
    double nacc = 0.0;
    const long long np = N >> 1;
    int lc[NMAX];
#pragma unroll
    for (int l = 0; l < NMAX; ++l) lc[l] = l < nout ? l : nout - 1;
    for (long long q = threadIdx.x; q < np; q += NT) {
        const long long p = 2 * q;
        d2v a[NMAX];
#pragma unroll
        for (int l = 0; l < NMAX; ++l) a[l] = ld2(Y + lc[l] * ldy + p);
        int c = 0;
        for (; c + 8 <= nc; c += 8) {
            d2v v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = ld2(V + (long long)(c + u) * ld + p);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int l = 0; l < NMAX; ++l) {
                    const double mm = lds(M + (c + u) * ldm + lc[l]);
                    a[l].x = fma(v[u].x, mm, a[l].x);
                    a[l].y = fma(v[u].y, mm, a[l].y);
                }
        }
        for (; c < nc; ++c) {
            const d2v v = ld2(V + (long long)c * ld + p);
#pragma unroll
            for (int l = 0; l < NMAX; ++l) {
                const double mm = lds(M + c * ldm + lc[l]);
                a[l].x = fma(v.x, mm, a[l].x);
                a[l].y = fma(v.y, mm, a[l].y);
            }
        }
#pragma unroll
        for (int l = 0; l < NMAX; ++l)
            if (l < nout) st2(Y + l * ldy + p, a[l]);
        if (norm) nacc += a[0].x * a[0].x + a[0].y * a[0].y;
    }
    if ((N & 1) && threadIdx.x == 0) {
        const long long p = N - 1;
        double a[NMAX];
#pragma unroll
        for (int l = 0; l < NMAX; ++l) a[l] = ldg(Y + lc[l] * ldy + p);
        for (int c = 0; c < nc; ++c) {
            const double v = ldg(V + (long long)c * ld + p);
#pragma unroll
            for (int l = 0; l < NMAX; ++l) a[l] = fma(v, lds(M + c * ldm + lc[l]), a[l]);
        }
#pragma unroll
        for (int l = 0; l < NMAX; ++l)
            if (l < nout) *(SSTEP_GLOBAL double*)(Y + l * ldy + p) = a[l];
        if (norm) nacc += a[0] * a[0];
    }
    return nacc;
}

// out[a * nz + j] = sum_p X[:, a][p] Z[:, j][p] (a < ncx, j < nz <= KZ): tiles of
// CA columns of X against all of Z, point pairs per thread, one workgroup
// reduction per tile.  Columns past ncx / nz are clamped to valid ones and
// their sums dropped.
template <int NT, int CA, int KZ>
__device__ void wg_gram(const double* X, long long ldx, int ncx, const double* Z, long long ldz,
                        int nz, long long N, double* out /* [ncx][nz] */, double* red) {
    const long long np = N >> 1;
    const double* zc[KZ];
#pragma unroll
    for (int j = 0; j < KZ; ++j) zc[j] = Z + (long long)(j < nz ? j : nz - 1) * ldz;
    for (int c0 = 0; c0 < ncx; c0 += CA) {
        const double* xc[CA];
#pragma unroll
        for (int a = 0; a < CA; ++a) xc[a] = X + (long long)(c0 + a < ncx ? c0 + a : ncx - 1) * ldx;
        double acc[CA][KZ];
#pragma unroll
        for (int a = 0; a < CA; ++a)
#pragma unroll
            for (int j = 0; j < KZ; ++j) acc[a][j] = 0.0;
        for (long long q = threadIdx.x; q < np; q += NT) {
            const long long p = 2 * q;
            d2v z[KZ], x[CA];
#pragma unroll
            for (int j = 0; j < KZ; ++j) z[j] = ld2(zc[j] + p);
#pragma unroll
            for (int a = 0; a < CA; ++a) x[a] = ld2(xc[a] + p);
#pragma unroll
            for (int a = 0; a < CA; ++a)
#pragma unroll
                for (int j = 0; j < KZ; ++j)
                    acc[a][j] = fma(x[a].y, z[j].y, fma(x[a].x, z[j].x, acc[a][j]));
        }
        if ((N & 1) && threadIdx.x == 0) {
            const long long p = N - 1;
#pragma unroll
            for (int a = 0; a < CA; ++a) {
                const double xv = ldg(xc[a] + p);
#pragma unroll
                for (int j = 0; j < KZ; ++j) acc[a][j] = fma(xv, ldg(zc[j] + p), acc[a][j]);
            }
        }
        // workgroup reduction of the CA*KZ sums (wave shuffles, then LDS)
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < CA; ++a)
#pragma unroll
            for (int j = 0; j < KZ; ++j) {
                const double t = wave_sum(acc[a][j]);
                if (lane == 0) red[wave * CA * KZ + a * KZ + j] = t;
            }
        __syncthreads();
        for (int k = threadIdx.x; k < CA * KZ; k += NT) {
            const int a = k / KZ, j = k % KZ;
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += red[w * CA * KZ + k];
            if (c0 + a < ncx && j < nz) out[(c0 + a) * nz + j] = t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// one-thread FP64 scalar steps (kept out of line so that their registers do
// not weigh on the streaming loops)
// ---------------------------------------------------------------------------

// Scalar1 of block kb: equilibrated Cholesky of W_k (from the block's own
// Gram in W.C, start column scaled by inv_nu) and g = W_k^{-1} V_k^T Yhat_s;
// sh[0..s) = g, sh[s..2s) = N4b coefficients, sh[2 kMaxS] = ||Yhat_s||^2.
__device__ __noinline__ void scalar_factor(BatchSlot& W, int kb, int s, double rank_tol,
                                           double* lw, GramFactor* lf, double* sh) {
    const int s1 = s + 1;
    const double d0 = W.inv_nu[kb];
    double* Wk = lw;
    for (int q = 0; q < s; ++q)
        for (int pp = 0; pp < s; ++pp)
            Wk[pp + q * kMaxS] = W.C[pp * s1 + q] * (pp == 0 ? d0 : 1.0) * (q == 0 ? d0 : 1.0);
    gram_factor(Wk, kMaxS, s, rank_tol, lf);
    const int q = lf->rank;
    double* g = sh;
    double* h = sh + 2 * kMaxS + 4;
    if (q == s) {
        for (int pp = 0; pp < s; ++pp) h[pp] = W.C[pp * s1 + s] * (pp == 0 ? d0 : 1.0);
        gram_solve(*lf, h, g);
        for (int pp = 0; pp < s; ++pp) sh[s + pp] = -g[pp] * (pp == 0 ? d0 : 1.0);
    } else if (q > 0) {
        for (int pp = 0; pp < q; ++pp) h[pp] = Wk[pp + q * kMaxS];
        gram_solve_leading(*lf, q, h, g);
    }
    sh[2 * kMaxS] = W.C[s * s1 + s];
}

// Givens rotations of the q new columns of the L-scaled Hessenberg (the
// earlier rotations were applied column-parallel already), the rotated rhs,
// the next start-vector norm and the residual estimate sh[2 kMaxS + 1].
__device__ __noinline__ void scalar_givens(BatchSlot& W, int kb, int c0, int q, int ldg, double nu,
                                           double* sh) {
    for (int j = 0; j < q; ++j) {
        double* col = W.R + (c0 + j) * ldg;
        for (int i = c0; i < c0 + j; ++i) {
            const double x0 = col[i], x1 = col[i + 1];
            col[i] = W.cs[i] * x0 + W.sn[i] * x1;
            col[i + 1] = -W.sn[i] * x0 + W.cs[i] * x1;
        }
        const int cj = c0 + j;
        const double x0 = col[cj], x1 = col[cj + 1];
        double cth = 1.0, sth = 0.0;
        if (x1 != 0.0) {
            const double hh = hypot(x0, x1);
            cth = x0 / hh;
            sth = x1 / hh;
        }
        W.cs[cj] = cth;
        W.sn[cj] = sth;
        col[cj] = cth * x0 + sth * x1;
        col[cj + 1] = 0.0;
        const double g0 = W.rhs[cj];
        W.rhs[cj + 1] = -sth * g0;
        W.rhs[cj] = cth * g0;
    }
    W.nu[kb + 1] = nu;
    W.inv_nu[kb + 1] = nu > 0.0 ? 1.0 / nu : 0.0;
    sh[2 * kMaxS + 1] = fabs(W.rhs[c0 + q]);
}

// y = R^{-1} rhs (back substitution) and the assembly coefficients
// (start columns carry their 1/nu) into lm.
__device__ __noinline__ void scalar_ysolve(BatchSlot& W, int ncols, int s, int ldg, double* lm) {
    for (int i = ncols - 1; i >= 0; --i) {
        double v = W.rhs[i];
        for (int l = i + 1; l < ncols; ++l) v -= W.R[i + l * ldg] * W.y[l];
        W.y[i] = v / W.R[i + i * ldg];
    }
    for (int c = 0; c < ncols; ++c) lm[c] = W.y[c] * ((c % s == 0) ? W.inv_nu[c / s] : 1.0);
}

template <int NT, int CA, int KZ>
__device__ void solve_one(const BatchArgs& args, BatchSys& S, BatchSlot& W, double* red,
                          double* sh, double* lw, GramFactor* lf, double* lm,
                          const StencilView& A, long long* clk) {
    const int s = args.s, m = args.m, K = m * s, ldg = K + 1, s1 = s + 1;
    const long long N = A.N, ld = S.ld;
    double* V = S.ws;
    const int tid = threadIdx.x;
    // Basis change B (monomial): A Y[:,0:s] = Y B with B[j+1][j] = sigma
    const double sigma = S.sigma;

    PhaseClock pc{clk};
    pc.start();
    // ||f||
    double acc = 0.0;
    for (long long p = tid; p < N; p += NT) acc += S.f[p] * S.f[p];
    const double fnorm = sqrt(wg_sum<NT>(acc, red));
    pc.lap(SSTEP_K_VEC);
    const double tol_abs = args.tol * fnorm;
    int blocks = 0, cycles = 0, status = SSTEP_NOT_CONVERGED;
    double beta = 0.0;
    for (;;) {
        // r = f - A x into column 0, beta = ||r||
        acc = 0.0;
        acc = wg_stencil<NT>(A, S.x, V, 1.0, S.f);
        beta = sqrt(wg_sum<NT>(acc, red));
        pc.lap(SSTEP_K_RESID);
        if (!isfinite(beta)) { status = SSTEP_ERR_NONFINITE; break; }
        if (beta <= tol_abs) { status = SSTEP_OK; break; }
        if (blocks >= args.max_blocks) { status = SSTEP_NOT_CONVERGED; break; }
        ++cycles;
        for (int i = tid; i <= K; i += NT) W.rhs[i] = i == 0 ? beta : 0.0;
        if (tid == 0) {
            W.nu[0] = beta;
            W.inv_nu[0] = 1.0 / beta;
        }
        __syncthreads();
        int ncols = 0;
        bool err = false;
        for (int kb = 0; kb < m && blocks < args.max_blocks; ++kb) {
            const int c0 = kb * s;
            double* Yk = V + (long long)c0 * ld;
            // matrix powers: y_j = A y_{j-1} / sigma, y_0 = stored column * inv_nu
            for (int jl = 1; jl <= s; ++jl) {
                const double* in = Yk + (long long)(jl - 1) * ld;
                double* out = Yk + (long long)jl * ld;
                const double sc = (jl == 1 ? W.inv_nu[kb] : 1.0) / sigma;
                (void)wg_stencil<NT>(A, in, out, sc, nullptr);
                __syncthreads();
            }
            pc.lap(SSTEP_K_MPK);
            if (kb > 0) {
                // C = V_prev^T [y_1..y_s]
                wg_gram<NT, CA, KZ>(V, ld, c0, Yk + ld, ld, s, N, W.C, red);
                pc.lap(SSTEP_K_GRAM);
                // T_i = W_i^{-1} C_i, update coefficients
                for (int idx = tid; idx < kb * s; idx += NT) {
                    const int i = idx / s, l = idx % s + 1;
                    double c[kMaxS];
                    for (int q = 0; q < s; ++q)
                        c[q] = W.C[(i * s + q) * s + (l - 1)] * (q == 0 ? W.inv_nu[i] : 1.0);
                    gram_solve(W.Wf[i], c, c);
                    for (int q = 0; q < s; ++q) {
                        W.T[(i * s + q) * s1 + l] = c[q];
                        lm[(i * s + q) * s + (l - 1)] = -c[q] * (q == 0 ? W.inv_nu[i] : 1.0);
                        if (l == 1) W.T[(i * s + q) * s1] = 0.0;
                    }
                }
                __syncthreads();
                pc.lap(SSTEP_K_SCALAR);
                // y_j -= sum_c V_c coefM[c][j]  (coefficients in LDS)
                wg_lincomb<NT, KZ>(V, ld, c0, lm, s, Yk + ld, ld, s, N, false);
                __syncthreads();
                pc.lap(SSTEP_K_UPDATE);
            }
            // block Gram of [w_k, y_1..y_s]
            wg_gram<NT, CA, KZ + 1>(Yk, ld, s1, Yk, ld, s1, N, W.C, red);
            pc.lap(SSTEP_K_GRAM);
            // Scalar1: factor W_k in LDS (one thread), copy the factor out
            if (tid == 0) scalar_factor(W, kb, s, args.rank_tol, lw, lf, sh);
            __syncthreads();
            {
                const double* src = reinterpret_cast<const double*>(lf);
                double* dst = reinterpret_cast<double*>(&W.Wf[kb]);
                for (int i = tid; i < (int)(sizeof(GramFactor) / sizeof(double)); i += NT) dst[i] = src[i];
            }
            __syncthreads();
            pc.lap(SSTEP_K_SCALAR);
            const int q = W.Wf[kb].rank;
            if (q == 0) { err = true; break; }
            double nu = 0.0;
            if (q == s) {
                // w_hat = Yhat_s - V_k g, nu^2
                double* ys = Yk + (long long)s * ld;
                acc = wg_lincomb<NT, 1>(Yk, ld, s, sh + s, 1, ys, ld, 1, N, true);
                nu = sqrt(wg_sum<NT>(acc, red));
            }
            pc.lap(SSTEP_K_VEC);
            const bool lucky = (q == s) && !(nu > args.lucky_tol * sqrt(sh[2 * kMaxS]));
            // Hessenberg block column, rows 0..c0+q
            for (int idx = tid; idx < q * (c0 + q + 1); idx += NT) {
                const int j = idx / (c0 + q + 1), r = idx % (c0 + q + 1);
                double val = 0.0;
                // Z_k B[:, j] with B[j+1][j] = sigma: column l = j+1 of Z_k
                const int l = j + 1;
                double z;
                if (r < c0) z = W.T[r * s1 + l];
                else if (r < c0 + q) z = (l < q) ? (r - c0 == l ? 1.0 : 0.0) : sh[r - c0];
                else z = (l == q) ? nu : 0.0;
                val = sigma * z;
                if (r <= c0) {
                    for (int cp = (r > 0 ? r - 1 : 0); cp < c0; ++cp) {
                        const double t = W.T[cp * s1 + j];
                        if (t != 0.0) val -= W.G[r + cp * ldg] * t;
                    }
                }
                W.G[r + (c0 + j) * ldg] = val;
            }
            __syncthreads();
            for (int idx = tid; idx < q * (c0 + q + 1); idx += NT) {
                const int j = idx / (c0 + q + 1), r = idx % (c0 + q + 1);
                const double* gc = W.G + (c0 + j) * ldg;
                double val;
                if (r == c0 + q) {
                    val = gc[r];
                } else {
                    const int i = r / s, pp = r % s;
                    const int qi = (i < kb) ? s : q;
                    val = 0.0;
                    for (int b = pp; b < qi; ++b) val += gram_L(W.Wf[i], pp, b) * gc[i * s + b];
                }
                W.R[r + (c0 + j) * ldg] = val;
            }
            __syncthreads();
            if (tid < q) {
                double* col = W.R + (c0 + tid) * ldg;
                double x0 = col[0];
                for (int i = 0; i < c0; ++i) {
                    const double cth = W.cs[i], sth = W.sn[i], x1 = col[i + 1];
                    col[i] = cth * x0 + sth * x1;
                    x0 = -sth * x0 + cth * x1;
                }
                col[c0] = x0;
            }
            __syncthreads();
            if (tid == 0) scalar_givens(W, kb, c0, q, ldg, nu, sh);
            __syncthreads();
            pc.lap(SSTEP_K_SCALAR);
            ncols = c0 + q;
            ++blocks;
            const double est = sh[2 * kMaxS + 1];
            if (!isfinite(est)) { err = true; break; }
            if (est <= tol_abs || lucky || q < s) break;
        }
        if (err) { status = SSTEP_ERR_NONFINITE; break; }
        // y = R^{-1} rhs, assembly coefficients
        if (tid == 0) scalar_ysolve(W, ncols, s, ldg, lm);
        __syncthreads();
        wg_lincomb<NT, 1>(V, ld, ncols, lm, 1, S.x, N, 1, N, false);
        __syncthreads();
        pc.lap(SSTEP_K_UPDATE);
    }
    if (tid == 0) {
        S.status = status;
        S.blocks = blocks;
        S.cycles = cycles;
        S.rel_resid = fnorm > 0.0 ? beta / fnorm : beta;
        for (int c = 0; c < SSTEP_K_NCLASS; ++c) S.ticks[c] = pc.acc[c];
    }
    __syncthreads();
}

template <int NT, int CA, int KZ>
__global__ __launch_bounds__(NT) void k_batched_gmres(BatchArgs args) {
    __shared__ double red[(NT / 64) * CA * (KZ + 1)];
    __shared__ double sh[3 * kMaxS + 4];
    __shared__ double lw[kMaxS * kMaxS];
    __shared__ GramFactor lf;
    __shared__ double lm[512 * 8];  // update / assembly coefficients
    __shared__ StencilView sA;      // the current system's operator
    __shared__ long long clk[SSTEP_K_NCLASS + 1];
    __shared__ int next;
    BatchSlot& W = args.slots[blockIdx.x];
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(args.queue, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();
        if (k >= args.nsys) break;
        BatchSys& S = args.sys[args.order[k]];
        if (threadIdx.x == 0) sA = S.A;
        __syncthreads();
        solve_one<NT, CA, KZ>(args, S, W, red, sh, lw, &lf, lm, sA, clk);
    }
}

// queue reset, recorded as a kernel node (no memset node in the graph)
static __global__ void k_batch_reset(int* queue) { *queue = 0; }

// ---------------------------------------------------------------------------
// host side: a plan uploads the system table once, captures the queue reset
// and the persistent launch in a hipGraph, and replays it per execution.
// ---------------------------------------------------------------------------
struct BatchPlan {
    int nsys = 0, s = 0, m = 0, threads = 512, wgs_per_cu = 1, nslots = 0;
    double tick_khz = 1e5;  // wall-clock rate of the device (kHz)
    hipStream_t st = nullptr;
    void* ws = nullptr;
    bool owned = false;
    BatchSys* dsys = nullptr;
    std::vector<BatchSys> hs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchArgs args{};
};

static void batch_enqueue(const BatchPlan& P, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, P.args.queue);
    const dim3 g(P.nslots);
#define SSTEP_BATCH(NT, CA, KZ) \
    hipLaunchKernelGGL((k_batched_gmres<NT, CA, KZ>), g, dim3(NT), 0, s, P.args)
    if (P.s <= 4) {
        if (P.threads == 256) SSTEP_BATCH(256, 8, 4);
        else if (P.threads == 512) SSTEP_BATCH(512, 8, 4);
        else SSTEP_BATCH(1024, 4, 4);
    } else {
        if (P.threads == 256) SSTEP_BATCH(256, 4, 8);
        else if (P.threads == 512) SSTEP_BATCH(512, 4, 8);
        else SSTEP_BATCH(1024, 2, 8);
    }
#undef SSTEP_BATCH
}

size_t batched_workspace_bytes(int nsys, const sstep_stencil* A, int s, int m, int nslots) {
    size_t tot = 0;
    for (int i = 0; i < nsys; ++i)
        tot += ((size_t)(m * s + 1) * col_stride(grid_points(A[i])) * sizeof(double) + 255) / 256 * 256;
    tot += (sizeof(BatchSlot) * (size_t)nslots + 255) / 256 * 256 + 4096 +
           (sizeof(BatchSys) * (size_t)nsys + 255) / 256 * 256 + (sizeof(int) * (size_t)nsys + 255) / 256 * 256;
    return tot;
}

int batched_slots(int nsys, int wgs_per_cu) {
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return std::min(nsys, std::max(1, ncu) * wgs_per_cu);
}

int batched_plan_create(void** out, int nsys, const sstep_stencil* A, const double* const* f,
                        double* const* x, int s, int m, double tol, const sstep_options& opt) {
    BatchPlan* P = new BatchPlan();
    P->nsys = nsys;
    P->s = s;
    P->m = m;
    P->threads = opt.batch_threads > 0 ? opt.batch_threads : 512;
    P->wgs_per_cu = opt.batch_wgs_per_cu > 0 ? opt.batch_wgs_per_cu : 1;
    P->nslots = batched_slots(nsys, P->wgs_per_cu);
    P->st = (hipStream_t)opt.stream;
    {
        int dev = 0, khz = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            P->tick_khz = khz;
        else
            (void)hipGetLastError();
    }
    const size_t need = batched_workspace_bytes(nsys, A, s, m, P->nslots);
    if (opt.workspace) {
        if (opt.workspace_bytes < need || ((uintptr_t)opt.workspace & 255u)) {
            delete P;
            return SSTEP_ERR_NOMEM;
        }
        P->ws = opt.workspace;
    } else {
        if (hipMalloc(&P->ws, need) != hipSuccess) {
            (void)hipGetLastError();
            delete P;
            return SSTEP_ERR_NOMEM;
        }
        P->owned = true;
    }
    try {
        char* base = (char*)P->ws;
        size_t off = 0;
        auto take = [&](size_t b) {
            const size_t o = off;
            off += (b + 255) / 256 * 256;
            return base + o;
        };
        BatchSlot* slots = (BatchSlot*)take(sizeof(BatchSlot) * P->nslots);
        int* queue = (int*)take(4096);
        P->dsys = (BatchSys*)take(sizeof(BatchSys) * nsys);
        int* dorder = (int*)take(sizeof(int) * nsys);
        P->hs.resize(nsys);
        for (int i = 0; i < nsys; ++i) {
            BatchSys& b = P->hs[i];
            std::memset(&b, 0, sizeof(b));
            b.A = make_view(A[i]);
            b.f = f[i];
            b.x = x[i];
            b.ld = col_stride(b.A.N);
            b.ws = (double*)take((size_t)(m * s + 1) * b.ld * sizeof(double));
            // sigma: power-of-two Gershgorin bound (per-point coefficients are
            // scanned on the device; the queue word is free scratch until launch)
            b.sigma = op_params(A[i], opt.sigma, P->st, (double*)queue).sigma;
        }
        std::vector<int> order(nsys);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return P->hs[a].A.N > P->hs[b].A.N; });
        SSTEP_HIP(hipMemcpyAsync(P->dsys, P->hs.data(), sizeof(BatchSys) * nsys,
                                 hipMemcpyHostToDevice, P->st));
        SSTEP_HIP(hipMemcpyAsync(dorder, order.data(), sizeof(int) * nsys, hipMemcpyHostToDevice,
                                 P->st));
        SSTEP_HIP(hipStreamSynchronize(P->st));
        BatchArgs& args = P->args;
        args.sys = P->dsys;
        args.order = dorder;
        args.nsys = nsys;
        args.s = s;
        args.m = m;
        args.tol = tol;
        args.max_blocks = opt.max_iters > 0 ? opt.max_iters : 10000;
        args.rank_tol = 1e-14;
        args.lucky_tol = 1e-14;
        args.slots = slots;
        args.queue = queue;
        if (opt.batch_graph) {
            // capture on a private stream (capture needs a non-default stream)
            hipStream_t cs;
            SSTEP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            SSTEP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            batch_enqueue(*P, cs);
            SSTEP_HIP(hipStreamEndCapture(cs, &P->graph));
            SSTEP_HIP(hipStreamDestroy(cs));
            SSTEP_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
        }
    } catch (...) {
        if (P->owned) (void)hipFree(P->ws);
        delete P;
        throw;
    }
    *out = P;
    return SSTEP_OK;
}

int batched_plan_execute(void* plan, sstep_info* info, double* ms_out) {
    BatchPlan* P = (BatchPlan*)plan;
    hipEvent_t e0, e1;
    SSTEP_HIP(hipEventCreate(&e0));
    SSTEP_HIP(hipEventCreate(&e1));
    SSTEP_HIP(hipEventRecord(e0, P->st));
    if (P->exec) SSTEP_HIP(hipGraphLaunch(P->exec, P->st));
    else batch_enqueue(*P, P->st);
    SSTEP_HIP(hipGetLastError());
    SSTEP_HIP(hipEventRecord(e1, P->st));
    SSTEP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    SSTEP_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_out) *ms_out = ms;
    SSTEP_HIP(hipMemcpy(P->hs.data(), P->dsys, sizeof(BatchSys) * P->nsys, hipMemcpyDeviceToHost));
    int status = SSTEP_OK;
    for (int i = 0; i < P->nsys; ++i) {
        const BatchSys& b = P->hs[i];
        if (info) {
            std::memset(&info[i], 0, sizeof(sstep_info));
            info[i].status = b.status;
            info[i].iters = b.blocks;
            info[i].cycles = b.cycles;
            info[i].rel_resid = b.rel_resid;
            info[i].sigma = b.sigma;
            info[i].ms_total = ms;
            for (int c = 0; c < SSTEP_K_NCLASS; ++c) info[i].ms[c] = (double)b.ticks[c] / P->tick_khz;
        }
        if (b.status < 0 && status >= 0) status = b.status;
        else if (b.status == SSTEP_NOT_CONVERGED && status == SSTEP_OK) status = SSTEP_NOT_CONVERGED;
    }
    return status;
}

void batched_plan_destroy(void* plan) {
    BatchPlan* P = (BatchPlan*)plan;
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->owned) (void)hipFree(P->ws);
    delete P;
}

}  // namespace sstep
