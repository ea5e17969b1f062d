/*
 * sstep_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Implements, in the paper's order and notation (Chronopoulos & Kim,
 * arXiv 2001.04886):
 *   - the matrix-free stencil operator of the test problems (Sec. 1 and 5:
 *     5-point Laplacian with central first derivatives; 7-point in 3-D);
 *   - Omin(k) / GCR (Sec. 2, Alg. 2.1);
 *   - GMRES(M) (Sec. 2, Alg. 2.2 with eqs. (2)-(3), modified Gram-Schmidt and
 *     Givens QR for the least-squares problem);
 *   - s-step Orthomin(k) / s-step GCR (Sec. 3, Alg. 3.1);
 *   - s-step GMRES(m) (Sec. 4, Alg. 4.1 and 4.2, eqs. (4)-(8));
 *   - ILU(0) right preconditioning of both s-step methods (Sec. 5).
 *
 * Readings of the paper used here (each is listed with its justification in
 * the design notes of the repository):
 *   - Omin window: the k most recent blocks, j from max(0, i-k+1) to i.
 *   - Scalar1 right-hand side of s-Omin is m_i = (AP_i)^T r_i.
 *   - c_j^l of s-Omin is (A^l r_{i+1})^T (A p_j^q), i.e. C_j = AP_j^T AR_{i+1},
 *     and B_j = -W_j^{-1} C_j, P_{i+1} = R_{i+1} + sum_j P_j B_j.
 *   - m in s-GMRES(m) counts s-blocks; one cycle spans a Krylov space of
 *     dimension m*s (Remark 4.1).
 *   - Matrix powers are scaled: y_j = A y_{j-1} / sigma (sigma a power of two
 *     bounding ||A||_inf), or the Chebyshev three-term form with the same span.
 *   - Every block start vector w_{k+1} is normalised and its norm nu_k is
 *     carried in the Hessenberg matrix (the paper normalises only v_1^1).
 *   - The next block starts from A^s w_k projected on the blocks so far; this
 *     equals A v_k^s projected (the paper's step 2) up to a vector already in
 *     the span, so the same w_{k+1} results with s matvecs per block.
 *   - Gram matrices are factored by Cholesky of the diagonally equilibrated
 *     matrix; a pivot below ORC_RANK_TOL marks numerical rank deficiency and
 *     the block is truncated to its leading full-rank columns.
 *   - Stopping: true relative residual ||f - A x|| / ||f|| <= tol, with
 *     least-squares (GMRES) or recurrence (Omin) estimates as triggers.
 */
#include "sstep_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_RANK_TOL 1e-14     /* equilibrated Cholesky pivot threshold       */
#define ORC_LUCKY_TOL 1e-14    /* nu_k <= this * ||Yhat_s||: invariant subspace */

/* ------------------------------------------------------------------------ */
/* small dense helpers (plain loops)                                         */
/* ------------------------------------------------------------------------ */

/* Timing build only (compiled with -fopenmp, see build_omp in oracle/__init__.py):
 * the N-length loops below run on all host cores; inner products are then
 * summed in fixed blocks of ORC_OMP_BLOCK points whose sums are added in
 * order, so the result does not depend on the thread count.  The plain
 * build (no -fopenmp) ignores every pragma and sums in index order. */
#define ORC_OMP_BLOCK 32768LL

static double dot(long long n, const double *a, const double *b)
{
#ifdef _OPENMP
    if (n > ORC_OMP_BLOCK) {
        const long long nb = (n + ORC_OMP_BLOCK - 1) / ORC_OMP_BLOCK;
        double *part = malloc(sizeof(double) * nb);
        if (part) {
#pragma omp parallel for schedule(static)
            for (long long k = 0; k < nb; ++k) {
                const long long p1 = (k + 1) * ORC_OMP_BLOCK < n ? (k + 1) * ORC_OMP_BLOCK : n;
                double t = 0.0;
                for (long long p = k * ORC_OMP_BLOCK; p < p1; ++p) t += a[p] * b[p];
                part[k] = t;
            }
            double s = 0.0;
            for (long long k = 0; k < nb; ++k) s += part[k];
            free(part);
            return s;
        }
    }
#endif
    double s = 0.0;
    for (long long p = 0; p < n; ++p) s += a[p] * b[p];
    return s;
}

static double nrm2(long long n, const double *a) { return sqrt(dot(n, a, a)); }

static void axpy(long long n, double alpha, const double *x, double *y)
{
#pragma omp parallel for schedule(static) if (n > ORC_OMP_BLOCK)
    for (long long p = 0; p < n; ++p) y[p] += alpha * x[p];
}

static int all_finite(long long n, const double *a)
{
    for (long long p = 0; p < n; ++p)
        if (!isfinite(a[p])) return 0;
    return 1;
}

/* Cholesky factor of the equilibrated matrix S W S, S = diag(W_ii)^(-1/2).
 * W is n x n, column-major with leading dimension ldw.  On return
 * U (n x n, column-major, ld n) is upper triangular with U^T U = S W S on its
 * leading q x q part, sc[i] = S_ii, and the return value is the numerical rank
 * q: the factorisation stops at the first pivot (squared) below ORC_RANK_TOL. */
typedef struct {
    int n, q;
    double U[16 * 16];
    double sc[16];
} orc_chol;

static void chol_eq(const double *W, int ldw, int n, orc_chol *F)
{
    F->n = n;
    F->q = n;
    memset(F->U, 0, sizeof(F->U));
    for (int i = 0; i < n; ++i) {
        double d = W[i + i * ldw];
        F->sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    for (int j = 0; j < n; ++j) {
        if (F->sc[j] == 0.0) { F->q = j; return; }
        /* U[i][j] for i < j */
        for (int i = 0; i < j; ++i) {
            double a = F->sc[i] * W[i + j * ldw] * F->sc[j];
            for (int l = 0; l < i; ++l) a -= F->U[l + i * n] * F->U[l + j * n];
            F->U[i + j * n] = a / F->U[i + i * n];
        }
        double piv = F->sc[j] * W[j + j * ldw] * F->sc[j];
        for (int l = 0; l < j; ++l) piv -= F->U[l + j * n] * F->U[l + j * n];
        if (!(piv > ORC_RANK_TOL)) { F->q = j; return; }
        F->U[j + j * n] = sqrt(piv);
    }
}

/* Solve W z = b on the leading q x q part of a factored W; entries q..n-1 of
 * z are set to zero (truncated block).  b and z may alias. */
static void chol_solve(const orc_chol *F, const double *b, double *z)
{
    int n = F->n, q = F->q;
    double t[16];
    for (int i = 0; i < q; ++i) t[i] = F->sc[i] * b[i];
    /* U^T u = t */
    for (int i = 0; i < q; ++i) {
        double a = t[i];
        for (int l = 0; l < i; ++l) a -= F->U[l + i * n] * t[l];
        t[i] = a / F->U[i + i * n];
    }
    /* U v = u */
    for (int i = q - 1; i >= 0; --i) {
        double a = t[i];
        for (int l = i + 1; l < q; ++l) a -= F->U[i + l * n] * t[l];
        t[i] = a / F->U[i + i * n];
    }
    for (int i = 0; i < q; ++i) z[i] = F->sc[i] * t[i];
    for (int i = q; i < n; ++i) z[i] = 0.0;
}

/* Upper Cholesky factor L of W itself (L^T L = W on the leading q x q part),
 * recovered from the equilibrated factor: L = U S^{-1}. */
static void chol_upper_of_W(const orc_chol *F, double *L /* n x n col-major */)
{
    int n = F->n;
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < F->q; ++j)
        for (int i = 0; i <= j; ++i) L[i + j * n] = F->U[i + j * n] / F->sc[j];
}

/* ------------------------------------------------------------------------ */
/* operator (Sec. 1 and 5: 5-point / 7-point finite-difference stencil)      */
/* ------------------------------------------------------------------------ */

long long orc_size(const orc_stencil *A)
{
    long long nz = A->ndim == 3 ? A->nz : 1;
    return (long long)A->nx * A->ny * nz;
}

/* y = A x.  Each row sums its neighbour terms in the fixed order
 * -x, +x, -y, +y, -z, +z and then adds the centre term.  With ILU(0) factors
 * attached (A->ilu), y = A (L U)^{-1} x. */
void orc_apply(const orc_stencil *A, const double *x, double *y)
{
    const int nx = A->nx, ny = A->ny, nz = A->ndim == 3 ? A->nz : 1;
    const long long N = orc_size(A);
    const long long sx = 1, sy = nx, sz = (long long)nx * ny;
    double *t = NULL;
    if (A->ilu) {
        t = malloc(sizeof(double) * N);
        if (!t) { for (long long p = 0; p < N; ++p) y[p] = NAN; return; }
        orc_ilu0_solve(A, A->ilu, x, t);
        x = t;
    }
#pragma omp parallel for collapse(2) schedule(static) if (N > ORC_OMP_BLOCK)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long long p = i + sy * j + sz * l;
                double c[7];
                for (int q = 0; q < 7; ++q) c[q] = A->coef ? A->coef[q * N + p] : A->c[q];
                double acc = 0.0;
                if (i > 0) acc += c[1] * x[p - sx];
                if (i < nx - 1) acc += c[2] * x[p + sx];
                if (j > 0) acc += c[3] * x[p - sy];
                if (j < ny - 1) acc += c[4] * x[p + sy];
                if (A->ndim == 3) {
                    if (l > 0) acc += c[5] * x[p - sz];
                    if (l < nz - 1) acc += c[6] * x[p + sz];
                }
                y[p] = acc + c[0] * x[p];
            }
    free(t);
}

/* Power scaling sigma: the smallest power of two >= max_row sum_q |a_pq|
 * (Gershgorin bound on the spectrum).  A power of two makes the scaling exact
 * in floating point. */
double orc_sigma(const orc_stencil *A)
{
    /* the preconditioned operator is close to the identity: no scaling */
    if (A->ilu) return 1.0;
    const long long N = orc_size(A);
    const int nq = A->ndim == 3 ? 7 : 5;
    double bound = 0.0;
    if (!A->coef) {
        for (int q = 0; q < nq; ++q) bound += fabs(A->c[q]);
    } else {
        for (long long p = 0; p < N; ++p) {
            double b = 0.0;
            for (int q = 0; q < nq; ++q) b += fabs(A->coef[q * N + p]);
            if (b > bound) bound = b;
        }
    }
    if (!(bound > 0.0)) return 1.0;
    int e;
    double m = frexp(bound, &e); /* bound = m 2^e, m in [0.5,1) */
    return m == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

/* Interval [centre - half_width, centre + half_width] of the Chebyshev basis.
 * For constant coefficients it is the exact spectrum of the symmetric part
 * (A + A^T)/2: per axis a tridiagonal Toeplitz matrix with off-diagonal
 * (c_- + c_+)/2 whose eigenvalues are cos(j pi/(n+1)) multiples; for variable
 * coefficients the Gershgorin interval of A's rows. */
void orc_cheb_interval(const orc_stencil *A, double *centre, double *half_width)
{
    const int nd = A->ndim == 3 ? 3 : 2;
    const int n[3] = {A->nx, A->ny, A->ndim == 3 ? A->nz : 1};
    if (!A->coef) {
        double hw = 0.0;
        for (int a = 0; a < nd; ++a)
            hw += fabs(A->c[1 + 2 * a] + A->c[2 + 2 * a]) * cos(ORC_PI / (n[a] + 1));
        *centre = A->c[0];
        *half_width = hw;
    } else {
        const long long N = orc_size(A);
        double lo = INFINITY, hi = -INFINITY;
        for (long long p = 0; p < N; ++p) {
            double r = 0.0;
            for (int q = 1; q <= 2 * nd; ++q) r += fabs(A->coef[q * N + p]);
            double c0 = A->coef[p];
            if (c0 - r < lo) lo = c0 - r;
            if (c0 + r > hi) hi = c0 + r;
        }
        *centre = 0.5 * (lo + hi);
        *half_width = 0.5 * (hi - lo);
    }
    if (!(*half_width > 0.0)) *half_width = fabs(*centre) > 0.0 ? fabs(*centre) : 1.0;
}

void orc_newton_shifts(int s, double cc, double cd, double *th)
{
    double pts[16];
    int used[16] = {0};
    for (int k = 0; k < s; ++k) pts[k] = cc + cd * cos((2.0 * k + 1.0) * ORC_PI / (2.0 * s));
    for (int n = 0; n < s; ++n) {
        int best = -1;
        double bv = -1.0;
        for (int k = 0; k < s; ++k) {
            if (used[k]) continue;
            double v;
            if (n == 0) {
                v = fabs(pts[k]);
            } else {
                v = 1.0;
                for (int j = 0; j < n; ++j) v *= fabs(pts[k] - th[j]);
            }
            if (v > bv) { bv = v; best = k; }
        }
        used[best] = 1;
        th[n] = pts[best];
    }
}

/* Matrix powers of one vector (Sec. 3-4: the s directions r, Ar, ..., A^s r).
 * Y is [(s+1)][N]; Y[0] = y0.
 *   monomial : y_j = A y_{j-1} / sigma
 *   Chebyshev: y_1 = (A - c) y_0 / d,  y_{j+1} = 2 (A - c) y_j / d - y_{j-1}
 *   Newton   : y_{j+1} = (A - th_j) y_j / d, th the Leja-ordered shifts
 * All give span{y_0..y_j} = span{y_0, A y_0, ..., A^j y_0}. */
void orc_mpk(const orc_stencil *A, const double *y0, int s, int basis, double sigma,
             double cc, double cd, double *Y)
{
    const long long N = orc_size(A);
    double th[16];
    if (basis == ORC_BASIS_NEWTON) orc_newton_shifts(s, cc, cd, th);
    if (Y != y0) memcpy(Y, y0, sizeof(double) * N);
    for (int j = 1; j <= s; ++j) {
        double *yj = Y + (long long)j * N;
        const double *yp = Y + (long long)(j - 1) * N;
        orc_apply(A, yp, yj);
        if (basis == ORC_BASIS_NEWTON) {
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
            for (long long p = 0; p < N; ++p) yj[p] = (yj[p] - th[j - 1] * yp[p]) / cd;
        } else if (basis == ORC_BASIS_CHEBYSHEV) {
            if (j == 1) {
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
                for (long long p = 0; p < N; ++p) yj[p] = (yj[p] - cc * yp[p]) / cd;
            } else {
                const double *ypp = Y + (long long)(j - 2) * N;
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
                for (long long p = 0; p < N; ++p)
                    yj[p] = 2.0 * (yj[p] - cc * yp[p]) / cd - ypp[p];
            }
        } else {
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
            for (long long p = 0; p < N; ++p) yj[p] /= sigma;
        }
    }
}

/* Matrix B ((s+1) x s, column-major ld s+1) with A Y[:,0:s] = Y B for the
 * basis produced by orc_mpk. */
static void basis_change(int s, int basis, double sigma, double cc, double cd, double *B)
{
    memset(B, 0, sizeof(double) * (s + 1) * s);
    double th[16];
    if (basis == ORC_BASIS_NEWTON) orc_newton_shifts(s, cc, cd, th);
    for (int j = 0; j < s; ++j) {
        if (basis == ORC_BASIS_NEWTON) {
            B[j + j * (s + 1)] = th[j];
            B[(j + 1) + j * (s + 1)] = cd;
        } else if (basis == ORC_BASIS_CHEBYSHEV) {
            if (j == 0) {
                B[0 + 0 * (s + 1)] = cc;
                B[1 + 0 * (s + 1)] = cd;
            } else {
                B[(j - 1) + j * (s + 1)] = 0.5 * cd;
                B[j + j * (s + 1)] = cc;
                B[(j + 1) + j * (s + 1)] = 0.5 * cd;
            }
        } else {
            B[(j + 1) + j * (s + 1)] = sigma;
        }
    }
}

static double true_residual(const orc_stencil *A, const double *f, const double *x, double *r)
{
    const long long N = orc_size(A);
    orc_apply(A, x, r);
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
    for (long long p = 0; p < N; ++p) r[p] = f[p] - r[p];
    return nrm2(N, r);
}

/* Givens rotation zeroing b in (a, b): c a + s b = rho, -s a + c b = 0. */
static void givens(double a, double b, double *c, double *s)
{
    if (b == 0.0) { *c = 1.0; *s = 0.0; return; }
    double h = hypot(a, b);
    *c = a / h;
    *s = b / h;
}

static void set_result(orc_result *res, int status, int iters, int cycles, int matvecs,
                       double rel, double est, int nhist)
{
    if (!res) return;
    res->status = status;
    res->iters = iters;
    res->cycles = cycles;
    res->matvecs = matvecs;
    res->rel_resid = rel;
    res->rel_resid_est = est;
    res->nhist = nhist;
}

/* ------------------------------------------------------------------------ */
/* GMRES(M) -- Sec. 2, Alg. 2.2, eqs. (2)-(3)                                */
/* ------------------------------------------------------------------------ */

/* Restarted GMRES(M): Arnoldi by modified Gram-Schmidt, least squares
 * min ||beta e_1 - G_M y|| by Givens QR, x_M = x_0 + Q_M y_M, restart on the
 * true residual.  The residual estimate |g_{j+1}| is checked after every step.
 * max_steps bounds the total number of Arnoldi steps (0: 1000 cycles).
 * If Q_out / H_out are given, the first cycle's basis ([M+1][N]) and
 * Hessenberg ([(M+1)][M] column-major, ld M+1) are stored there. */
int orc_gmres(const orc_stencil *A, const double *f, double *x, int M, double tol,
              int max_steps, orc_result *res, double *hist, int hist_cap,
              double *Q_out, double *H_out)
{
    const long long N = orc_size(A);
    if (N <= 0 || M < 1 || tol < 0.0) { set_result(res, ORC_ERR_ARG, 0, 0, 0, NAN, NAN, 0); return ORC_ERR_ARG; }
    if (max_steps <= 0) max_steps = 1000 * M;
    double *Q = malloc(sizeof(double) * N * (M + 1));
    double *H = calloc((size_t)(M + 1) * M, sizeof(double));  /* Hessenberg G_M      */
    double *Rm = calloc((size_t)(M + 1) * M, sizeof(double)); /* its Givens rotation */
    double *cs = malloc(sizeof(double) * M), *sn = malloc(sizeof(double) * M);
    double *g = malloc(sizeof(double) * (M + 1)), *y = malloc(sizeof(double) * M);
    double *r = malloc(sizeof(double) * N);
    if (!Q || !H || !Rm || !cs || !sn || !g || !y || !r) {
        free(Q); free(H); free(Rm); free(cs); free(sn); free(g); free(y); free(r);
        set_result(res, ORC_ERR_NOMEM, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_NOMEM;
    }
    const double nf = nrm2(N, f);
    const double tol_abs = tol * nf;
    int steps = 0, cycles = 0, matvecs = 0, nh = 0, status = ORC_NOT_CONVERGED;
    double est = NAN;
    double beta = true_residual(A, f, x, r);
    ++matvecs;
    for (;;) {
        if (!isfinite(beta)) { status = ORC_ERR_NONFINITE; break; }
        if (beta <= tol_abs) { status = ORC_OK; break; }
        if (steps >= max_steps) break;
        ++cycles;
        memset(H, 0, sizeof(double) * (M + 1) * M);
        for (long long p = 0; p < N; ++p) Q[p] = r[p] / beta;
        memset(g, 0, sizeof(double) * (M + 1));
        g[0] = beta;
        int j = 0;
        for (; j < M && steps < max_steps; ++j) {
            double *w = Q + (long long)(j + 1) * N;
            orc_apply(A, Q + (long long)j * N, w);
            ++matvecs;
            for (int i = 0; i <= j; ++i) { /* modified Gram-Schmidt */
                double h = dot(N, Q + (long long)i * N, w);
                H[i + j * (M + 1)] = h;
                axpy(N, -h, Q + (long long)i * N, w);
            }
            double hn = nrm2(N, w);
            H[(j + 1) + j * (M + 1)] = hn;
            if (hn > 0.0)
                for (long long p = 0; p < N; ++p) w[p] /= hn;
            ++steps;
            if (cycles == 1) {
                if (Q_out) memcpy(Q_out, Q, sizeof(double) * N * (j + 2));
                if (H_out) memcpy(H_out, H, sizeof(double) * (M + 1) * M);
            }
            /* apply previous rotations to the new column, then a new one */
            double *hc = Rm + j * (M + 1);
            memcpy(hc, H + j * (M + 1), sizeof(double) * (M + 1));
            for (int i = 0; i < j; ++i) {
                double a = hc[i], b = hc[i + 1];
                hc[i] = cs[i] * a + sn[i] * b;
                hc[i + 1] = -sn[i] * a + cs[i] * b;
            }
            givens(hc[j], hc[j + 1], &cs[j], &sn[j]);
            hc[j] = cs[j] * hc[j] + sn[j] * hc[j + 1];
            hc[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            est = fabs(g[j + 1]);
            if (hist && nh < hist_cap) hist[nh++] = est / nf;
            if (est <= tol_abs || hn == 0.0) { ++j; break; }
        }
        /* back substitution R y = g */
        for (int i = j - 1; i >= 0; --i) {
            double a = g[i];
            for (int l = i + 1; l < j; ++l) a -= Rm[i + l * (M + 1)] * y[l];
            y[i] = a / Rm[i + i * (M + 1)];
        }
        for (int i = 0; i < j; ++i) axpy(N, y[i], Q + (long long)i * N, x);
        beta = true_residual(A, f, x, r);
        ++matvecs;
    }
    set_result(res, status, steps, cycles, matvecs, beta / nf, est / nf, nh);
    free(Q); free(H); free(Rm); free(cs); free(sn); free(g); free(y); free(r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Omin(k) / GCR -- Sec. 2, Alg. 2.1                                         */
/* ------------------------------------------------------------------------ */

/* Omin(k): a_i = r_i^T Ap_i / (Ap_i)^T Ap_i; x += a p; r -= a Ap;
 * b_j = (A r_{i+1})^T Ap_j / (Ap_j)^T Ap_j over the k most recent j;
 * p_{i+1} = r_{i+1} - sum b_j p_j; Ap_{i+1} = A r_{i+1} - sum b_j Ap_j.
 * k >= max_iters gives GCR.  The recurrence residual triggers a true-residual
 * check; if that fails, r is replaced by the true residual and the direction
 * window restarts. */
int orc_omin(const orc_stencil *A, const double *f, double *x, int k, double tol,
             int max_iters, orc_result *res, double *hist, int hist_cap)
{
    const long long N = orc_size(A);
    if (N <= 0 || k < 1 || tol < 0.0) { set_result(res, ORC_ERR_ARG, 0, 0, 0, NAN, NAN, 0); return ORC_ERR_ARG; }
    if (max_iters <= 0) max_iters = 100000;
    double *P = malloc(sizeof(double) * N * k), *AP = malloc(sizeof(double) * N * k);
    double *apn = malloc(sizeof(double) * k);
    double *r = malloc(sizeof(double) * N), *Ar = malloc(sizeof(double) * N);
    double *rt = malloc(sizeof(double) * N);
    double *pn = malloc(sizeof(double) * N), *apnw = malloc(sizeof(double) * N);
    double *b = malloc(sizeof(double) * k);
    if (!P || !AP || !apn || !r || !Ar || !rt || !pn || !apnw || !b) {
        free(P); free(AP); free(apn); free(r); free(Ar); free(rt); free(pn); free(apnw); free(b);
        set_result(res, ORC_ERR_NOMEM, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_NOMEM;
    }
    const double nf = nrm2(N, f), tol_abs = tol * nf;
    int it = 0, cycles = 0, matvecs = 0, nh = 0, status = ORC_NOT_CONVERGED;
    double rn = true_residual(A, f, x, r), est = rn;
    ++matvecs;
    while (status == ORC_NOT_CONVERGED) {
        if (!isfinite(rn)) { status = ORC_ERR_NONFINITE; break; }
        if (rn <= tol_abs) { status = ORC_OK; break; }
        if (it >= max_iters) break;
        ++cycles;
        /* direction j is held in slot j % k */
        memcpy(P, r, sizeof(double) * N);
        orc_apply(A, r, AP);
        ++matvecs;
        int i = 0;
        for (;;) {
            int si = i % k;
            double *p = P + (long long)si * N, *ap = AP + (long long)si * N;
            double w = dot(N, ap, ap);
            if (!(w > 0.0)) { status = ORC_ERR_BREAKDOWN; break; }
            apn[si] = w;
            double a = dot(N, r, ap) / w;
            axpy(N, a, p, x);
            axpy(N, -a, ap, r);
            ++it;
            est = nrm2(N, r);
            if (hist && nh < hist_cap) hist[nh++] = est / nf;
            if (!isfinite(est)) { status = ORC_ERR_NONFINITE; break; }
            if (est <= tol_abs || it >= max_iters) {
                rn = true_residual(A, f, x, rt);
                ++matvecs;
                if (rn <= tol_abs) { status = ORC_OK; break; }
                memcpy(r, rt, sizeof(double) * N);
                break; /* residual replacement: restart the window */
            }
            orc_apply(A, r, Ar);
            ++matvecs;
            int j0 = i - k + 1 > 0 ? i - k + 1 : 0;
            int sn = (i + 1) % k;
            /* the new direction goes into the slot of the oldest one once
             * all coefficients are known */
            for (int j = j0; j <= i; ++j) {
                const double *apj = AP + (long long)(j % k) * N;
                b[j - j0] = dot(N, Ar, apj) / apn[j % k];
            }
            memcpy(pn, r, sizeof(double) * N);
            memcpy(apnw, Ar, sizeof(double) * N);
            for (int j = j0; j <= i; ++j) {
                axpy(N, -b[j - j0], P + (long long)(j % k) * N, pn);
                axpy(N, -b[j - j0], AP + (long long)(j % k) * N, apnw);
            }
            memcpy(P + (long long)sn * N, pn, sizeof(double) * N);
            memcpy(AP + (long long)sn * N, apnw, sizeof(double) * N);
            ++i;
        }
        if (status != ORC_NOT_CONVERGED) break;
        if (it >= max_iters) break;
    }
    if (status == ORC_NOT_CONVERGED || status == ORC_OK) {
        rn = true_residual(A, f, x, rt);
        if (!isfinite(rn)) status = ORC_ERR_NONFINITE;
    }
    set_result(res, status, it, cycles, matvecs, rn / nf, est / nf, nh);
    free(P); free(AP); free(apn); free(r); free(Ar); free(rt); free(pn); free(apnw); free(b);
    return status;
}

/* ------------------------------------------------------------------------ */
/* s-step Orthomin(k) / s-step GCR -- Sec. 3, Alg. 3.1                       */
/* ------------------------------------------------------------------------ */

/* Larger-s variant (Sec. 3, after Alg. 3.1): the new direction block is made
 * A^T A-orthogonal by modified Gram-Schmidt on the columns of AP (the same
 * combinations applied to P), so W = AP^T AP becomes diagonal.  Column q,
 * after its components along columns 0..q-1 are removed, keeps a fraction
 * w_q / n0_q of its squared length n0_q; at or below ORC_RANK_TOL it is
 * numerically dependent and is set to zero (the Cholesky of W then truncates
 * the block there, the same rank rule as without the orthogonalisation). */
static void mgs_ata(long long N, int s, double *P, double *AP)
{
    for (int q = 0; q < s; ++q) {
        double *aq = AP + (long long)q * N, *pq = P + (long long)q * N;
        const double n0 = dot(N, aq, aq);
        for (int l = 0; l < q; ++l) {
            const double *al = AP + (long long)l * N;
            const double wl = dot(N, al, al);
            if (!(wl > 0.0)) continue;
            const double c = dot(N, al, aq) / wl;
            axpy(N, -c, al, aq);
            axpy(N, -c, P + (long long)l * N, pq);
        }
        const double w = dot(N, aq, aq);
        if (!(w > ORC_RANK_TOL * n0) || !isfinite(w)) {
            memset(aq, 0, sizeof(double) * N);
            memset(pq, 0, sizeof(double) * N);
        }
    }
}

/* One s-step iteration i:
 *   W_i = AP_i^T AP_i, m_i = AP_i^T r_i            (step 1)
 *   W_i a_i = m_i                                   (step 2, Scalar1)
 *   x_{i+1} = x_i + P_i a_i, r_{i+1} = r_i - AP_i a_i   (steps 3-4)
 *   R_{i+1} = [r, Ar, ..] via matrix powers, AR_{i+1} = A R_{i+1}   (step 5)
 *   C_j = AP_j^T AR_{i+1}, W_j B_j = -C_j           (steps 6-7, Scalar2)
 *   P_{i+1} = R_{i+1} + sum_j P_j B_j, AP_{i+1} = AR_{i+1} + sum_j AP_j B_j (8-9)
 * over the window j = max(0, i-k+1) .. i.  P_0 = R_0.
 * With the monomial basis R = [r, Ar/sigma, ..., A^{s-1} r/sigma^{s-1}]. */
int orc_somin(const orc_stencil *A, const double *f, double *x, int s, int k, double tol,
              int max_iters, int basis, orc_result *res, double *hist, int hist_cap,
              orc_omin_dump *dump)
{
    return orc_somin_ex(A, f, x, s, k, tol, max_iters, basis, 0, res, hist, hist_cap, dump);
}

int orc_somin_ex(const orc_stencil *A, const double *f, double *x, int s, int k, double tol,
                 int max_iters, int basis, int mgs, orc_result *res, double *hist, int hist_cap,
                 orc_omin_dump *dump)
{
    const long long N = orc_size(A);
    if (N <= 0 || s < 1 || s > 16 || k < 1 || tol < 0.0) {
        set_result(res, ORC_ERR_ARG, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_ARG;
    }
    if (max_iters <= 0) max_iters = 100000;
    const double sigma = orc_sigma(A);
    double cc = 0.0, cd = 1.0;
    if (basis != ORC_BASIS_MONOMIAL) orc_cheb_interval(A, &cc, &cd);
    double B[17 * 16];
    basis_change(s, basis, sigma, cc, cd, B);

    const long long sN = (long long)s * N;
    double *P = malloc(sizeof(double) * sN * k), *AP = malloc(sizeof(double) * sN * k);
    double *Y = malloc(sizeof(double) * N * (s + 1));
    double *AR = malloc(sizeof(double) * sN);
    double *Pn = malloc(sizeof(double) * sN), *APn = malloc(sizeof(double) * sN);
    double *r = malloc(sizeof(double) * N), *rt = malloc(sizeof(double) * N);
    orc_chol *Wf = malloc(sizeof(orc_chol) * k);
    if (!P || !AP || !Y || !AR || !Pn || !APn || !r || !rt || !Wf) {
        free(P); free(AP); free(Y); free(AR); free(Pn); free(APn); free(r); free(rt); free(Wf);
        set_result(res, ORC_ERR_NOMEM, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_NOMEM;
    }
    const double nf = nrm2(N, f), tol_abs = tol * nf;
    int it = 0, cycles = 0, matvecs = 0, nh = 0, status = ORC_NOT_CONVERGED;
    int last_i = -1;
    double rn = true_residual(A, f, x, r), est = rn;
    ++matvecs;

    /* R, AR of the current residual into Pdst, APdst */
#define BUILD_R_AR(Pdst, APdst)                                                         \
    do {                                                                                \
        orc_mpk(A, r, s, basis, sigma, cc, cd, Y);                                      \
        matvecs += s;                                                                   \
        memcpy((Pdst), Y, sizeof(double) * sN);                                         \
        for (int q = 0; q < s; ++q) {                                                   \
            double *o = (APdst) + (long long)q * N;                                     \
            memset(o, 0, sizeof(double) * N);                                           \
            for (int l = 0; l <= s; ++l) {                                              \
                double bl = B[l + q * (s + 1)];                                         \
                if (bl != 0.0) axpy(N, bl, Y + (long long)l * N, o);                    \
            }                                                                           \
        }                                                                               \
    } while (0)

    while (status == ORC_NOT_CONVERGED) {
        if (!isfinite(rn)) { status = ORC_ERR_NONFINITE; break; }
        if (rn <= tol_abs) { status = ORC_OK; break; }
        if (it >= max_iters) break;
        ++cycles;
        BUILD_R_AR(P, AP); /* P_0 = R_0, AP_0 = AR_0 in slot 0 */
        if (mgs) mgs_ata(N, s, P, AP);
        int i = 0;
        for (;;) {
            int si = i % k;
            double *Pi = P + si * sN, *APi = AP + si * sN;
            /* step 1: W_i, m_i */
            double W[256], mv[16], a[16];
            for (int q = 0; q < s; ++q) {
                for (int l = 0; l < s; ++l) W[l + q * s] = dot(N, APi + (long long)l * N, APi + (long long)q * N);
                mv[q] = dot(N, APi + (long long)q * N, r);
            }
            /* step 2: Scalar1 */
            chol_eq(W, s, s, &Wf[si]);
            if (Wf[si].q == 0) { status = ORC_ERR_BREAKDOWN; break; }
            chol_solve(&Wf[si], mv, a);
            /* steps 3-4 */
            for (int q = 0; q < s; ++q) {
                axpy(N, a[q], Pi + (long long)q * N, x);
                axpy(N, -a[q], APi + (long long)q * N, r);
            }
            ++it;
            last_i = i;
            est = nrm2(N, r);
            if (hist && nh < hist_cap) hist[nh++] = est / nf;
            if (!isfinite(est)) { status = ORC_ERR_NONFINITE; break; }
            if (est <= tol_abs || it >= max_iters) {
                rn = true_residual(A, f, x, rt);
                ++matvecs;
                if (rn <= tol_abs) { status = ORC_OK; break; }
                memcpy(r, rt, sizeof(double) * N);
                break;
            }
            /* step 5: R_{i+1}, AR_{i+1} */
            BUILD_R_AR(Pn, AR);
            /* steps 6-9 over the window */
            int j0 = i - k + 1 > 0 ? i - k + 1 : 0;
            memcpy(APn, AR, sizeof(double) * sN);
            for (int j = j0; j <= i; ++j) {
                const double *Pj = P + (j % k) * sN, *APj = AP + (j % k) * sN;
                double Bj[256];
                for (int l = 0; l < s; ++l) { /* column l of C_j, then B_j */
                    double c[16];
                    for (int q = 0; q < s; ++q) c[q] = dot(N, APj + (long long)q * N, AR + (long long)l * N);
                    chol_solve(&Wf[j % k], c, c);
                    for (int q = 0; q < s; ++q) Bj[q + l * s] = -c[q];
                }
                for (int l = 0; l < s; ++l)
                    for (int q = 0; q < s; ++q) {
                        axpy(N, Bj[q + l * s], Pj + (long long)q * N, Pn + (long long)l * N);
                        axpy(N, Bj[q + l * s], APj + (long long)q * N, APn + (long long)l * N);
                    }
            }
            if (mgs) mgs_ata(N, s, Pn, APn);
            int sn = (i + 1) % k;
            memcpy(P + sn * sN, Pn, sizeof(double) * sN);
            memcpy(AP + sn * sN, APn, sizeof(double) * sN);
            ++i;
        }
        if (status != ORC_NOT_CONVERGED) break;
        if (it >= max_iters) break;
    }
#undef BUILD_R_AR
    if (status == ORC_NOT_CONVERGED || status == ORC_OK) {
        rn = true_residual(A, f, x, rt);
        if (!isfinite(rn)) status = ORC_ERR_NONFINITE;
    }
    if (dump && last_i >= 0) {
        int j0 = last_i - k + 1 > 0 ? last_i - k + 1 : 0;
        int nbk = 0;
        for (int j = j0; j <= last_i; ++j, ++nbk) {
            if (dump->P) memcpy(dump->P + nbk * sN, P + (j % k) * sN, sizeof(double) * sN);
            if (dump->AP) memcpy(dump->AP + nbk * sN, AP + (j % k) * sN, sizeof(double) * sN);
        }
        if (dump->r) memcpy(dump->r, r, sizeof(double) * N);
        dump->nblocks = nbk;
    }
    set_result(res, status, it, cycles, matvecs, rn / nf, est / nf, nh);
    free(P); free(AP); free(Y); free(AR); free(Pn); free(APn); free(r); free(rt); free(Wf);
    return status;
}

/* ------------------------------------------------------------------------ */
/* s-step GMRES(m) -- Sec. 4, Alg. 4.1 (s-step Arnoldi), eqs. (4)-(8),       */
/* Alg. 4.2 (restarted s-step GMRES)                                         */
/* ------------------------------------------------------------------------ */

/* One restart cycle.  Notation: V_k = [Vbar_1 .. Vbar_k] (mutually
 * orthogonal s-blocks, not orthogonal inside a block), U_k = [V_k, w_{k+1}],
 * A V_k = U_k Gbar_k (eq. (5) with the factors in matrix order),
 * D = U_k^T U_k = blockdiag(W_1, .., W_k, 1) = L^T L, and the least-squares
 * problem min_y || beta e_1 - L Gbar_k y || (eq. (7)), x = x_0 + V_k y (eq. (8)).
 *
 * Block k, starting from the normalised w_k:
 *   Y = [y_0 .. y_s] = matrix powers of w_k                         (s Mv)
 *   C_i = Vbar_i^T Y[:,1:s+1], T_i = W_i^{-1} C_i  (i < k)           (Scalar2)
 *   Vbar_k[:,j] = y_j - sum_i Vbar_i T_i[:,j]  (j = 1..s-1; column 0 is w_k)
 *   Yhat_s     = y_s - sum_i Vbar_i T_i[:,s]
 *   W_k = Vbar_k^T Vbar_k, g = W_k^{-1} Vbar_k^T Yhat_s              (Scalar1)
 *   w_{k+1} = (Yhat_s - Vbar_k g) / nu_k,  nu_k = ||Yhat_s - Vbar_k g||
 * Coordinates of Y in U_k: Z_k = [T_1; ..; T_{k-1}; [I_s | g]; nu_k e_s^T],
 * so the new Hessenberg block column is
 *   Gbar[:, block k] = Z_k B - sum_{i<k} Gbar[:, block i] T_i[:, 0:s]
 * with B the basis-change matrix (A Y[:,0:s] = Y B).                         */
static int sgmres_cycle(const orc_stencil *A, double *x, int s, int m,
                        int basis, double sigma, double cc, double cd, const double *Bc,
                        double tol_abs, int max_blocks, double nf, int *blocks_done,
                        int *matvecs, double *est_out, double *hist, int hist_cap, int *nh,
                        orc_cycle_dump *dump, double *work_r, double beta)
{
    const long long N = orc_size(A);
    const int K = m * s;     /* Krylov dimension of a full cycle */
    const int ldg = K + 1;
    double *V = malloc(sizeof(double) * N * (K + 1));
    double *Y = malloc(sizeof(double) * N * (s + 1));
    double *G = calloc((size_t)ldg * K, sizeof(double));  /* Gbar           */
    double *R = calloc((size_t)ldg * K, sizeof(double));  /* rotated L Gbar */
    double *T = malloc(sizeof(double) * (size_t)K * (s + 1));
    double *cs = malloc(sizeof(double) * K), *sn = malloc(sizeof(double) * K);
    double *rhs = calloc(K + 1, sizeof(double)), *y = malloc(sizeof(double) * K);
    orc_chol *Wf = malloc(sizeof(orc_chol) * m);
    double *Ls = malloc(sizeof(double) * (size_t)m * s * s);
    if (!V || !Y || !G || !R || !T || !cs || !sn || !rhs || !y || !Wf || !Ls) {
        free(V); free(Y); free(G); free(R); free(T); free(cs); free(sn); free(rhs); free(y);
        free(Wf); free(Ls);
        return ORC_ERR_NOMEM;
    }
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
    for (long long p = 0; p < N; ++p) V[p] = work_r[p] / beta; /* w_1 = r_0 / beta */
    rhs[0] = beta;
    int ncols = 0, nb = 0, stop = 0;
    double est = beta;
    for (int kb = 0; kb < m && *blocks_done < max_blocks && !stop; ++kb) {
        const int c0 = kb * s;
        /* matrix powers of w_k */
        orc_mpk(A, V + (long long)c0 * N, s, basis, sigma, cc, cd, Y);
        *matvecs += s;
        /* Scalar2: projection coefficients on the previous blocks */
        for (int i = 0; i < kb; ++i) {
            double *Ti = T + (size_t)i * s * (s + 1); /* s x (s+1), col-major ld s */
            for (int q = 0; q < s; ++q) Ti[q] = 0.0;   /* column 0: w_k is already orthogonal */
            for (int l = 1; l <= s; ++l) {
                double c[16];
                for (int q = 0; q < s; ++q)
                    c[q] = dot(N, V + (long long)(i * s + q) * N, Y + (long long)l * N);
                chol_solve(&Wf[i], c, c);
                for (int q = 0; q < s; ++q) Ti[q + l * s] = c[q];
            }
        }
        /* Vbar_k and Yhat_s (block classical Gram-Schmidt, one pass) */
        for (int l = 1; l <= s; ++l) {
            double *yl = Y + (long long)l * N;
            for (int i = 0; i < kb; ++i) {
                const double *Ti = T + (size_t)i * s * (s + 1);
                for (int q = 0; q < s; ++q) axpy(N, -Ti[q + l * s], V + (long long)(i * s + q) * N, yl);
            }
        }
        for (int l = 1; l < s; ++l) memcpy(V + (long long)(c0 + l) * N, Y + (long long)l * N, sizeof(double) * N);
        const double *yhat = Y + (long long)s * N;
        /* Scalar1: W_k, Vbar_k^T Yhat_s */
        double Wk[17 * 17];
        for (int a = 0; a <= s; ++a)
            for (int b = 0; b <= s; ++b) {
                const double *va = a < s ? V + (long long)(c0 + a) * N : yhat;
                const double *vb = b < s ? V + (long long)(c0 + b) * N : yhat;
                Wk[a + b * (s + 1)] = dot(N, va, vb);
            }
        chol_eq(Wk, s + 1, s, &Wf[kb]);
        const int q = Wf[kb].q;
        double g[16], nu = 0.0;
        int lucky = 0;
        if (q == s) {
            double h[16];
            for (int a = 0; a < s; ++a) h[a] = Wk[a + s * (s + 1)];
            chol_solve(&Wf[kb], h, g);
            double *w = V + (long long)(c0 + s) * N;
            memcpy(w, yhat, sizeof(double) * N);
            for (int a = 0; a < s; ++a) axpy(N, -g[a], V + (long long)(c0 + a) * N, w);
            nu = nrm2(N, w);
            if (nu <= ORC_LUCKY_TOL * sqrt(Wk[s + s * (s + 1)])) lucky = 1;
            if (nu > 0.0)
#pragma omp parallel for schedule(static) if (N > ORC_OMP_BLOCK)
                for (long long p = 0; p < N; ++p) w[p] /= nu;
        } else {
            /* truncated block: column q depends on columns 0..q-1 numerically;
             * its coordinates g' = W[0:q,0:q]^{-1} W[0:q,q], and nu = 0 */
            double h[16];
            orc_chol Fq = Wf[kb];
            Fq.n = q;
            /* re-pack the leading q x q factor into an n = q layout */
            for (int jj = 0; jj < q; ++jj)
                for (int ii = 0; ii < q; ++ii) Fq.U[ii + jj * q] = Wf[kb].U[ii + jj * s];
            for (int a = 0; a < q; ++a) h[a] = Wk[a + q * (s + 1)];
            chol_solve(&Fq, h, g);
            nu = 0.0;
            stop = 1;
        }
        /* Hessenberg block column: Gbar[:, c0+j] = Z_k B[:, j] - sum_i Gbar[:, block i] T_i[:, j] */
        const int nq = q; /* columns contributed by this block */
        for (int jc = 0; jc < nq; ++jc) {
            double *gc = G + (size_t)(c0 + jc) * ldg;
            for (int rr = 0; rr < ldg; ++rr) gc[rr] = 0.0;
            for (int l = 0; l <= nq; ++l) {
                double bl = Bc[l + jc * (s + 1)];
                if (bl == 0.0) continue;
                /* column l of Z_k: coordinates of Y[:, l] in U_k; for a
                 * truncated block the last column is Y[:, nq] itself */
                const int lz = l;
                for (int i = 0; i < kb; ++i) {
                    const double *Ti = T + (size_t)i * s * (s + 1);
                    for (int a = 0; a < s; ++a) gc[i * s + a] += bl * Ti[a + lz * s];
                }
                if (l < nq) {
                    gc[c0 + l] += bl;
                } else {
                    for (int a = 0; a < nq; ++a) gc[c0 + a] += bl * g[a];
                    gc[c0 + nq] += bl * nu;
                }
            }
            for (int i = 0; i < kb; ++i) {
                const double *Ti = T + (size_t)i * s * (s + 1);
                for (int l = 0; l < s; ++l) {
                    double t = Ti[l + jc * s];
                    if (t == 0.0) continue;
                    const double *gi = G + (size_t)(i * s + l) * ldg;
                    for (int rr = 0; rr < ldg; ++rr) gc[rr] -= gi[rr] * t;
                }
            }
        }
        /* L scaling of the new columns: D = blockdiag(W_1..W_k, 1) = L^T L */
        double *Lk = Ls + (size_t)kb * s * s;
        chol_upper_of_W(&Wf[kb], Lk);
        for (int jc = 0; jc < nq; ++jc) {
            const double *gc = G + (size_t)(c0 + jc) * ldg;
            double *rc = R + (size_t)(c0 + jc) * ldg;
            for (int rr = 0; rr < ldg; ++rr) rc[rr] = 0.0;
            for (int i = 0; i <= kb; ++i) {
                const double *Li = Ls + (size_t)i * s * s;
                int qi = Wf[i].q;
                for (int a = 0; a < qi; ++a) {
                    double acc = 0.0;
                    for (int b = a; b < qi; ++b) acc += Li[a + b * s] * gc[i * s + b];
                    rc[i * s + a] = acc;
                }
            }
            rc[c0 + nq] = gc[c0 + nq];
            /* Givens QR of the upper Hessenberg L Gbar */
            const int cj = c0 + jc;
            for (int i = 0; i < cj; ++i) {
                double a = rc[i], b = rc[i + 1];
                rc[i] = cs[i] * a + sn[i] * b;
                rc[i + 1] = -sn[i] * a + cs[i] * b;
            }
            givens(rc[cj], rc[cj + 1], &cs[cj], &sn[cj]);
            rc[cj] = cs[cj] * rc[cj] + sn[cj] * rc[cj + 1];
            rc[cj + 1] = 0.0;
            rhs[cj + 1] = -sn[cj] * rhs[cj];
            rhs[cj] = cs[cj] * rhs[cj];
        }
        ncols = c0 + nq;
        est = fabs(rhs[ncols]);
        ++nb;
        ++*blocks_done;
        if (hist && *nh < hist_cap) hist[(*nh)++] = est / nf;
        if (!isfinite(est)) { stop = 2; break; }
        if (lucky || est <= tol_abs) stop = 1;
    }
    /* y = R^{-1} rhs, x = x_0 + V y */
    int status = ORC_OK;
    if (stop == 2) status = ORC_ERR_NONFINITE;
    if (status == ORC_OK) {
        for (int i = ncols - 1; i >= 0; --i) {
            double a = rhs[i];
            for (int l = i + 1; l < ncols; ++l) a -= R[i + (size_t)l * ldg] * y[l];
            y[i] = a / R[i + (size_t)i * ldg];
        }
        for (int i = 0; i < ncols; ++i) axpy(N, y[i], V + (long long)i * N, x);
    }
    if (dump) {
        if (dump->V) memcpy(dump->V, V, sizeof(double) * N * (ncols + 1));
        if (dump->G) memcpy(dump->G, G, sizeof(double) * ldg * K);
        if (dump->D) {
            memset(dump->D, 0, sizeof(double) * ldg * ldg);
            for (int i = 0; i < nb; ++i) {
                double *Li = Ls + (size_t)i * s * s;
                for (int a = 0; a < s; ++a)
                    for (int b = 0; b < s; ++b) {
                        double acc = 0.0;
                        for (int l = 0; l < s; ++l) acc += Li[l + a * s] * Li[l + b * s];
                        dump->D[(i * s + a) + (size_t)(i * s + b) * ldg] = acc;
                    }
            }
            dump->D[ncols + (size_t)ncols * ldg] = 1.0;
        }
        dump->ncols = ncols;
        dump->blocks = nb;
    }
    *est_out = est;
    free(V); free(Y); free(G); free(R); free(T); free(cs); free(sn); free(rhs); free(y);
    free(Wf); free(Ls);
    return status;
}

/* Restarted s-step GMRES (Alg. 4.2): r_0 = f - A x_0, one cycle of at most m
 * s-blocks, x_m = x_0 + V y, restart from the true residual until
 * ||f - A x|| <= tol ||f|| or max_blocks s-blocks have been built. */
int orc_sgmres(const orc_stencil *A, const double *f, double *x, int s, int m, double tol,
               int max_blocks, int basis, orc_result *res, double *hist, int hist_cap,
               orc_cycle_dump *dump)
{
    const long long N = orc_size(A);
    if (N <= 0 || s < 1 || s > 16 || m < 1 || tol < 0.0) {
        set_result(res, ORC_ERR_ARG, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_ARG;
    }
    if (max_blocks <= 0) max_blocks = 1000 * m;
    const double sigma = orc_sigma(A);
    double cc = 0.0, cd = 1.0;
    if (basis != ORC_BASIS_MONOMIAL) orc_cheb_interval(A, &cc, &cd);
    double Bc[17 * 16];
    basis_change(s, basis, sigma, cc, cd, Bc);
    double *r = malloc(sizeof(double) * N);
    if (!r) { set_result(res, ORC_ERR_NOMEM, 0, 0, 0, NAN, NAN, 0); return ORC_ERR_NOMEM; }
    const double nf = nrm2(N, f), tol_abs = tol * nf;
    int blocks = 0, cycles = 0, matvecs = 0, nh = 0, status = ORC_NOT_CONVERGED;
    double est = NAN;
    double beta = true_residual(A, f, x, r);
    ++matvecs;
    for (;;) {
        if (!isfinite(beta) || !all_finite(N, x)) { status = ORC_ERR_NONFINITE; break; }
        if (beta <= tol_abs) { status = ORC_OK; break; }
        if (blocks >= max_blocks) break;
        ++cycles;
        int st = sgmres_cycle(A, x, s, m, basis, sigma, cc, cd, Bc, tol_abs, max_blocks, nf,
                              &blocks, &matvecs, &est, hist, hist_cap, &nh,
                              cycles == 1 ? dump : NULL, r, beta);
        if (st != ORC_OK) { status = st; break; }
        beta = true_residual(A, f, x, r);
        ++matvecs;
    }
    set_result(res, status, blocks, cycles, matvecs, beta / nf, est / nf, nh);
    free(r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* ILU(0) right preconditioning (Sec. 5)                                     */
/* ------------------------------------------------------------------------ */

/* Column of slot q of row p, or -1 if it lies outside the grid. */
static long long ilu_col(const orc_stencil *A, long long p, int q)
{
    const int nx = A->nx, ny = A->ny;
    const int i = (int)(p % nx), j = (int)(p / nx);
    switch (q) {
        case 0: return j > 0 ? p - nx : -1;
        case 1: return i > 0 ? p - 1 : -1;
        case 2: return p;
        case 3: return i < nx - 1 ? p + 1 : -1;
        default: return j < ny - 1 ? p + nx : -1;
    }
}

/* Incomplete LU with the sparsity pattern of A (no fill): Gaussian
 * elimination row by row (i-k-j order), where an update a_pj -= l_pk u_kj is
 * carried out only if (p, j) is in the pattern and dropped otherwise. */
int orc_ilu0_factor(const orc_stencil *A, double *LU)
{
    if (A->ndim != 2) return ORC_ERR_ARG;
    const long long N = orc_size(A);
    /* slot q of LU <- stencil coefficient index: south 3, west 1, centre 0,
     * east 2, north 4 */
    static const int from[5] = {3, 1, 0, 2, 4};
    for (int q = 0; q < 5; ++q)
        for (long long p = 0; p < N; ++p)
            LU[q * N + p] = ilu_col(A, p, q) < 0 ? 0.0
                            : (A->coef ? A->coef[from[q] * N + p] : A->c[from[q]]);
    for (long long p = 0; p < N; ++p) {
        /* lower entries in increasing column order: p - nx before p - 1 */
        for (int qk = 0; qk < 2; ++qk) {
            const long long k = ilu_col(A, p, qk);
            if (k < 0) continue;
            const double ukk = LU[2 * N + k];
            if (ukk == 0.0 || !isfinite(ukk)) return ORC_ERR_BREAKDOWN;
            const double lpk = LU[qk * N + p] / ukk;
            LU[qk * N + p] = lpk;
            for (int qj = 0; qj < 5; ++qj) {
                const long long cj = ilu_col(A, p, qj);
                if (cj <= k) continue;
                for (int qq = 2; qq < 5; ++qq)  /* U part of row k */
                    if (ilu_col(A, k, qq) == cj) LU[qj * N + p] -= lpk * LU[qq * N + k];
            }
        }
        if (LU[2 * N + p] == 0.0 || !isfinite(LU[2 * N + p])) return ORC_ERR_BREAKDOWN;
    }
    return ORC_OK;
}

/* z = (L U)^{-1} r: forward substitution with the unit lower factor, then
 * back substitution with U, in the natural order of the unknowns. */
void orc_ilu0_solve(const orc_stencil *A, const double *LU, const double *r, double *z)
{
    const long long N = orc_size(A);
    for (long long p = 0; p < N; ++p) {
        double v = r[p];
        for (int q = 0; q < 2; ++q) {
            const long long c = ilu_col(A, p, q);
            if (c >= 0) v -= LU[q * N + p] * z[c];
        }
        z[p] = v;
    }
    for (long long p = N - 1; p >= 0; --p) {
        double v = z[p];
        for (int q = 3; q < 5; ++q) {
            const long long c = ilu_col(A, p, q);
            if (c >= 0) v -= LU[q * N + p] * z[c];
        }
        z[p] = v / LU[2 * N + p];
    }
}

/* y = L (U x). */
void orc_ilu0_mul(const orc_stencil *A, const double *LU, const double *x, double *y)
{
    const long long N = orc_size(A);
    double *w = malloc(sizeof(double) * N);
    if (!w) { for (long long p = 0; p < N; ++p) y[p] = NAN; return; }
    for (long long p = 0; p < N; ++p) {
        double v = 0.0;
        for (int q = 2; q < 5; ++q) {
            const long long c = ilu_col(A, p, q);
            if (c >= 0) v += LU[q * N + p] * x[c];
        }
        w[p] = v;
    }
    for (long long p = 0; p < N; ++p) {
        double v = w[p];
        for (int q = 0; q < 2; ++q) {
            const long long c = ilu_col(A, p, q);
            if (c >= 0) v += LU[q * N + p] * w[c];
        }
        y[p] = v;
    }
    free(w);
}

/* Shared frame of the right-preconditioned solves: factor, u = L U x, run the
 * method on A (L U)^{-1}, x = (L U)^{-1} u. */
typedef int (*orc_rp_method)(const orc_stencil *B, const double *f, double *u, void *args,
                             orc_result *res, double *hist, int hist_cap);

static int orc_right_precond(const orc_stencil *A, const double *f, double *x,
                             orc_rp_method run, void *args, orc_result *res, double *hist,
                             int hist_cap)
{
    const long long N = orc_size(A);
    if (A->ndim != 2 || N <= 0) {
        set_result(res, ORC_ERR_ARG, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_ARG;
    }
    double *LU = malloc(sizeof(double) * 5 * N), *u = malloc(sizeof(double) * N);
    if (!LU || !u) {
        free(LU); free(u);
        set_result(res, ORC_ERR_NOMEM, 0, 0, 0, NAN, NAN, 0);
        return ORC_ERR_NOMEM;
    }
    int st = orc_ilu0_factor(A, LU);
    if (st != ORC_OK) {
        set_result(res, st, 0, 0, 0, NAN, NAN, 0);
    } else {
        orc_ilu0_mul(A, LU, x, u);
        orc_stencil B = *A;
        B.ilu = LU;
        st = run(&B, f, u, args, res, hist, hist_cap);
        orc_ilu0_solve(A, LU, u, x);
    }
    free(LU); free(u);
    return st;
}

typedef struct { int s, k, max_iters; double tol; } orc_somin_args;
typedef struct { int s, m, max_blocks; double tol; } orc_sgmres_args;

static int rp_somin(const orc_stencil *B, const double *f, double *u, void *a_, orc_result *res,
                    double *hist, int hist_cap)
{
    const orc_somin_args *a = a_;
    return orc_somin(B, f, u, a->s, a->k, a->tol, a->max_iters, ORC_BASIS_MONOMIAL, res, hist,
                     hist_cap, NULL);
}

static int rp_sgmres(const orc_stencil *B, const double *f, double *u, void *a_, orc_result *res,
                     double *hist, int hist_cap)
{
    const orc_sgmres_args *a = a_;
    return orc_sgmres(B, f, u, a->s, a->m, a->tol, a->max_blocks, ORC_BASIS_MONOMIAL, res, hist,
                      hist_cap, NULL);
}

int orc_somin_ilu0(const orc_stencil *A, const double *f, double *x, int s, int k, double tol,
                   int max_iters, orc_result *res, double *hist, int hist_cap)
{
    orc_somin_args a = {s, k, max_iters, tol};
    return orc_right_precond(A, f, x, rp_somin, &a, res, hist, hist_cap);
}

int orc_sgmres_ilu0(const orc_stencil *A, const double *f, double *x, int s, int m, double tol,
                    int max_blocks, orc_result *res, double *hist, int hist_cap)
{
    orc_sgmres_args a = {s, m, max_blocks, tol};
    return orc_right_precond(A, f, x, rp_sgmres, &a, res, hist, hist_cap);
}
