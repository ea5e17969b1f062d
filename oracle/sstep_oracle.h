/*
 * sstep_oracle.h -- plain, slow, FP64 CPU oracle for the s-step Orthomin(k)
 * and s-step GMRES(m) methods of Chronopoulos & Kim, "s-Step Orthomin and
 * GMRES implemented on parallel computers" (arXiv 2001.04886).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the GPU library never calls it.
 *
 * Every routine is single-threaded, sums in index order, and keeps all
 * vectors in host memory as plain double arrays.
 */
#ifndef SSTEP_ORACLE_H
#define SSTEP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Matrix-free operator of a 5-point (2-D) or 7-point (3-D) stencil on an
 * nx*ny*nz interior grid, unknown index p = i + nx*(j + ny*l) (x fastest).
 * Coefficient order: centre, -x, +x, -y, +y, -z, +z.  Neighbours outside the
 * grid are dropped (homogeneous Dirichlet).  If coef != NULL it is a
 * [7][N] per-point array in the same order and c[] is ignored. */
typedef struct {
    int ndim;
    int nx, ny, nz;
    double c[7];
    const double *coef;
    /* optional ILU(0) factors of this operator (orc_ilu0_factor layout).  If
     * set, the operator is the right-preconditioned A (L U)^{-1} of Sec. 5. */
    const double *ilu;
} orc_stencil;

/* basis of the s-dimensional Krylov block */
enum { ORC_BASIS_MONOMIAL = 0, ORC_BASIS_CHEBYSHEV = 1, ORC_BASIS_NEWTON = 2 };

/* Shifts of the Newton basis (the larger-s stabilisation of Sec. 3-4): the s
 * Chebyshev points centre + half_width cos((2k+1) pi / (2s)), k = 0..s-1, of
 * the spectral interval, in Leja order (first the point of largest modulus,
 * then each time the point maximising the product of distances to those
 * already taken; ties to the smaller k).  th: [s]. */
void orc_newton_shifts(int s, double centre, double half_width, double *th);

/* status codes (same meaning as the GPU library's, independently defined) */
enum {
    ORC_OK = 0,
    ORC_NOT_CONVERGED = 1,
    ORC_ERR_ARG = -1,
    ORC_ERR_BREAKDOWN = -2,
    ORC_ERR_NONFINITE = -3,
    ORC_ERR_NOMEM = -5
};

typedef struct {
    int status;
    int iters;      /* Omin: (s-)steps; GMRES: Arnoldi steps (standard) or s-blocks (s-step) */
    int cycles;     /* GMRES restart cycles started; Omin: residual replacements + 1 */
    int matvecs;
    double rel_resid;     /* true ||f - A x|| / ||f|| at exit */
    double rel_resid_est; /* last recurrence / least-squares estimate / ||f|| */
    int nhist;            /* entries written to hist */
} orc_result;

/* optional per-cycle inspection buffers (any pointer may be NULL) */
typedef struct {
    double *V;      /* [(ms+1)][N]  basis columns actually used, normalised (U_k)  */
    double *G;      /* [(ms+1)][ms] column-major Hessenberg Gbar, leading dim ms+1 */
    double *D;      /* [(ms+1)][(ms+1)] column-major D = U^T U (block diagonal)    */
    int ncols;      /* number of basis columns in the least-squares problem        */
    int blocks;     /* s-blocks built in the cycle                                 */
} orc_cycle_dump;

/* Inspection of the final s-Omin window (any pointer may be NULL). */
typedef struct {
    double *P;      /* [k*s][N] direction blocks, oldest first */
    double *AP;     /* [k*s][N] their images                  */
    double *r;      /* [N] recurrence residual                 */
    int nblocks;    /* blocks written                          */
} orc_omin_dump;

long long orc_size(const orc_stencil *A);
void orc_apply(const orc_stencil *A, const double *x, double *y);
double orc_sigma(const orc_stencil *A);
void orc_cheb_interval(const orc_stencil *A, double *centre, double *half_width);
void orc_mpk(const orc_stencil *A, const double *y0, int s, int basis, double sigma,
             double centre, double half_width, double *Y);

int orc_gmres(const orc_stencil *A, const double *f, double *x, int M, double tol,
              int max_steps, orc_result *res, double *hist, int hist_cap,
              double *Q_out, double *H_out);
int orc_omin(const orc_stencil *A, const double *f, double *x, int k, double tol,
             int max_iters, orc_result *res, double *hist, int hist_cap);
int orc_somin(const orc_stencil *A, const double *f, double *x, int s, int k, double tol,
              int max_iters, int basis, orc_result *res, double *hist, int hist_cap,
              orc_omin_dump *dump);
/* orc_somin with mgs = 1: every new direction block is made A^T A-orthogonal
 * by modified Gram-Schmidt (Sec. 3, the larger-s variant), so Scalar1 and
 * Scalar2 see diagonal W. */
int orc_somin_ex(const orc_stencil *A, const double *f, double *x, int s, int k, double tol,
                 int max_iters, int basis, int mgs, orc_result *res, double *hist, int hist_cap,
                 orc_omin_dump *dump);
int orc_sgmres(const orc_stencil *A, const double *f, double *x, int s, int m, double tol,
               int max_blocks, int basis, orc_result *res, double *hist, int hist_cap,
               orc_cycle_dump *dump);

/* ILU(0) right preconditioning (Sec. 5: [A K] K^{-1} x = f with K the inverse
 * of the incomplete factors, ILU(0) as the paper's preconditioner).  2-D
 * five-point operators only.  LU is [5][N]; row p keeps the entries of the
 * factors in the five columns of A's pattern, slot 0: p - nx, 1: p - 1,
 * 2: p, 3: p + 1, 4: p + nx (0 where the column lies outside the grid).
 * Slots 0-1 are L (unit diagonal implied), slots 2-4 are U.
 * orc_ilu0_factor returns ORC_OK, ORC_ERR_ARG (not 2-D) or ORC_ERR_BREAKDOWN
 * (a zero pivot). */
int orc_ilu0_factor(const orc_stencil *A, double *LU);
void orc_ilu0_solve(const orc_stencil *A, const double *LU, const double *r, double *z);
void orc_ilu0_mul(const orc_stencil *A, const double *LU, const double *x, double *y);
/* s-step methods on the right-preconditioned system: u = L U x, the method
 * runs on A (L U)^{-1} u = f, then x = (L U)^{-1} u.  Monomial basis only
 * (ORC_ERR_ARG otherwise); residuals reported are true residuals f - A x. */
int orc_somin_ilu0(const orc_stencil *A, const double *f, double *x, int s, int k, double tol,
                   int max_iters, orc_result *res, double *hist, int hist_cap);
int orc_sgmres_ilu0(const orc_stencil *A, const double *f, double *x, int s, int m, double tol,
                    int max_blocks, orc_result *res, double *hist, int hist_cap);

#ifdef __cplusplus
}
#endif
#endif
