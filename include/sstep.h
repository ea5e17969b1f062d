/*
 * sstep.h -- C ABI of the MI355X (gfx950) s-step Krylov solver library
 * (libsstep.so).
 *
 * Methods (Chronopoulos & Kim, "s-Step Orthomin and GMRES implemented on
 * parallel computers", arXiv 2001.04886):
 *   - s-step Orthomin(k)   (Sec. 3, Alg. 3.1)
 *   - s-step GMRES(m)      (Sec. 4, Alg. 4.1 s-step Arnoldi, eqs. (4)-(8),
 *                           Alg. 4.2 restarted s-step GMRES)
 * for the linear system A x = f (Sec. 1, eq. (1)) with A a matrix-free
 * 5-point (2-D) or 7-point (3-D) finite-difference stencil (Sec. 1 and 5).
 *
 * Conventions that hold for every entry point:
 *   - Every N-length array is a DEVICE pointer owned by the caller, FP64,
 *     contiguous, 16-byte aligned, x-fastest lexicographic order
 *     p = i + nx*(j + ny*l).  Column blocks (primitives) have an even stride.
 *     The library never frees caller memory and keeps no pointer after the
 *     call returns.
 *   - Host structs are read only during the call.
 *   - All GPU work is enqueued on opt->stream (a hipStream_t; NULL = the
 *     default stream).  Solver entry points return after the work has
 *     completed; primitives (sstep_stencil_apply, sstep_kernel_*) only
 *     enqueue and return.
 *   - Return value: a status code (sstep_status); also written to
 *     info->status when info is given.  Arguments are validated before any
 *     launch.  No exception crosses the boundary.
 *   - Calls on different streams are independent; the library holds no
 *     mutable global state besides a lazily created per-device stream-less
 *     kernel configuration and the per-GPU scratch array of
 *     sstep_gmres_solve_noalloc (shared by that entry point's calls only).
 */
#ifndef SSTEP_H
#define SSTEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSTEP_OK = 0,               /* converged: ||f - A x|| <= tol ||f|| (true residual, FP64) */
    SSTEP_NOT_CONVERGED = 1,    /* iteration cap reached; x holds the last iterate          */
    SSTEP_ERR_ARG = -1,         /* invalid argument; nothing was launched                   */
    SSTEP_ERR_BREAKDOWN = -2,   /* s-Omin: Gram matrix W_i of a direction block is zero     */
    SSTEP_ERR_NONFINITE = -3,   /* NaN / Inf in a residual or estimate; x holds the last
                                   finite iterate of the previous restart                    */
    SSTEP_ERR_HIP = -4,         /* a HIP runtime call failed                                 */
    SSTEP_ERR_NOMEM = -5        /* workspace too small / allocation failed                   */
} sstep_status;

/* Matrix-free stencil operator A (Sec. 1, Sec. 5).
 * Row p of A x sums c[q] * x[neighbour q] over the neighbours inside the grid
 * (neighbours outside are dropped: homogeneous Dirichlet) plus c[0] * x[p].
 * Coefficient order: 0 centre, 1 -x, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z.
 * If coef != NULL it is a DEVICE array [7][N] of per-point coefficients in
 * the same order (variable coefficients) and c[] is ignored.
 * Sizes: nx, ny (and nz) >= 1 and N = nx * ny * nz <= 2^31 - 1 grid points
 * (16 GiB per FP64 vector; 1290^3 is the largest cube); a larger or empty
 * grid is SSTEP_ERR_ARG before anything is launched. Unknowns are numbered
 * x fastest: p = i + nx * (j + ny * l). */
typedef struct {
    int32_t ndim;               /* 2 or 3                                         */
    int32_t nx, ny, nz;         /* interior points per axis; nz ignored for ndim 2 */
    double c[7];
    const double *coef;         /* optional DEVICE [7][N]                          */
} sstep_stencil;

/* Krylov basis of the matrix-powers kernel (all span the same space):
 * monomial y_j = A y_{j-1} / sigma; Chebyshev three-term recurrence on the
 * spectral interval [c - d, c + d]; Newton y_j = (A - th_{j-1}) y_{j-1} / d
 * with th the s Chebyshev points of that interval in Leja order (the
 * larger-s stabilisation; s-Omin and s-GMRES, not the batched solver). */
enum { SSTEP_BASIS_MONOMIAL = 0, SSTEP_BASIS_CHEBYSHEV = 1, SSTEP_BASIS_NEWTON = 2 };
enum { SSTEP_FP64 = 0, SSTEP_MIXED = 1 };
enum { SSTEP_METHOD_OMIN = 0, SSTEP_METHOD_GMRES = 1 };
enum { SSTEP_PRECOND_NONE = 0, SSTEP_PRECOND_ILU0 = 1 };
enum { SSTEP_ORTH_CHOL = 0, SSTEP_ORTH_MGS = 1 };

typedef struct {
    int32_t max_iters;    /* s-Omin: s-step iterations; s-GMRES: s-blocks over all cycles;
                             0 = 10000                                                     */
    int32_t precision;    /* SSTEP_FP64, or SSTEP_MIXED (s-GMRES only): basis vectors,
                             matrix powers and block updates in FP32; Gram matrices,
                             small solves, Hessenberg least squares, x and the restart
                             residual in FP64 (iterative refinement by restarts)           */
    int32_t basis;        /* SSTEP_BASIS_MONOMIAL (y_j = A y_{j-1} / sigma),
                             SSTEP_BASIS_CHEBYSHEV or SSTEP_BASIS_NEWTON (same Krylov
                             span, better conditioned)                                    */
    int32_t profile;      /* 1: time each kernel class with HIP events into info           */
    double sigma;         /* power scaling; 0 = smallest power of two >= Gershgorin bound */
    double inner_tol;     /* SSTEP_MIXED: a cycle stops once its least-squares residual
                             falls below inner_tol * (its starting residual); 0 = 1e-5     */
    void *workspace;      /* optional caller-owned DEVICE workspace (256-byte aligned) of
                             at least sstep_workspace_bytes(); NULL = allocated per call  */
    size_t workspace_bytes;
    void *stream;         /* hipStream_t                                                   */
    /* batched solver only (sstep_batch_plan_create): launch shape of the
       persistent kernel; 0 = defaults (512 threads, 1 workgroup per CU, no teams) */
    int32_t batch_threads;     /* 256, 512 or 1024 threads per workgroup               */
    int32_t batch_wgs_per_cu;  /* resident workgroups per compute unit (1..4)          */
    int32_t batch_graph;       /* 1: capture the launch in a hipGraph, replay it       */
    int32_t batch_team;        /* 1, 2, 4 or 8 workgroups solving one large system
                                  together (systems of >= 16384 points per member)   */
    /* single-system solvers: SSTEP_PRECOND_ILU0 runs the method on the right-
       preconditioned system A M^{-1} u = f, u = M x, M the ILU(0) factors of A
       (Sec. 5); 2-D only, nx <= 1024, FP64, monomial basis; sigma 0 means 1.
       A caller-owned workspace must hold sstep_workspace_bytes() +
       sstep_precond_workspace_bytes() bytes. */
    int32_t precond;
    /* s-Omin only (ERR_ARG for s-GMRES): SSTEP_ORTH_CHOL solves Scalar1 /
       Scalar2 with the Cholesky factor of W (the paper's Alg. 3.1);
       SSTEP_ORTH_MGS makes every new direction block A^T A-orthogonal by
       modified Gram-Schmidt first, so W is diagonal -- the variant Sec. 3
       proposes for larger s.  A column whose remaining squared length falls
       to 1e-14 of its length before the block's orthogonalisation is set to
       zero (the block is truncated there). */
    int32_t orth;
    /* s-GMRES: 1 captures the launches of a restart cycle in a hipGraph on
       first use and replays it for every later cycle (fewer launch gaps on
       small grids); ignored with profile = 1 */
    int32_t graph;
    /* batched solver only: stored-block columns each wave takes per pass of
       the block Gram (the Gram's column tile): 0 = default (4 for s <= 4,
       2 for s <= 8); s <= 4 accepts 2 or 4, s <= 8 accepts 1 or 2, any
       other value makes sstep_batch_plan_create return SSTEP_ERR_ARG */
    int32_t batch_gram_cols;
} sstep_options;

/* kernel classes reported in sstep_info (index into the arrays below) */
enum {
    SSTEP_K_MPK = 0,      /* matrix powers                                            */
    SSTEP_K_GRAM = 1,     /* block Gram against the stored blocks (partial + reduce)  */
    SSTEP_K_UPDATE = 2,   /* block update against the stored blocks                   */
    SSTEP_K_RESID = 3,    /* true residual r = f - A x                                */
    SSTEP_K_SCALAR = 4,   /* small FP64 solves                                        */
    SSTEP_K_VEC = 5,      /* short vector passes: block self-Gram, next start vector,
                             solution assembly, x / r updates, norms                  */
    SSTEP_K_NCLASS = 6
};

typedef struct {
    int32_t status;
    int32_t iters;        /* s-Omin: s-step iterations; s-GMRES: s-blocks built            */
    int32_t cycles;       /* s-GMRES: restart cycles; s-Omin: recurrence restarts + 1     */
    int32_t matvecs;      /* applications of A                                             */
    double rel_resid;     /* true ||f - A x|| / ||f|| at exit (FP64)                       */
    double rel_resid_est; /* last least-squares / recurrence estimate / ||f||              */
    double sigma;         /* scaling used                                                  */
    double cheb_centre, cheb_half_width;   /* Chebyshev interval used (basis 1)            */
    double ms_total;      /* wall time of the call (HIP events on the stream)              */
    /* with profile = 1: per kernel class launches, summed duration and the
       algorithmic bytes (each vector element read or written once) */
    int64_t launches[SSTEP_K_NCLASS];
    double ms[SSTEP_K_NCLASS];
    double bytes[SSTEP_K_NCLASS];
} sstep_info;

/* Fill *opt with the defaults (all zero / NULL). */
void sstep_default_options(sstep_options *opt);

/* Human-readable name of a status code (static string). */
const char *sstep_status_string(int status);

/* Device workspace (bytes) a solve needs for this operator and parameters.
 * method: SSTEP_METHOD_OMIN (k_or_m = k) or SSTEP_METHOD_GMRES (k_or_m = m).
 * Returns 0 for invalid arguments. */
size_t sstep_workspace_bytes(const sstep_stencil *A, int method, int s, int k_or_m,
                             int precision);

/* Restarted s-step GMRES(m) (Sec. 4, Alg. 4.2).  Solves A x = f.
 *   f   : DEVICE [N] right-hand side (read only)
 *   x   : DEVICE [N] initial guess x0 on entry, solution on exit
 *   s   : block size, 1 <= s <= 16 (s = 1 is standard GMRES(m))
 *   m   : s-blocks per restart cycle, 1 <= m; Krylov dimension m*s <= 2048
 *   tol : relative tolerance on the true residual, >= 0
 * One cycle: r0 = f - A x0, w_1 = r0/||r0||; per block k the matrix powers
 * of w_k, one Gram of all inner products against the previous blocks, the
 * block update (Scalar1/Scalar2 solved on the device in FP64), the next
 * normalised start vector w_{k+1}, one Hessenberg block column and its Givens
 * rotations; exit at m blocks, when the least-squares residual reaches tol, or
 * on breakdown; x = x0 + V y (eq. (8)).  Returns SSTEP_OK, SSTEP_NOT_CONVERGED
 * (max_iters blocks built) or an error. */
int sstep_gmres_solve(const sstep_stencil *A, const double *f, double *x, int s, int m,
                      double tol, const sstep_options *opt, sstep_info *info);

/* Largest workspace sstep_gmres_solve_noalloc serves (bytes): 128 MiB, the
 * size of the library's static per-GPU scratch array.  For example s-GMRES
 * (m = 30, s = 8) on a 256 x 256 grid needs about 127 MB. */
#define SSTEP_NOALLOC_MAX_WORKSPACE ((size_t)134217728)

/* sstep_gmres_solve for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid allocation): the same method, kernels
 * and results, with the workspace taken from a static device array of
 * SSTEP_NOALLOC_MAX_WORKSPACE bytes that the library holds on every GPU it
 * runs on until the process ends.  No hipMalloc / hipFree, no event or
 * stream creation.  Arguments as sstep_gmres_solve, plus:
 *   - opt->workspace must be NULL, opt->profile and opt->graph 0
 *     (SSTEP_ERR_ARG otherwise); info->ms_total is not measured (0);
 *   - a solve whose workspace (sstep_workspace_bytes, plus
 *     sstep_precond_workspace_bytes with ILU(0)) exceeds
 *     SSTEP_NOALLOC_MAX_WORKSPACE returns SSTEP_ERR_NOMEM before anything is
 *     launched; x is then untouched.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 * (other host threads, other streams) race and must be serialised by the
 * caller.  The solve never reads workspace it has not written in the same
 * call, so nothing has to be cleared between calls.  The call synchronises
 * opt->stream once per restart cycle, like sstep_gmres_solve. */
int sstep_gmres_solve_noalloc(const sstep_stencil *A, const double *f, double *x, int s, int m,
                              double tol, const sstep_options *opt, sstep_info *info);

/* s-step Orthomin(k) (Sec. 3, Alg. 3.1).  Solves A x = f.
 *   s : block size 1..16 (s = 1 is Omin(k));  k : window of previous
 *   direction blocks, 1 <= k <= 64 (k >= iterations gives s-step GCR).
 * Per iteration: W_i = AP_i^T AP_i, m_i = AP_i^T r_i, a_i = W_i^{-1} m_i,
 * x += P_i a_i, r -= AP_i a_i; matrix powers of r give R, AR; C_j = AP_j^T AR,
 * B_j = -W_j^{-1} C_j; P_{i+1} = R + sum P_j B_j, AP_{i+1} = AR + sum AP_j B_j.
 * The recurrence residual triggers a true-residual check; on failure r is
 * replaced by the true residual and the window restarts.
 * precision must be SSTEP_FP64. */
int sstep_omin_solve(const sstep_stencil *A, const double *f, double *x, int s, int k,
                     double tol, const sstep_options *opt, sstep_info *info);

/* ---------------------------------------------------------------------- */
/* ILU(0) right preconditioning (Sec. 5)                                   */
/* ---------------------------------------------------------------------- */

/* The paper solves the right-preconditioned form [A K] K^{-1} x = f with K
 * the inverse of the ILU(0) factors of A.  For a 2-D five-point matrix in
 * the natural ordering (x fastest) ILU(0) keeps A's off-diagonal entries and
 * changes only the pivots:
 *   M = L U = (D + Lo) D^{-1} (D + Up),
 *   d_p = a_pp - a_{p,p-nx} a_{p-nx,p} / d_{p-nx} - a_{p,p-1} a_{p-1,p} / d_{p-1},
 * with Lo / Up the strictly lower / upper parts of A (neighbours outside the
 * grid dropped).  The triangular sweeps run over anti-diagonals on one wave
 * of the device (latency bound: about nx + ny steps in sequence).
 * Requirements for all three calls: A 2-D (ERR_ARG otherwise),
 * 1 <= nx <= 1024, N * 8 < 2^31; every array a DEVICE array, 8-byte aligned,
 * caller-owned; the call is asynchronous on `stream` except where noted. */

/* Device workspace (bytes) that precond adds to a solve (0 for
 * SSTEP_PRECOND_NONE or an unsupported operator). */
size_t sstep_precond_workspace_bytes(const sstep_stencil *A, int precond);

/* d : DEVICE [2N]; d[0..N) receives the pivots d_p, d[N..2N) their
 * reciprocals.  Synchronises `stream`; returns SSTEP_ERR_BREAKDOWN if a
 * pivot is zero or not finite. */
int sstep_ilu0_factor(const sstep_stencil *A, double *d, void *stream);

/* z = M^{-1} r (forward then backward sweep).  d as written by
 * sstep_ilu0_factor; r, z : DEVICE [N], z must not alias r or d.  Allocates
 * (stream-ordered) and frees a scratch buffer for the sweep layout of d and
 * the coefficients on every call; the solvers keep theirs in the workspace. */
int sstep_ilu0_solve(const sstep_stencil *A, const double *d, const double *r, double *z,
                     void *stream);

/* u = M x.  d as written by sstep_ilu0_factor; x, u : DEVICE [N], distinct. */
int sstep_ilu0_mul(const sstep_stencil *A, const double *d, const double *x, double *u,
                   void *stream);

/* ---------------------------------------------------------------------- */
/* Batched s-step GMRES: many independent systems in one persistent launch */
/* ---------------------------------------------------------------------- */

/* Opaque plan: system table on the device, per-system basis workspace and
 * (with opt->batch_graph) the captured hipGraph of the launch. */
typedef struct sstep_batch_plan_s *sstep_batch_plan;

/* Device workspace (bytes) of a batch plan (sum of the systems' bases plus
 * per-workgroup dense state). */
size_t sstep_batch_workspace_bytes(int nsys, const sstep_stencil *A, int s, int m,
                                   const sstep_options *opt);

/* Create a plan for nsys independent systems A[i] x[i] = f[i] (restarted
 * s-step GMRES(m), Sec. 4, Alg. 4.2, FP64, monomial basis).
 *   A    : HOST array [nsys] of stencils, constant coefficients or per-point
 *          ones (coef: DEVICE [7][N], valid for the life of the plan)
 *   f, x : HOST arrays [nsys] of DEVICE pointers (x: initial guess in, solution
 *          out at every execution; the pointers must stay valid for the plan)
 *   s    : 1..8;  m: s-blocks per cycle, m <= 128 and m*s <= 512
 * One persistent kernel of (compute units x batch_wgs_per_cu) workgroups;
 * each workgroup takes systems from a queue (largest first) and runs a whole
 * solve with workgroup-local synchronisation only.  Returns SSTEP_OK or an
 * error; *plan is NULL on error. */
int sstep_batch_plan_create(sstep_batch_plan *plan, int nsys, const sstep_stencil *A,
                            const double *const *f, double *const *x, int s, int m, double tol,
                            const sstep_options *opt);

/* Run the plan once (replays the graph when captured) and wait.  info: HOST
 * array [nsys] or NULL; ms_total of every entry is the batch wall time.
 * Returns SSTEP_OK if every system converged, SSTEP_NOT_CONVERGED if any hit
 * the cap, or the first error. */
int sstep_batch_plan_execute(sstep_batch_plan plan, sstep_info *info);

/* Free the plan (and its workspace if the library allocated it). */
void sstep_batch_plan_destroy(sstep_batch_plan plan);

/* Convenience: create, execute once, destroy. */
int sstep_gmres_solve_batched(int nsys, const sstep_stencil *A, const double *const *f,
                              double *const *x, int s, int m, double tol,
                              const sstep_options *opt, sstep_info *info);

/* ---------------------------------------------------------------------- */
/* Primitives (the building blocks of the solvers; enqueue only)           */
/* ---------------------------------------------------------------------- */

/* y = A x (Sec. 1 operator).  x, y DEVICE [N], must not alias. */
int sstep_stencil_apply(const sstep_stencil *A, const double *x, double *y, void *stream);

/* Matrix-powers kernel (Sec. 3-4: the s directions from one vector).
 * Y: DEVICE, s+1 columns of N doubles with column stride ldy >= N; column 0
 * is the input w (read), columns 1..s are written:
 *   basis 0: y_0 = w * in_scale, y_j = A y_{j-1} / sigma
 *   basis 1: y_1 = (A - c) y_0 / d, y_{j+1} = 2 (A - c) y_j / d - y_{j-1}
 * Column 0 itself is not rewritten (it keeps w; y_0 is w * in_scale).
 * Always the fused (several levels per pass) kernel, whatever the grid size;
 * the solvers switch to one stencil launch per level on small grids. */
int sstep_kernel_mpk(const sstep_stencil *A, double *Y, int64_t ldy, int s, int basis,
                     double in_scale, double sigma, double cheb_c, double cheb_d,
                     void *stream);

/* Block Gram G = X^T Z accumulated in FP64 with a fixed reduction order
 * (Sec. 3-4: all inner products of one s-step at once).
 *   X: DEVICE, ncx columns of N doubles, stride ldx;  Z: DEVICE, ncz <= 16
 *   columns, stride ldz;  G: DEVICE ncx x ncz, row-major (G[c*ncz + j]).
 * The result is deterministic for fixed (N, ncx, ncz). */
int sstep_kernel_gram(const double *X, int64_t ldx, int ncx, const double *Z, int64_t ldz,
                      int ncz, int64_t N, double *G, void *stream);

/* Block update Y[:, l] += sum_c X[:, c] * M[c*ncy + l]  (l < ncy <= 16)
 * (Sec. 3-4 linear combinations).  X: DEVICE ncx columns, stride ldx;
 * Y: DEVICE ncy columns, stride ldy (updated in place; may not overlap X);
 * M: DEVICE ncx x ncy row-major FP64 coefficients.  X and M may be NULL when
 * ncx == 0. */
int sstep_kernel_update(const double *X, int64_t ldx, int ncx, double *Y, int64_t ldy,
                        int ncy, const double *M, int64_t N, void *stream);

/* ------------------------------------------------------------------------
 * Learned initial guess.  Alg 4.2 restarts from whatever x0 it is given; the
 * network below proposes one from the problem data of the variable-
 * coefficient diffusion family  -div(k grad u) = f  on an nx x ny grid
 * (extension beyond the paper, which always starts from a fixed x0).
 *
 * Network: input channels (log k, f / rms(f)) per grid point, rms over the
 * grid of one sample; four dilated 3x3 convolutions with channels
 * 2 -> 32 -> 32 -> 32 -> 1, dilations 1, 2, 4, 8, zero padding equal to the
 * dilation, ReLU after the first three; x0 = out * rms(f) * out_scale.
 * Training loss: mean over all points of the batch of
 * (out - x / (rms(f) * out_scale))^2; optimiser Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected).
 *
 * params: DEVICE float[sstep_cnn_param_count()] = 19393, layer by layer
 * W_l[Cout][Cin][3][3] then b_l[Cout].  Activations are stored in bf16 with
 * FP32 accumulation; the two 32 -> 32 layers run on bf16 matrix cores.
 *
 * Batched arrays are DEVICE [batch][ny][nx] (x fastest), 16-byte aligned:
 * logk float, f and x double.  Every call enqueues on opt->stream and returns
 * after completion.  Workspace: opt->workspace of at least
 * sstep_cnn_workspace_bytes(batch, nx, ny, training) bytes (16-byte aligned),
 * or NULL for a temporary allocation.  Errors: SSTEP_ERR_ARG for bad sizes,
 * pointers, alignment or a non-positive out_scale / lr; SSTEP_ERR_NOMEM,
 * SSTEP_ERR_HIP.  The caller owns every pointer.
 * ---------------------------------------------------------------------- */
size_t sstep_cnn_param_count(void);
size_t sstep_cnn_workspace_bytes(int batch, int nx, int ny, int training);

/* Forward pass: out (float [batch][ny][nx], raw network output, may be NULL)
 * and/or x0 (double, the scaled guess, may be NULL; not both NULL). */
int sstep_cnn_forward(const float *params, double out_scale, int batch, int nx, int ny,
                      const float *logk, const double *f, float *out, double *x0,
                      const sstep_options *opt);

/* Loss (HOST double, may be NULL) and its gradient grad (DEVICE float
 * [param_count]) for targets x (the solutions of the batch). */
int sstep_cnn_gradient(const float *params, double out_scale, int batch, int nx, int ny,
                       const float *logk, const double *f, const double *x, float *grad,
                       double *loss, const sstep_options *opt);

/* One Adam step (step >= 1 counts updates, for the bias correction) on
 * params with moments m, v (DEVICE float[param_count], zero before step 1). */
int sstep_cnn_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                   const sstep_options *opt);

/* sstep_cnn_gradient followed by sstep_cnn_adam, sharing the workspace. */
int sstep_cnn_train_step(float *params, float *m, float *v, int step, float lr,
                         double out_scale, int batch, int nx, int ny, const float *logk,
                         const double *f, const double *x, double *loss,
                         const sstep_options *opt);

/* Initial guess for one 2-D system A x = f (A: ndim 2, stencil of the same
 * grid; logk and f DEVICE [ny][nx]).  With use_fallback != 0, x0 is reset to
 * 0 when ||f - A x0|| >= ||f|| and *used_fallback (HOST, may be NULL) says so. */
int sstep_x0_predict(const float *params, double out_scale, const sstep_stencil *A,
                     const float *logk, const double *f, double *x0, int use_fallback,
                     int *used_fallback, const sstep_options *opt);

/* Block averages: out[b][J][I] = mean of the factor x factor block of
 * in[b][ny][nx] with corner (factor J, factor I); sums in FP64.  in, out
 * DEVICE doubles, out [batch][ny/factor][nx/factor]; nx and ny must be
 * multiples of factor (else SSTEP_ERR_ARG).  Enqueued on stream; returns after
 * completion.  (Used to build the coarse inputs and targets of the network
 * below from fine-grid data.) */
int sstep_grid_pool(const double *in, double *out, int batch, int nx, int ny, int factor,
                    void *stream);

/* Coarse-grid initial guess for one 2-D system A x = f on an nx x ny grid
 * (nx, ny multiples of factor).  log k and f are block-averaged over
 * factor x factor cells (as sstep_grid_pool; log k summed in FP64, stored as
 * float); the network above runs on the (ny/factor) x (nx/factor) coarse grid,
 * where its receptive field of 31 points spans a factor-times larger part of
 * the domain; its guess (out * rms(pooled f) * out_scale) is interpolated
 * bilinearly onto the fine grid, coarse values sitting at the block centres
 * (fine point i at coarse coordinate (i + 1/2)/factor - 1/2, clamped to the
 * coarse grid); then `sweeps` damped Jacobi sweeps x += 0.8 (f - A x)/diag(A)
 * remove the interpolation's high-frequency error; then the fallback test of
 * sstep_x0_predict if use_fallback != 0.  params / out_scale: a model trained
 * on block-averaged data of the same factor.  Workspace: opt->workspace of at
 * least sstep_x0_coarse_workspace_bytes(nx, ny, factor) bytes or NULL.
 * Errors as sstep_x0_predict; factor < 1, nx or ny not a multiple of factor,
 * or sweeps outside 0..100000 give SSTEP_ERR_ARG. */
size_t sstep_x0_coarse_workspace_bytes(int nx, int ny, int factor);
int sstep_x0_predict_coarse(const float *params, double out_scale, int factor, int sweeps,
                            const sstep_stencil *A, const float *logk, const double *f,
                            double *x0, int use_fallback, int *used_fallback,
                            const sstep_options *opt);

#ifdef __cplusplus
}
#endif
#endif
