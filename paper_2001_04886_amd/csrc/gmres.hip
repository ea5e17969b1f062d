// gmres.hip -- restarted s-step GMRES(m) (Sec. 4: Alg. 4.1 s-step Arnoldi,
// eqs. (4)-(8) least squares, Alg. 4.2 restarts) on one GPU.
//
// Storage.  The basis holds m*s+1 columns (FP64, or FP32 in mixed precision).
// Column k*s is the start of block k as produced (unnormalised: the residual
// r0 for block 0, the projected vector w_hat for later blocks); its norm
// nu_k is kept in device state and 1/nu_k is applied when the column is read
// by the matrix-powers kernel and folded into the coefficients of every other
// consumer.  The matrix-powers kernel writes y_1..y_s into columns
// k*s+1..k*s+s, which are then projected in place; column k*s+s ends up as the
// start of block k+1.  Nothing is copied.
//
// Per block k (all on the device; the host only enqueues):
//   MPK        y_j = A y_{j-1} / sigma (or Chebyshev), y_0 = w_k
//   Gram       C = [Vbar_1..Vbar_{k-1}]^T [y_1..y_s]
//   scalar     T_i = W_i^{-1} C_i                    (Scalar2)
//   update     y_j -= sum_i Vbar_i T_i[:, j]          (one pass, in place)
//   Gram       [w_k, y_1..y_s]^T [w_k, y_1..y_s]      (W_k, Vbar_k^T Yhat_s)
//   scalar     factor W_k, g = W_k^{-1} Vbar_k^T Yhat_s   (Scalar1)
//   update     w_hat = Yhat_s - Vbar_k g, nu_k^2 = ||w_hat||^2
//   scalar     Hessenberg block column, L scaling, Givens, residual estimate
// A done flag in device state makes the remaining launches of a cycle return
// at once after the least-squares residual reaches the tolerance or the
// Krylov space breaks down; the host synchronises once per cycle.
#include <hip/hip_runtime.h>

#include <functional>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.hpp"
#include "launch.hpp"
#include "solvers.hpp"

namespace sstep {

constexpr int kMaxBlocks = 2048;
constexpr int kMaxCols = 2048;  // m * s, checked at the C ABI

struct GmState {
    // parameters
    int s, m, K, ldg, basis, mixed;
    double sigma, cc, cd;
    double tol_rel, fnorm, tol_abs, inner_rel, rank_tol, lucky_tol;
    double Bc[(kMaxS + 1) * kMaxS];
    // cycle state
    double beta, est, stop_abs, yhat2, nu_cur;
    int kb, ncols, done, skip_n4b, skip_asm, active, conv, err, blocks_total, cycles, lucky;
    int asm_cols;  // columns combined by the last solution assembly
    double g[kMaxS], coefN4b[kMaxS];
    double nu[kMaxBlocks + 1], inv_nu[kMaxBlocks + 1];
};

struct GmArrays {
    GmState* st;
    double* G;       // Hessenberg Gbar, (K+1) x K column-major
    double* R;       // Givens-rotated L Gbar
    double* cs;
    double* sn;
    double* rhs;     // rotated beta e_1
    double* y;
    double* T;       // projection coefficients of the current block, [K][s+1]
    double* coefM;   // update coefficients, [K][s]
    double* coefA;   // assembly coefficients, [K]
    double* Gout;    // Gram output
    GramFactor* Wf;  // factors of W_1..W_m
};

// ---------------------------------------------------------------------------
// scalar kernels (one workgroup)
// ---------------------------------------------------------------------------

// ||f||^2 partials -> fnorm, absolute tolerance
__global__ __launch_bounds__(kThreads) void k_gm_init(GmArrays a, const double* __restrict__ part,
                                                      int npart) {
    __shared__ double lds[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < npart; i += kThreads) acc += part[i];
    double v[1] = {acc}, o[1];
    block_sum<1>(v, lds, o);
    if (threadIdx.x == 0) {
        GmState* st = a.st;
        st->fnorm = sqrt(o[0]);
        st->tol_abs = st->tol_rel * st->fnorm;
        st->blocks_total = 0;
        st->cycles = 0;
        st->conv = 0;
        st->err = 0;
    }
}

// Start of a cycle (Alg. 4.2 step 1): beta = ||r0|| from the residual
// partials; converged if beta <= tol ||f||.
__global__ __launch_bounds__(kThreads) void k_gm_cycle_start(GmArrays a,
                                                             const double* __restrict__ part,
                                                             int npart) {
    __shared__ double lds[4];
    __shared__ int go;
    GmState* st = a.st;
    double acc = 0.0;
    for (int i = threadIdx.x; i < npart; i += kThreads) acc += part[i];
    double v[1] = {acc}, o[1];
    block_sum<1>(v, lds, o);
    if (threadIdx.x == 0) {
        const double beta = sqrt(o[0]);
        st->beta = beta;
        st->kb = 0;
        // a vector load: a scalar load of ncols is not ordered before the
        // vector store that clears it below
        st->asm_cols = __atomic_load_n(&st->ncols, __ATOMIC_RELAXED);
        st->ncols = 0;
        st->lucky = 0;
        st->skip_n4b = 1;
        st->skip_asm = 1;
        go = 0;
        if (!isfinite(beta)) {
            st->err = SSTEP_ERR_NONFINITE;
            st->done = 1;
            st->active = 0;
        } else if (beta <= st->tol_abs) {
            st->conv = 1;
            st->done = 1;
            st->active = 0;
        } else {
            st->done = 0;
            st->skip_n4b = 0;
            st->skip_asm = 0;
            st->active = 1;
            st->cycles += 1;
            st->est = beta;
            st->nu[0] = beta;
            st->inv_nu[0] = 1.0 / beta;
            st->stop_abs = st->mixed ? fmax(st->tol_abs, st->inner_rel * beta) : st->tol_abs;
            go = 1;
        }
    }
    __syncthreads();
    if (go) {
        for (int i = threadIdx.x; i <= st->K; i += kThreads) a.rhs[i] = (i == 0) ? st->beta : 0.0;
    }
}

// Scalar2 (Sec. 4): T_i = W_i^{-1} C_i for every previous block i, from the
// Gram of the stored basis against y_1..y_s.  Stored column 0 of block i is
// nu_i times the normalised w_i, hence the row scaling by 1/nu_i.
__global__ __launch_bounds__(kThreads) void k_gm_proj(GmArrays a) {
    // workgroup i: the s columns of T_i, from the factor of W_i staged in LDS
    // (the triangular solves then run on LDS instead of chains of global loads)
    __shared__ GramFactor F;
    GmState* st = a.st;
    if (st->done) return;
    const int s = st->s, kb = st->kb, i = blockIdx.x;
    if (i >= kb) return;
    {
        const double* src = reinterpret_cast<const double*>(&a.Wf[i]);
        double* dst = reinterpret_cast<double*>(&F);
        for (int t = threadIdx.x; t < (int)(sizeof(GramFactor) / sizeof(double)); t += kThreads)
            dst[t] = src[t];
    }
    __syncthreads();
    const double inu = st->inv_nu[i];
    for (int l = 1 + (int)threadIdx.x; l <= s; l += kThreads) {  // Y column l
        double c[kMaxS];
        for (int q = 0; q < s; ++q) c[q] = a.Gout[(i * s + q) * s + (l - 1)] * (q == 0 ? inu : 1.0);
        gram_solve(F, c, c);
        for (int q = 0; q < s; ++q) {
            a.T[(i * s + q) * (s + 1) + l] = c[q];
            a.coefM[(i * s + q) * s + (l - 1)] = -c[q] * (q == 0 ? inu : 1.0);
            if (l == 1) a.T[(i * s + q) * (s + 1)] = 0.0;
        }
    }
}

// Scalar1 (Sec. 4): factor W_k = Vbar_k^T Vbar_k, g = W_k^{-1} Vbar_k^T Yhat_s.
// Gout is the Gram of the stored columns [w_hat_k, y_1..y_s] (s+1 square).
// A rank-deficient W_k (pivot below rank_tol) truncates the block to its
// leading q columns; column q then plays the role of Yhat_s with nu = 0.
// The factor is computed in LDS by the wave, the solves by one thread, then
// the factor is copied out.
__global__ __launch_bounds__(64) void k_gm_block(GmArrays a) {
    __shared__ GramFactor F;
    __shared__ double W[kMaxS * kMaxS];
    GmState* st = a.st;
    if (st->done) return;
    const int s = st->s, kb = st->kb, s1 = s + 1;
    const double d0 = st->inv_nu[kb];
    for (int idx = threadIdx.x; idx < s * s; idx += 64) {
        const int p = idx % s, q = idx / s;
        W[p + q * kMaxS] = a.Gout[p * s1 + q] * (p == 0 ? d0 : 1.0) * (q == 0 ? d0 : 1.0);
    }
    __syncthreads();
    gram_factor_wave(W, s, st->rank_tol, &F);  // W is overwritten
    __syncthreads();
    if (threadIdx.x == 0) {
        st->yhat2 = a.Gout[s * s1 + s];
        const int q = F.rank;
        if (q == s) {
            double h[kMaxS], g[kMaxS];
            for (int p = 0; p < s; ++p) h[p] = a.Gout[p * s1 + s] * (p == 0 ? d0 : 1.0);
            gram_solve(F, h, g);
            for (int p = 0; p < s; ++p) {
                st->g[p] = g[p];
                st->coefN4b[p] = -g[p] * (p == 0 ? d0 : 1.0);
            }
            st->skip_n4b = 0;
        } else if (q > 0) {
            double h[kMaxS], g[kMaxS];
            for (int p = 0; p < q; ++p) h[p] = a.Gout[p * s1 + q] * (p == 0 ? d0 : 1.0);
            gram_solve_leading(F, q, h, g);
            for (int p = 0; p < s; ++p) st->g[p] = p < q ? g[p] : 0.0;
            st->skip_n4b = 1;
        } else {
            st->err = SSTEP_ERR_NONFINITE;
            st->done = 1;
            st->skip_n4b = 1;
        }
    }
    __syncthreads();
    // copy the factor out
    const double* src = reinterpret_cast<const double*>(&F);
    double* dst = reinterpret_cast<double*>(&a.Wf[kb]);
    for (int i = threadIdx.x; i < (int)(sizeof(GramFactor) / sizeof(double)); i += 64) dst[i] = src[i];
}

// nu_k = ||w_hat|| from the partial sums of the N4b pass (0 for a truncated
// block) and the lucky-breakdown test.
__global__ __launch_bounds__(kThreads) void k_gm_nu(GmArrays a, const double* __restrict__ part,
                                                    int npart) {
    __shared__ double lds[4];
    GmState* st = a.st;
    if (st->done) return;
    const int s = st->s, q = a.Wf[st->kb].rank;
    const double acc = q == s ? strided_partial_sum(part, npart) : 0.0;
    double v[1] = {acc}, o[1];
    block_sum<1>(v, lds, o);
    if (threadIdx.x == 0) {
        const double nu = q == s ? sqrt(o[0]) : 0.0;
        st->nu_cur = nu;
        st->lucky = (q == s) && !(nu > st->lucky_tol * sqrt(st->yhat2));
    }
}

// Hessenberg block column (eq. (5)) and its L scaling (eq. (7)).  In
// coordinates of U = [Vbar_1 .. Vbar_k, w_{k+1}]:  Y = U Z_k with
//   Z_k = [T_1; ..; T_{k-1}; [I | g]; nu e^T],
//   Gbar[:, block k] = Z_k B - sum_{i<k} Gbar[:, block i] T_i[:, 0:s],
// then rows of block i are multiplied by the upper Cholesky factor L_i of
// W_i (D = L^T L).  Workgroup i handles the rows of block i (workgroup kb
// also the row of w_{k+1}).
__global__ __launch_bounds__(kThreads) void k_gm_hess_cols(GmArrays a) {
    // chunk of earlier basis columns staged in LDS: CH rows of T and the
    // workgroup's rows of Gbar over those columns (loaded by all threads, so
    // the long sum over earlier columns runs on LDS, not on chains of global loads)
    constexpr int CH = 128;
    __shared__ double gs[(kMaxS + 1) * kMaxS];
    __shared__ double Tl[CH * (kMaxS + 1)];
    __shared__ double Gl[(kMaxS + 1) * CH];
    __shared__ GramFactor F;
    GmState* st = a.st;
    if (st->done) return;
    const int s = st->s, kb = st->kb, c0 = kb * s, ldg = st->ldg, s1 = s + 1;
    const int q = a.Wf[kb].rank;
    const int bi = blockIdx.x;                 // row block
    const int r0 = bi * s;
    const int nr = (bi < kb) ? s : q + 1;      // rows handled
    const double nu = st->nu_cur;
    const double* Bc = st->Bc;
    {
        const double* src = reinterpret_cast<const double*>(&a.Wf[bi < kb ? bi : kb]);
        double* dst = reinterpret_cast<double*>(&F);
        for (int i = threadIdx.x; i < (int)(sizeof(GramFactor) / sizeof(double)); i += kThreads)
            dst[i] = src[i];
    }
    // Z_k B part of each entry (rr, j)
    for (int idx = threadIdx.x; idx < nr * q; idx += kThreads) {
        const int rr = idx % nr, j = idx / nr, r = r0 + rr;
        double val = 0.0;
        for (int l = 0; l <= q; ++l) {
            const double bl = Bc[l + j * s1];
            if (bl == 0.0) continue;
            double z;
            if (r < c0) z = a.T[r * s1 + l];
            else if (r < c0 + q) z = (l < q) ? (r - c0 == l ? 1.0 : 0.0) : st->g[r - c0];
            else z = (l == q) ? nu : 0.0;
            val += bl * z;
        }
        gs[rr + j * (kMaxS + 1)] = val;
    }
    // minus sum over earlier columns cp >= r - 1 of Gbar[r, cp] T[cp, j], rows r <= c0
    const int rlast = (r0 + nr - 1 < c0) ? r0 + nr - 1 : c0;  // last row taking part
    const int cstart = r0 > 0 ? r0 - 1 : 0;
    if (r0 <= c0) {
        for (int cb = cstart; cb < c0; cb += CH) {
            const int nc = (c0 - cb < CH) ? c0 - cb : CH;
            __syncthreads();
            for (int t = threadIdx.x; t < nc * s1; t += kThreads) Tl[t] = a.T[(long long)cb * s1 + t];
            for (int t = threadIdx.x; t < nc * nr; t += kThreads) {
                const int cc = t / nr, rr = t % nr;
                Gl[rr * CH + cc] = a.G[r0 + rr + (long long)(cb + cc) * ldg];
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < nr * q; idx += kThreads) {
                const int rr = idx % nr, j = idx / nr, r = r0 + rr;
                if (r > rlast) continue;
                const int lo = (r > 0 ? r - 1 : 0) - cb;
                double acc = 0.0;
                for (int cc = lo > 0 ? lo : 0; cc < nc; ++cc) acc += Gl[rr * CH + cc] * Tl[cc * s1 + j];
                gs[rr + j * (kMaxS + 1)] -= acc;
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nr * q; idx += kThreads) {
        const int rr = idx % nr, j = idx / nr;
        a.G[r0 + rr + (long long)(c0 + j) * ldg] = gs[rr + j * (kMaxS + 1)];
    }
    // L scaling: rows of block bi (rank qi), plus the unit row of w_{k+1}
    const int qi = (bi < kb) ? s : q;
    for (int idx = threadIdx.x; idx < nr * q; idx += kThreads) {
        const int rr = idx % nr, j = idx / nr;
        double val;
        if (bi == kb && rr == q) {
            val = gs[rr + j * (kMaxS + 1)];
        } else {
            val = 0.0;
            for (int b = rr; b < qi; ++b) val += gram_L(F, rr, b) * gs[b + j * (kMaxS + 1)];
        }
        a.R[r0 + rr + (long long)(c0 + j) * ldg] = val;
    }
}

// Givens QR of the new columns of L Gbar and the least-squares residual
// estimate |rhs[ncols]|; stopping tests of the block.
__global__ __launch_bounds__(64) void k_gm_givens(GmArrays a) {
    // rows c0 .. c0+q of the q new columns, their rotations and the rotated
    // rhs are worked on in LDS (read-modify-write chains through global
    // memory would wait a memory round trip per step)
    __shared__ double cw[kMaxS][kMaxS + 2];
    __shared__ double csl[kMaxS], snl[kMaxS], rh[kMaxS + 1];
    __shared__ double csa[kMaxCols], sna[kMaxCols];  // the earlier rotations
    GmState* st = a.st;
    if (st->done) return;
    const int s = st->s, kb = st->kb, c0 = kb * s, ldg = st->ldg;
    const int q = a.Wf[kb].rank;
    for (int i = threadIdx.x; i < c0; i += 64) {
        csa[i] = a.cs[i];
        sna[i] = a.sn[i];
    }
    __syncthreads();
    if ((int)threadIdx.x < q) {  // earlier rotations, one thread per new column
        double* col = a.R + (long long)(c0 + threadIdx.x) * ldg;
        double x0 = col[0];
#pragma unroll 16
        for (int i = 0; i < c0; ++i) {
            const double cth = csa[i], sth = sna[i], x1 = col[i + 1];
            col[i] = cth * x0 + sth * x1;
            x0 = -sth * x0 + cth * x1;
        }
        cw[threadIdx.x][0] = x0;
        for (int t = 1; t <= q; ++t) cw[threadIdx.x][t] = col[c0 + t];
    }
    for (int t = threadIdx.x; t <= q; t += 64) rh[t] = a.rhs[c0 + t];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < q; ++j) {
            double* cj = cw[j];
            for (int t = 0; t < j; ++t) {
                const double x0 = cj[t], x1 = cj[t + 1];
                cj[t] = csl[t] * x0 + snl[t] * x1;
                cj[t + 1] = -snl[t] * x0 + csl[t] * x1;
            }
            const double x0 = cj[j], x1 = cj[j + 1];
            double cth = 1.0, sth = 0.0;
            if (x1 != 0.0) {
                const double h = hypot(x0, x1);
                cth = x0 / h;
                sth = x1 / h;
            }
            csl[j] = cth;
            snl[j] = sth;
            cj[j] = cth * x0 + sth * x1;
            cj[j + 1] = 0.0;
            const double g0 = rh[j];
            rh[j + 1] = -sth * g0;
            rh[j] = cth * g0;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < q) {
        double* col = a.R + (long long)(c0 + threadIdx.x) * ldg;
        for (int t = 0; t <= q; ++t) col[c0 + t] = cw[threadIdx.x][t];
        a.cs[c0 + threadIdx.x] = csl[threadIdx.x];
        a.sn[c0 + threadIdx.x] = snl[threadIdx.x];
    }
    for (int t = threadIdx.x; t <= q; t += 64) a.rhs[c0 + t] = rh[t];
    if (threadIdx.x == 0) {
        const double est = fabs(rh[q]);
        const double nu = st->nu_cur;
        st->est = est;
        st->ncols = c0 + q;
        st->kb = kb + 1;
        st->blocks_total += 1;
        st->nu[kb + 1] = nu;
        st->inv_nu[kb + 1] = nu > 0.0 ? 1.0 / nu : 0.0;
        if (!isfinite(est)) {
            st->err = SSTEP_ERR_NONFINITE;
            st->done = 1;
        } else if (est <= st->stop_abs || st->lucky || q < s || kb + 1 == st->m) {
            st->done = 1;
        }
        if (st->done) st->skip_n4b = 1;
    }
}

// Least-squares solution y = R^{-1} rhs (eq. (8)) and assembly coefficients.
// Back substitution over the columns of R, last first.  Thread t owns rows
// t, t + kThreads, ... (ROWS of them) of the right-hand side, kept in
// registers; the column
// of step i is loaded kSolvePf steps ahead, so a step costs one barrier (the
// owner of row i publishes y_i through LDS) instead of two dependent global
// loads.  The barrier orders LDS only: a full __syncthreads() would also wait
// for the columns in flight.  Each row is updated by the same operations in
// the same order as a plain column-oriented back substitution.
constexpr int kSolvePf = 4;  // columns of R in flight
static_assert(8 * kThreads >= kMaxCols, "8 rows per thread must cover kMaxCols");
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
template <int ROWS>
__global__ __launch_bounds__(kThreads) void k_gm_solve(GmArrays a) {
    constexpr int kSolveRows = ROWS;  // rows per thread: ROWS * kThreads >= m * s
    __shared__ double ypub[2];
    GmState* st = a.st;
    if (!st->active) return;
    const int n = st->ncols, s = st->s, ldg = st->ldg;
    const int t = threadIdx.x;
    double b[kSolveRows], yv[kSolveRows];
#pragma unroll
    for (int k = 0; k < kSolveRows; ++k) {
        const int r = t + k * kThreads;
        b[k] = r < n ? a.rhs[r] : 0.0;
        yv[k] = 0.0;
    }
    // column i of R as this thread's rows r <= i (zeros elsewhere); every load
    // is issued (out-of-range ones read R[0]), so the loads in flight can be
    // counted and only the column a step uses is waited for
    auto load_col = [&](int i, double (&dst)[kSolveRows]) {
#pragma unroll
        for (int k = 0; k < kSolveRows; ++k) {
            const int r = t + k * kThreads;
            const bool in = i >= 0 && r <= i;
            const double x = a.R[in ? r + (long long)i * ldg : 0];
            dst[k] = in ? x : 0.0;
        }
    };
    // step i: the owner of row i forms y_i, every row r < i takes its share;
    // then the slot refills with the column kSolvePf steps ahead
    auto step = [&](int i, double (&c)[kSolveRows]) {
        const int ko = i / kThreads;
        if (t == i % kThreads) {
            double bi = 0.0, di = 1.0;
#pragma unroll
            for (int k = 0; k < kSolveRows; ++k)
                if (k == ko) {
                    bi = b[k];
                    di = c[k];
                }
            const double yi = bi / di;
#pragma unroll
            for (int k = 0; k < kSolveRows; ++k)
                if (k == ko) yv[k] = yi;
            ypub[i & 1] = yi;
        }
        lds_barrier();
        const double v = ypub[i & 1];
#pragma unroll
        for (int k = 0; k < kSolveRows; ++k)
            if (t + k * kThreads < i) b[k] -= c[k] * v;
        load_col(i - kSolvePf, c);
    };
    double col[kSolvePf][kSolveRows];
#pragma unroll
    for (int u = 0; u < kSolvePf; ++u) load_col(n - 1 - u, col[u]);
    int i = n - 1;
    for (; i >= kSolvePf - 1; i -= kSolvePf) {  // whole groups of kSolvePf steps
#pragma unroll
        for (int u = 0; u < kSolvePf; ++u) step(i - u, col[u]);
    }
#pragma unroll
    for (int u = 0; u < kSolvePf - 1; ++u)  // the last i + 1 < kSolvePf steps
        if (i - u >= 0) step(i - u, col[u]);
#pragma unroll
    for (int k = 0; k < kSolveRows; ++k) {
        const int r = t + k * kThreads;
        if (r < n) {
            a.y[r] = yv[k];
            a.coefA[r] = yv[k] * ((r % s == 0) ? st->inv_nu[r / s] : 1.0);
        }
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct GmLayout {
    long long N, ld;
    int s, m, K;
    size_t off_basis, off_state, off_G, off_R, off_cs, off_sn, off_rhs, off_y, off_T, off_coefM,
        off_coefA, off_Gout, off_Wf, off_gpart, off_npart, off_rpart, off_scratch, total;
};

static GmLayout gm_layout(const sstep_stencil& A, int s, int m, int precision) {
    GmLayout L{};
    L.N = grid_points(A);
    L.ld = col_stride(L.N);
    L.s = s;
    L.m = m;
    L.K = m * s;
    const size_t esz = precision == SSTEP_MIXED ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const int K = L.K;
    L.off_basis = take((size_t)(K + 1) * L.ld * esz);
    L.off_state = take(sizeof(GmState));
    L.off_G = take(sizeof(double) * (size_t)(K + 1) * K);
    L.off_R = take(sizeof(double) * (size_t)(K + 1) * K);
    L.off_cs = take(sizeof(double) * (K + 1));
    L.off_sn = take(sizeof(double) * (K + 1));
    L.off_rhs = take(sizeof(double) * (K + 1));
    L.off_y = take(sizeof(double) * (K + 1));
    L.off_T = take(sizeof(double) * (size_t)K * (s + 1));
    L.off_coefM = take(sizeof(double) * (size_t)K * s);
    L.off_coefA = take(sizeof(double) * (K + 1));
    L.off_Gout = take(sizeof(double) * (size_t)(K + 1) * (s + 1));
    L.off_Wf = take(sizeof(GramFactor) * (size_t)m);
    size_t gp = gram_partial_doubles(L.N, s + 1, s + 1);
    for (int ncx = s; ncx < K; ncx += s) gp = std::max(gp, gram_partial_doubles(L.N, ncx, s));
    L.off_gpart = take(sizeof(double) * gp);
    L.off_npart = take(sizeof(double) * (size_t)std::max<long long>(update_blocks(L.N), norm_blocks(L.N)));
    const StencilView v = make_view(A);
    L.off_rpart = take(sizeof(double) * (size_t)stencil_blocks(v));
    L.off_scratch = take(sizeof(double) * 64 * 3);
    L.total = off;
    return L;
}

size_t gmres_workspace_bytes(const sstep_stencil& A, int s, int m, int precision) {
    return gm_layout(A, s, m, precision).total;
}

template <typename T>
static void gmres_enqueue_cycle(Ctx& c, const StencilView& v, GmArrays& a, GmState* dst, T* basis,
                                long long N, long long ld, int s, int K, int nb,
                                const sstep_options& opt, const OpParams& P, double* gpart,
                                double* npart, int nnpart, double vb, double* x,
                                const std::function<void()>& residual_and_start);

// A captured restart cycle (opt.graph): graph, executable, the private
// capture stream and the block count it was captured for.
struct CycleGraph {
    bool on = false;
    int nb = -1;
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (g) (void)hipGraphDestroy(g);
        if (cs) (void)hipStreamDestroy(cs);
        exec = nullptr;
        g = nullptr;
        cs = nullptr;
        nb = -1;
    }
    ~CycleGraph() { reset(); }
};

template <typename T>
static int gmres_run(Ctx& c, const sstep_stencil& Ast, const double* f, double* x, int s, int m,
                     double tol, const sstep_options& opt, sstep_info* info, char* ws,
                     const GmLayout& L) {
    const StencilView v = make_view(Ast);
    const long long N = L.N, ld = L.ld;
    const int K = L.K;
    T* basis = reinterpret_cast<T*>(ws + L.off_basis);
    GmArrays a;
    a.st = reinterpret_cast<GmState*>(ws + L.off_state);
    a.G = reinterpret_cast<double*>(ws + L.off_G);
    a.R = reinterpret_cast<double*>(ws + L.off_R);
    a.cs = reinterpret_cast<double*>(ws + L.off_cs);
    a.sn = reinterpret_cast<double*>(ws + L.off_sn);
    a.rhs = reinterpret_cast<double*>(ws + L.off_rhs);
    a.y = reinterpret_cast<double*>(ws + L.off_y);
    a.T = reinterpret_cast<double*>(ws + L.off_T);
    a.coefM = reinterpret_cast<double*>(ws + L.off_coefM);
    a.coefA = reinterpret_cast<double*>(ws + L.off_coefA);
    a.Gout = reinterpret_cast<double*>(ws + L.off_Gout);
    a.Wf = reinterpret_cast<GramFactor*>(ws + L.off_Wf);
    double* gpart = reinterpret_cast<double*>(ws + L.off_gpart);
    double* npart = reinterpret_cast<double*>(ws + L.off_npart);
    double* rpart = reinterpret_cast<double*>(ws + L.off_rpart);
    double* scratch = reinterpret_cast<double*>(ws + L.off_scratch);
    GmState* dst = a.st;

    OpParams P = op_params(Ast, opt.sigma, c.st, scratch);
    if (opt.basis == SSTEP_BASIS_NEWTON) newton_shifts(s, P.cc, P.cd, P.th);
    // host-initialised parameters
    GmState h;
    std::memset(&h, 0, sizeof(h));
    h.s = s;
    h.m = m;
    h.K = K;
    h.ldg = K + 1;
    h.basis = opt.basis;
    h.mixed = (opt.precision == SSTEP_MIXED);
    h.sigma = P.sigma;
    h.cc = P.cc;
    h.cd = P.cd;
    h.tol_rel = tol;
    h.inner_rel = opt.inner_tol > 0.0 ? opt.inner_tol : 1e-5;
    h.rank_tol = 1e-14;
    h.lucky_tol = 1e-14;
    h.done = 1;
    basis_matrix(s, opt.basis, P, h.Bc);
    SSTEP_HIP(hipMemcpyAsync(dst, &h, sizeof(GmState), hipMemcpyHostToDevice, c.st));

    const int max_blocks = opt.max_iters > 0 ? opt.max_iters : 10000;
    const double vb = (double)N * sizeof(T);

    // ||f||
    c.cur_block = -1;
    launch_norm2(c, N, f, npart);
    c.begin(SSTEP_K_SCALAR, 0.0);
    hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(kThreads), 0, c.st, a, npart, norm_blocks(N));
    SSTEP_HIP(hipGetLastError());
    c.end();
    const int nrpart = (int)stencil_blocks(v);
    const int nnpart = (int)update_blocks_t<T, T, T>(N);
    auto residual_and_start = [&]() {
        c.cur_block = -1;
        launch_residual<T>(c, v, f, x, basis, rpart);
        c.begin(SSTEP_K_SCALAR, 0.0);
        hipLaunchKernelGGL(k_gm_cycle_start, dim3(1), dim3(kThreads), 0, c.st, a, rpart, nrpart);
        SSTEP_HIP(hipGetLastError());
        c.end();
    };
    struct Ret {
        int conv, err, blocks_total, cycles, ncols, kb, asm_cols;
        double est, beta, fnorm, tol_abs;
    } ret{};
    auto read_state = [&]() {
        GmState hs;
        SSTEP_HIP(hipMemcpyAsync(&hs, dst, sizeof(GmState), hipMemcpyDeviceToHost, c.st));
        SSTEP_HIP(hipStreamSynchronize(c.st));
        ret.conv = hs.conv;
        ret.err = hs.err;
        ret.blocks_total = hs.blocks_total;
        ret.cycles = hs.cycles;
        ret.ncols = hs.ncols;
        ret.kb = hs.kb;
        ret.asm_cols = hs.asm_cols;
        ret.est = hs.est;
        ret.beta = hs.beta;
        ret.fnorm = hs.fnorm;
        ret.tol_abs = hs.tol_abs;
    };

    residual_and_start();
    read_state();
    c.harvest(0);
    const std::function<void()> ras = residual_and_start;
    auto enqueue_cycle = [&](int nb) {
        gmres_enqueue_cycle<T>(c, v, a, dst, basis, N, ld, s, K, nb, opt, P, gpart, npart, nnpart,
                               vb, x, ras);
    };
    CycleGraph graph;
    graph.on = opt.graph != 0 && !c.profile;
    int matvecs = 1, cycles = 0;
    int status = SSTEP_NOT_CONVERGED;
    double last_est = ret.beta;
    for (;;) {
        if (ret.err) { status = ret.err; break; }
        if (ret.conv) { status = SSTEP_OK; break; }
        const int nb = std::min(m, max_blocks - ret.blocks_total);
        if (nb <= 0) { status = SSTEP_NOT_CONVERGED; break; }
        ++cycles;
        if (graph.on) {
            // the launches of a cycle depend only on nb: capture them once on
            // a private stream (capture needs one), replay every cycle
            if (!graph.exec || graph.nb != nb) {
                graph.reset();
                (void)device_cus();  // device queries happen before the capture
                SSTEP_HIP(hipStreamCreateWithFlags(&graph.cs, hipStreamNonBlocking));
                SSTEP_HIP(hipStreamBeginCapture(graph.cs, hipStreamCaptureModeThreadLocal));
                const hipStream_t user = c.st;
                c.st = graph.cs;
                try {
                    enqueue_cycle(nb);
                } catch (...) {
                    c.st = user;
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(graph.cs, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                c.st = user;
                SSTEP_HIP(hipStreamEndCapture(graph.cs, &graph.g));
                SSTEP_HIP(hipGraphInstantiate(&graph.exec, graph.g, nullptr, nullptr, 0));
                graph.nb = nb;
            }
            SSTEP_HIP(hipGraphLaunch(graph.exec, c.st));
        } else {
            enqueue_cycle(nb);
        }
        const int before = ret.blocks_total;
        read_state();
        const int ran = ret.blocks_total - before;
        matvecs += ran * s + 1;
        c.harvest(ran);
        // the assembly's column count was known only on the device: x (FP64)
        // and asm_cols basis columns read, x written
        c.add_bytes(SSTEP_K_VEC, ((double)ret.asm_cols * sizeof(T) + 16.0) * (double)N);
        last_est = ret.est;
    }
    if (info) {
        info->iters = ret.blocks_total;
        info->cycles = cycles;
        info->matvecs = matvecs;
        info->rel_resid = ret.fnorm > 0 ? ret.beta / ret.fnorm : ret.beta;
        info->rel_resid_est = ret.fnorm > 0 ? last_est / ret.fnorm : last_est;
        info->sigma = P.sigma;
        info->cheb_centre = P.cc;
        info->cheb_half_width = P.cd;
    }
    return status;
}

// The launches of one restart cycle of nb blocks, then the least-squares
// solve, the solution update and the next cycle's true residual.
template <typename T>
static void gmres_enqueue_cycle(Ctx& c, const StencilView& v, GmArrays& a, GmState* dst, T* basis,
                                long long N, long long ld, int s, int K, int nb,
                                const sstep_options& opt, const OpParams& P, double* gpart,
                                double* npart, int nnpart, double vb, double* x,
                                const std::function<void()>& residual_and_start) {
    {
        const int* done = &dst->done;
        for (int kb = 0; kb < nb; ++kb) {
            c.cur_block = kb;
            T* Yk = basis + (long long)kb * s * ld;
            launch_mpk<T>(c, v, Yk, ld, s, opt.basis, P, &dst->inv_nu[kb], done);
            if (kb > 0) {
                const int ncx = kb * s;
                launch_gram<T>(c, basis, ld, ncx, Yk + ld, ld, s, (const T*)nullptr, 0, 0, N, gpart,
                               a.Gout, done);
                c.begin(SSTEP_K_SCALAR, 0.0);
                hipLaunchKernelGGL(k_gm_proj, dim3(kb), dim3(kThreads), 0, c.st, a);
                SSTEP_HIP(hipGetLastError());
                c.end();
                launch_update<T, T, T, T, false>(c, N, Yk + ld, ld, basis, ld, ncx, nullptr,
                                                 a.coefM, Yk + ld, ld, s, nullptr, done,
                                                 vb * (ncx + 2 * s));
            }
            launch_gram<T>(c, Yk, ld, s + 1, Yk, ld, s + 1, (const T*)nullptr, 0, 0, N, gpart,
                           a.Gout, done, SSTEP_K_VEC);
            c.begin(SSTEP_K_SCALAR, 0.0);
            hipLaunchKernelGGL(k_gm_block, dim3(1), dim3(64), 0, c.st, a);
            SSTEP_HIP(hipGetLastError());
            c.end();
            launch_update<T, T, T, T, true>(c, N, Yk + (long long)s * ld, ld, Yk, ld, s, nullptr,
                                            dst->coefN4b, Yk + (long long)s * ld, ld, 1, npart,
                                            &dst->skip_n4b, vb * (s + 2), SSTEP_K_VEC);
            c.begin(SSTEP_K_SCALAR, 0.0);
            hipLaunchKernelGGL(k_gm_nu, dim3(1), dim3(kThreads), 0, c.st, a, npart, nnpart);
            hipLaunchKernelGGL(k_gm_hess_cols, dim3(kb + 1), dim3(kThreads), 0, c.st, a);
            hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(64), 0, c.st, a);
            SSTEP_HIP(hipGetLastError());
            c.end();
        }
        c.cur_block = -1;
        c.begin(SSTEP_K_SCALAR, 0.0);
        // rows per thread of the back substitution: enough for the m * s columns
        if (K <= kThreads)
            hipLaunchKernelGGL(k_gm_solve<1>, dim3(1), dim3(kThreads), 0, c.st, a);
        else if (K <= 2 * kThreads)
            hipLaunchKernelGGL(k_gm_solve<2>, dim3(1), dim3(kThreads), 0, c.st, a);
        else if (K <= 4 * kThreads)
            hipLaunchKernelGGL(k_gm_solve<4>, dim3(1), dim3(kThreads), 0, c.st, a);
        else
            hipLaunchKernelGGL(k_gm_solve<8>, dim3(1), dim3(kThreads), 0, c.st, a);
        SSTEP_HIP(hipGetLastError());
        c.end();
        // x = x0 + V y (eq. (8)); column count read on the device
        launch_update<T, double, double, double, false>(c, N, x, 0, basis, ld, K, &dst->ncols,
                                                        a.coefA, x, 0, 1, nullptr, &dst->skip_asm,
                                                        0.0, SSTEP_K_VEC);
        residual_and_start();
    }
}

int gmres_solve_impl(Ctx& c, const sstep_stencil& A, const double* f, double* x, int s, int m,
                     double tol, const sstep_options& opt, sstep_info* info, void* ws,
                     size_t ws_bytes) {
    const GmLayout L = gm_layout(A, s, m, opt.precision);
    if (ws_bytes < L.total) return SSTEP_ERR_NOMEM;
    if (opt.precision == SSTEP_MIXED)
        return gmres_run<float>(c, A, f, x, s, m, tol, opt, info, (char*)ws, L);
    return gmres_run<double>(c, A, f, x, s, m, tol, opt, info, (char*)ws, L);
}

}  // namespace sstep
