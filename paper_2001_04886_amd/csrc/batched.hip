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
    double coefM[512 * 16];
    double coefA[513];
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
struct PhaseClock {
    long long t0 = 0;
    long long acc[SSTEP_K_NCLASS] = {0, 0, 0, 0, 0, 0};
    __device__ void start() {
        if (threadIdx.x == 0) t0 = wall_clock64();
    }
    __device__ void lap(int cls) {
        if (threadIdx.x == 0) {
            const long long t = wall_clock64();
            acc[cls] += t - t0;
            t0 = t;
        }
    }
};

// one stencil level over all points of a system: out = a*(A y) with y = in*sc
__device__ __forceinline__ double stencil_at(const StencilView& A, const double* in, long long p,
                                             int i, int j, int l) {
    const long long sy = A.nx, sz = (long long)A.nx * A.ny;
    double acc = 0.0;
    if (i > 0) acc += A.c[1] * in[p - 1];
    if (i < A.nx - 1) acc += A.c[2] * in[p + 1];
    if (j > 0) acc += A.c[3] * in[p - sy];
    if (j < A.ny - 1) acc += A.c[4] * in[p + sy];
    if (A.ndim == 3) {
        if (l > 0) acc += A.c[5] * in[p - sz];
        if (l < A.nz - 1) acc += A.c[6] * in[p + sz];
    }
    return acc + A.c[0] * in[p];
}

template <int NT, int CA, int KZ>
__device__ void wg_gram(const double* X, long long ldx, int ncx, const double* Z, long long ldz,
                        int nz, long long N, double* out /* [ncx][nz] */, double* red) {
    // tiles of CA columns of X against nz <= KZ columns of Z, reduced per tile
    for (int c0 = 0; c0 < ncx; c0 += CA) {
        double acc[CA][KZ];
#pragma unroll
        for (int a = 0; a < CA; ++a)
#pragma unroll
            for (int j = 0; j < KZ; ++j) acc[a][j] = 0.0;
        for (long long p = threadIdx.x; p < N; p += NT) {
            double z[KZ];
#pragma unroll
            for (int j = 0; j < KZ; ++j) z[j] = j < nz ? Z[j * ldz + p] : 0.0;
#pragma unroll
            for (int a = 0; a < CA; ++a) {
                if (c0 + a < ncx) {
                    const double xv = X[(long long)(c0 + a) * ldx + p];
#pragma unroll
                    for (int j = 0; j < KZ; ++j) acc[a][j] = fma(xv, z[j], acc[a][j]);
                }
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

template <int NT, int CA, int KZ>
__device__ void solve_one(const BatchArgs& args, BatchSys& S, BatchSlot& W, double* red,
                          double* sh, double* lw, GramFactor* lf) {
    const int s = args.s, m = args.m, K = m * s, ldg = K + 1, s1 = s + 1;
    const StencilView A = S.A;
    const long long N = A.N, ld = S.ld;
    double* V = S.ws;
    const int tid = threadIdx.x;
    const int nx = A.nx, ny = A.ny;
    // Basis change B (monomial): A Y[:,0:s] = Y B with B[j+1][j] = sigma
    const double sigma = S.sigma;

    PhaseClock pc;
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
        for (long long p = tid; p < N; p += NT) {
            const int pi = (int)p, i = pi % nx, rest = pi / nx, j = rest % ny, l = rest / ny;
            const double r = S.f[p] - stencil_at(A, S.x, p, i, j, l);
            V[p] = r;
            acc += r * r;
        }
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
                for (long long p = tid; p < N; p += NT) {
                    const int pi = (int)p, i = pi % nx, rest = pi / nx, j = rest % ny, l = rest / ny;
                    out[p] = sc * stencil_at(A, in, p, i, j, l);
                }
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
                        W.coefM[(i * s + q) * s + (l - 1)] = -c[q] * (q == 0 ? W.inv_nu[i] : 1.0);
                        if (l == 1) W.T[(i * s + q) * s1] = 0.0;
                    }
                }
                __syncthreads();
                pc.lap(SSTEP_K_SCALAR);
                // y_j -= sum_c V_c coefM[c][j]
                for (long long p = tid; p < N; p += NT) {
                    double a[KZ];
#pragma unroll
                    for (int l = 0; l < KZ; ++l) a[l] = l < s ? Yk[(long long)(l + 1) * ld + p] : 0.0;
                    for (int cc = 0; cc < c0; ++cc) {
                        const double v = V[(long long)cc * ld + p];
#pragma unroll
                        for (int l = 0; l < KZ; ++l)
                            if (l < s) a[l] = fma(v, W.coefM[cc * s + l], a[l]);
                    }
#pragma unroll
                    for (int l = 0; l < KZ; ++l)
                        if (l < s) Yk[(long long)(l + 1) * ld + p] = a[l];
                }
                __syncthreads();
                pc.lap(SSTEP_K_UPDATE);
            }
            // block Gram of [w_k, y_1..y_s]
            wg_gram<NT, CA, KZ + 1>(Yk, ld, s1, Yk, ld, s1, N, W.C, red);
            pc.lap(SSTEP_K_GRAM);
            // Scalar1: factor W_k in LDS (one thread), copy the factor out
            if (tid == 0) {
                const double d0 = W.inv_nu[kb];
                double* Wk = lw;
                for (int q = 0; q < s; ++q)
                    for (int pp = 0; pp < s; ++pp)
                        Wk[pp + q * kMaxS] =
                            W.C[pp * s1 + q] * (pp == 0 ? d0 : 1.0) * (q == 0 ? d0 : 1.0);
                gram_factor(Wk, kMaxS, s, args.rank_tol, lf);
                const int q = lf->rank;
                double* g = sh;  // g[0..s), coefN4b[s..2s), scalars at sh[2 kMaxS ..]
                double* h = sh + 2 * kMaxS + 4;
                if (q == s) {
                    for (int pp = 0; pp < s; ++pp) h[pp] = W.C[pp * s1 + s] * (pp == 0 ? d0 : 1.0);
                    gram_solve(*lf, h, g);
                    for (int pp = 0; pp < s; ++pp) sh[s + pp] = -g[pp] * (pp == 0 ? d0 : 1.0);
                } else if (q > 0) {
                    for (int pp = 0; pp < q; ++pp) h[pp] = Wk[pp + q * kMaxS];
                    gram_solve_leading(*lf, q, h, g);
                }
                sh[2 * kMaxS] = W.C[s * s1 + s];  // ||Yhat_s||^2
            }
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
                acc = 0.0;
                for (long long p = tid; p < N; p += NT) {
                    double v = ys[p];
#pragma unroll
                    for (int l = 0; l < KZ; ++l)
                        if (l < s) v = fma(Yk[(long long)l * ld + p], sh[s + l], v);
                    ys[p] = v;
                    acc += v * v;
                }
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
            if (tid == 0) {
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
        if (tid == 0) {
            for (int i = ncols - 1; i >= 0; --i) {
                double v = W.rhs[i];
                for (int l = i + 1; l < ncols; ++l) v -= W.R[i + l * ldg] * W.y[l];
                W.y[i] = v / W.R[i + i * ldg];
            }
            for (int c = 0; c < ncols; ++c) W.coefA[c] = W.y[c] * ((c % s == 0) ? W.inv_nu[c / s] : 1.0);
        }
        __syncthreads();
        for (long long p = tid; p < N; p += NT) {
            double v = S.x[p];
            for (int c = 0; c < ncols; ++c) v = fma(V[(long long)c * ld + p], W.coefA[c], v);
            S.x[p] = v;
        }
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
    __shared__ int next;
    BatchSlot& W = args.slots[blockIdx.x];
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(args.queue, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();
        if (k >= args.nsys) break;
        solve_one<NT, CA, KZ>(args, args.sys[args.order[k]], W, red, sh, lw, &lf);
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
            double g = 0.0;
            for (int q = 0; q < 2 * A[i].ndim + 1; ++q) g += std::fabs(A[i].c[q]);
            b.sigma = opt.sigma > 0 ? opt.sigma : pow2_ceil(g);
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
