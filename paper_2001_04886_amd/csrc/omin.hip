// omin.hip -- s-step Orthomin(k) (Sec. 3, Alg. 3.1) on one GPU.
//
// Storage (all FP64, column stride ld):
//   buffer A = [Y (s+1 columns) | AP ring (k*s columns)]
//   buffer B = P ring (k*s columns)
// Y column 0 is the residual r itself; the matrix-powers kernel writes
// y_1..y_s after it, so R = Y[:, 0:s] and AR = Y Bbasis (monomial:
// sigma * Y[:, 1:s+1]).  Direction block j lives in ring slot j mod k; the
// new block overwrites the oldest one in place (each thread reads all inputs
// of its points before writing).  With Y adjacent to the AP ring, the
// update AP_{i+1} = AR + sum_j AP_j B_j is a single linear combination of
// contiguous columns.
//
// Per iteration i (device only; the host enqueues batches):
//   Gram     W_i = AP_i^T AP_i, m_i = AP_i^T r               (step 1)
//   scalar   a_i = W_i^{-1} m_i                              (Scalar1)
//   update   x += P_i a_i;  r -= AP_i a_i, ||r||^2           (steps 3-4)
//   MPK      y_j = A y_{j-1} / sigma                         (step 5)
//   Gram     AP_j^T Y for the window                         (step 6)
//   scalar   B_j = -W_j^{-1} (AP_j^T AR)                     (Scalar2)
//   update   P_{i+1} = R + sum P_j B_j;  AP_{i+1} = AR + sum AP_j B_j (8-9)
// With orth = SSTEP_ORTH_MGS every new block (P, AP) is then made
// A^T A-orthogonal by modified Gram-Schmidt on the device (the larger-s
// variant of Sec. 3): for q = 0..s-1 the first stage of a Gram of AP_q
// against AP_q..AP_{s-1}, one scalar kernel that sums its partials and forms
// the coefficients and the dependence test, and one pass over P_q..P_{s-1}
// and AP_q..AP_{s-1}.  W of the block is then
// diagonal, and the Cholesky of Scalar1 / Scalar2 reduces to it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.hpp"
#include "launch.hpp"
#include "solvers.hpp"

namespace sstep {


struct OmState {
    int s, k, basis, max_iters;
    double sigma, cc, cd, tol_rel, fnorm, tol_abs, rank_tol;
    double Bc[(kMaxS + 1) * kMaxS];
    int it, done, conv, err;
    double rnorm, est;
    double coef_x[kMaxS], coef_r[kMaxS];
    // modified Gram-Schmidt: coefficient row of the current step, and per
    // column the squared length removed by the steps so far
    double mgs_row[kMaxS], mgs_removed[kMaxS];
};

struct OmArrays {
    OmState* st;
    double* Gout;
    double* coefP;   // [k*s][s]
    double* coefAP;  // [(s+1) + k*s][s]
    GramFactor* Wf;  // per ring slot
};

__global__ __launch_bounds__(kThreads) void k_om_init(OmArrays a, const double* __restrict__ part,
                                                      int npart) {
    __shared__ double lds[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < npart; i += kThreads) acc += part[i];
    double v[1] = {acc}, o[1];
    block_sum<1>(v, lds, o);
    if (threadIdx.x == 0) {
        OmState* st = a.st;
        st->fnorm = sqrt(o[0]);
        st->tol_abs = st->tol_rel * st->fnorm;
        st->it = 0;
        st->conv = 0;
        st->err = 0;
        st->done = 1;
    }
}

// True residual check / (re)start of the recurrence: r = f - A x is in Y[:,0].
__global__ __launch_bounds__(kThreads) void k_om_start(OmArrays a, const double* __restrict__ part,
                                                       int npart) {
    __shared__ double lds[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < npart; i += kThreads) acc += part[i];
    double v[1] = {acc}, o[1];
    block_sum<1>(v, lds, o);
    if (threadIdx.x == 0) {
        OmState* st = a.st;
        const double rn = sqrt(o[0]);
        st->rnorm = rn;
        if (!isfinite(rn)) {
            st->err = SSTEP_ERR_NONFINITE;
            st->done = 1;
        } else if (rn <= st->tol_abs) {
            st->conv = 1;
            st->done = 1;
        } else {
            st->done = (st->it >= st->max_iters) ? 1 : 0;
        }
    }
}

// Scalar1: factor W_i (into ring slot), a_i = W_i^{-1} m_i.
// Gout: s x (s+1) = AP_i^T [AP_i | r].
__global__ __launch_bounds__(64) void k_om_step1(OmArrays a, int slot) {
    // the factorisation works on LDS copies (read-after-write chains through
    // global memory would wait a memory round trip per step); the factor is
    // copied out at the end
    __shared__ double W[kMaxS * kMaxS];
    __shared__ GramFactor F;
    OmState* st = a.st;
    if (st->done) return;
    const int s = st->s;
    for (int idx = threadIdx.x; idx < s * s; idx += blockDim.x) {
        const int p = idx % s, q = idx / s;
        W[p + q * kMaxS] = a.Gout[p * (s + 1) + q];
    }
    __syncthreads();
    gram_factor_wave(W, s, st->rank_tol, &F);  // the wave factors; W is overwritten
    __syncthreads();
    if (threadIdx.x == 0) {
        double m[kMaxS];
        for (int q = 0; q < s; ++q) m[q] = a.Gout[q * (s + 1) + s];
        if (F.rank == 0) {
            st->err = SSTEP_ERR_BREAKDOWN;
            st->done = 1;
        } else {
            double al[kMaxS];
            gram_solve(F, m, al);
            for (int q = 0; q < s; ++q) {
                st->coef_x[q] = al[q];
                st->coef_r[q] = -al[q];
            }
        }
    }
    __syncthreads();
    const double* src = reinterpret_cast<const double*>(&F);
    double* dst = reinterpret_cast<double*>(&a.Wf[slot]);
    for (int i = threadIdx.x; i < (int)(sizeof(GramFactor) / sizeof(double)); i += blockDim.x)
        dst[i] = src[i];
}

// After x, r updates: recurrence residual norm, iteration count, stop test.
__global__ __launch_bounds__(kThreads) void k_om_check(OmArrays a, const double* __restrict__ part,
                                                       int npart) {
    __shared__ double lds[4];
    OmState* st = a.st;
    if (st->done) return;
    double v[1] = {strided_partial_sum(part, npart)}, o[1];
    block_sum<1>(v, lds, o);
    if (threadIdx.x == 0) {
        const double rn = sqrt(o[0]);
        st->est = rn;
        st->it += 1;
        if (!isfinite(rn)) {
            st->err = SSTEP_ERR_NONFINITE;
            st->done = 1;
        } else if (rn <= st->tol_abs || st->it >= st->max_iters) {
            st->done = 1;  // host checks the true residual
        }
    }
}

// Scalar2: B_j = -W_j^{-1} C_j, C_j = (AP_j^T Y) Bbasis, for the nfill window
// blocks held in ring slots 0..nfill-1; coefficient rows for the P and AP
// updates.  Gout: (nfill*s) x (s+1) = AP_ring^T Y.
__global__ __launch_bounds__(kThreads) void k_om_step2(OmArrays a, int nfill) {
    // workgroup j: the s columns of B_j from the factor of W_j staged in LDS
    __shared__ GramFactor F;
    OmState* st = a.st;
    if (st->done) return;
    const int s = st->s, s1 = s + 1, j = blockIdx.x;
    const double* Bc = st->Bc;
    if (j == 0) {
        // rows for Y in the AP update: AR = Y Bbasis
        for (int idx = threadIdx.x; idx < s1 * s; idx += kThreads) {
            const int t = idx / s, l = idx % s;
            a.coefAP[t * s + l] = Bc[t + l * s1];
        }
    }
    if (j >= nfill) return;
    {
        const double* src = reinterpret_cast<const double*>(&a.Wf[j]);
        double* dst = reinterpret_cast<double*>(&F);
        for (int i = threadIdx.x; i < (int)(sizeof(GramFactor) / sizeof(double)); i += kThreads)
            dst[i] = src[i];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < s; l += kThreads) {  // column l of B_j
        double c[kMaxS];
        for (int q = 0; q < s; ++q) {
            double v = 0.0;
            for (int t = 0; t <= s; ++t) v += a.Gout[(j * s + q) * s1 + t] * Bc[t + l * s1];
            c[q] = v;
        }
        gram_solve(F, c, c);
        for (int q = 0; q < s; ++q) {
            a.coefP[(j * s + q) * s + l] = -c[q];
            a.coefAP[(s1 + j * s + q) * s + l] = -c[q];
        }
    }
}

// MGS step q.  The Gram row G = AP_q^T [AP_q .. AP_{s-1}] is summed here from
// the partials of the Gram's first stage (fixed order: lane-strided chunks,
// then a wave sum).  w = G[0] is the squared length of AP_q after its
// components along AP_0..AP_{q-1} were removed, n0 = w + (removed) its length
// before.  Column q is kept if w > rank_tol * n0 (else it is numerically
// dependent and set to zero); the coefficient row for columns q..s-1 is
// [keep - 1, -G[l]/w ...].
__global__ __launch_bounds__(64) void k_om_mgs(OmArrays a, int q, const double* __restrict__ part,
                                               int nchunk, int KZ) {
    __shared__ double G[kMaxS];
    OmState* st = a.st;
    if (st->done) return;
    const int s = st->s;
    for (int j = 0; j < s - q; ++j) {
        double v = 0.0;
        for (int ch = threadIdx.x; ch < nchunk; ch += 64) v += part[(long long)ch * KZ + j];
        v = wave_sum(v);
        if (threadIdx.x == 0) G[j] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (q == 0)
        for (int l = 0; l < s; ++l) st->mgs_removed[l] = 0.0;
    const double w = G[0];
    const double n0 = w + st->mgs_removed[q];
    const bool keep = std::isfinite(w) && w > st->rank_tol * n0;
    st->mgs_row[0] = keep ? 0.0 : -1.0;
    for (int l = q + 1; l < s; ++l) {
        const double g = G[l - q];
        const double c = keep ? g / w : 0.0;
        st->mgs_row[l - q] = -c;
        st->mgs_removed[l] += c * g;
    }
}

// MGS step q applied to both blocks: column q kept or zeroed, columns q+1..
// minus their coefficient times column q, for P and AP in one pass.
__global__ __launch_bounds__(kThreads) void k_om_mgs_apply(OmArrays a, long long N, double* P,
                                                           double* AP, long long ld, int ncol) {
    const OmState* st = a.st;
    if (st->done) return;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    const double* row = st->mgs_row;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        double* X = blk ? AP : P;
        const double xq = X[p];
        X[p] = fma(row[0], xq, xq);
        for (int l = 1; l < ncol; ++l) X[l * ld + p] = fma(row[l], xq, X[l * ld + p]);
    }
}

struct OmLayout {
    long long N, ld;
    int s, k;
    size_t off_bufA, off_bufB, off_state, off_Gout, off_coefP, off_coefAP, off_Wf, off_gpart,
        off_npart, off_rpart, off_scratch, total;
};

static OmLayout om_layout(const sstep_stencil& A, int s, int k) {
    OmLayout L{};
    L.N = grid_points(A);
    L.ld = col_stride(L.N);
    L.s = s;
    L.k = k;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L.off_bufA = take(sizeof(double) * (size_t)(s + 1 + k * s) * L.ld);
    L.off_bufB = take(sizeof(double) * (size_t)(k * s) * L.ld);
    L.off_state = take(sizeof(OmState));
    L.off_Gout = take(sizeof(double) * (size_t)(k * s) * (s + 1));
    L.off_coefP = take(sizeof(double) * (size_t)(k * s) * s);
    L.off_coefAP = take(sizeof(double) * (size_t)(s + 1 + k * s) * s);
    L.off_Wf = take(sizeof(GramFactor) * k);
    size_t gp = std::max(gram_partial_doubles(L.N, s, s + 1), gram_partial_doubles(L.N, 1, s));
    for (int nf = 1; nf <= k; ++nf) gp = std::max(gp, gram_partial_doubles(L.N, nf * s, s + 1));
    L.off_gpart = take(sizeof(double) * gp);
    L.off_npart = take(sizeof(double) * (size_t)std::max<long long>(update_blocks(L.N), norm_blocks(L.N)));
    L.off_rpart = take(sizeof(double) * (size_t)stencil_blocks(make_view(A)));
    L.off_scratch = take(sizeof(double) * 64 * 3);
    L.total = off;
    return L;
}

size_t omin_workspace_bytes(const sstep_stencil& A, int s, int k) {
    return om_layout(A, s, k).total;
}

int omin_solve_impl(Ctx& c, const sstep_stencil& Ast, const double* f, double* x, int s, int k,
                    double tol, const sstep_options& opt, sstep_info* info, void* wsv,
                    size_t ws_bytes) {
    const OmLayout L = om_layout(Ast, s, k);
    if (ws_bytes < L.total) return SSTEP_ERR_NOMEM;
    char* ws = (char*)wsv;
    const StencilView v = make_view(Ast);
    const long long N = L.N, ld = L.ld;
    double* Y = reinterpret_cast<double*>(ws + L.off_bufA);
    double* APr = Y + (long long)(s + 1) * ld;
    double* Pr = reinterpret_cast<double*>(ws + L.off_bufB);
    OmArrays a;
    a.st = reinterpret_cast<OmState*>(ws + L.off_state);
    a.Gout = reinterpret_cast<double*>(ws + L.off_Gout);
    a.coefP = reinterpret_cast<double*>(ws + L.off_coefP);
    a.coefAP = reinterpret_cast<double*>(ws + L.off_coefAP);
    a.Wf = reinterpret_cast<GramFactor*>(ws + L.off_Wf);
    double* gpart = reinterpret_cast<double*>(ws + L.off_gpart);
    double* npart = reinterpret_cast<double*>(ws + L.off_npart);
    double* rpart = reinterpret_cast<double*>(ws + L.off_rpart);
    double* scratch = reinterpret_cast<double*>(ws + L.off_scratch);
    OmState* dst = a.st;
    const int* done = &dst->done;

    OpParams P = op_params(Ast, opt.sigma, c.st, scratch);
    if (opt.basis == SSTEP_BASIS_NEWTON) newton_shifts(s, P.cc, P.cd, P.th);
    const int max_iters = opt.max_iters > 0 ? opt.max_iters : 10000;
    OmState h;
    std::memset(&h, 0, sizeof(h));
    h.s = s;
    h.k = k;
    h.basis = opt.basis;
    h.max_iters = max_iters;
    h.sigma = P.sigma;
    h.cc = P.cc;
    h.cd = P.cd;
    h.tol_rel = tol;
    h.rank_tol = 1e-14;
    h.done = 1;
    basis_matrix(s, opt.basis, P, h.Bc);
    SSTEP_HIP(hipMemcpyAsync(dst, &h, sizeof(OmState), hipMemcpyHostToDevice, c.st));

    const double vb = 8.0 * N;
    const int nrpart = (int)stencil_blocks(v), nnpart = (int)update_blocks_t<double, double, double>(N);
    auto scalar = [&](auto kern, int threads, auto... args) {
        c.begin(SSTEP_K_SCALAR, 0.0);
        hipLaunchKernelGGL(kern, dim3(1), dim3(threads), 0, c.st, a, args...);
        SSTEP_HIP(hipGetLastError());
        c.end();
    };
    // one workgroup per window slot (at least one)
    auto scalar_slots = [&](auto kern, int nslots, auto... args) {
        c.begin(SSTEP_K_SCALAR, 0.0);
        hipLaunchKernelGGL(kern, dim3(nslots > 0 ? nslots : 1), dim3(kThreads), 0, c.st, a, args...);
        SSTEP_HIP(hipGetLastError());
        c.end();
    };
    c.cur_block = -1;
    // ||f||
    launch_norm2(c, N, f, npart);
    scalar(k_om_init, kThreads, (const double*)npart, norm_blocks(N));
    auto true_residual = [&]() {
        c.cur_block = -1;
        launch_residual<double>(c, v, f, x, Y, rpart);
        scalar(k_om_start, kThreads, (const double*)rpart, nrpart);
    };
    OmState hs;
    auto read_state = [&]() {
        SSTEP_HIP(hipMemcpyAsync(&hs, dst, sizeof(OmState), hipMemcpyDeviceToHost, c.st));
        SSTEP_HIP(hipStreamSynchronize(c.st));
    };
    // A^T A-orthogonalise direction block `slot` in place (SSTEP_ORTH_MGS)
    const bool mgs = opt.orth == SSTEP_ORTH_MGS;
    auto orthogonalise = [&](int slot) {
        double* Pb = Pr + (long long)slot * s * ld;
        double* APb = APr + (long long)slot * s * ld;
        for (int q = 0; q < s; ++q) {
            double* Pq = Pb + (long long)q * ld;
            double* APq = APb + (long long)q * ld;
            // first stage of the Gram only: k_om_mgs sums the partials itself
            launch_gram<double>(c, APq, ld, 1, APq, ld, s - q, (const double*)nullptr, 0, 0, N,
                                gpart, a.Gout, done, SSTEP_K_VEC, /*reduce=*/false);
            int KZ, CA, nct, nchunk;
            long long chunk;
            gram_geometry(N, 1, s - q, &KZ, &CA, &nct, &nchunk, &chunk);
            scalar(k_om_mgs, 64, q, (const double*)gpart, nchunk, KZ);
            // columns q..s-1 of P and AP += column q x row (column q: kept or zeroed)
            c.begin(SSTEP_K_VEC, 2.0 * (2.0 * (s - q)) * vb);
            hipLaunchKernelGGL(k_om_mgs_apply, dim3((unsigned)((N + kThreads - 1) / kThreads)),
                               dim3(kThreads), 0, c.st, a, N, Pq, APq, ld, s - q);
            SSTEP_HIP(hipGetLastError());
            c.end();
        }
    };
    // R_0, AR_0 from the current r (Y[:,0]) into slot 0
    auto start_recurrence = [&]() {
        launch_mpk<double>(c, v, Y, ld, s, opt.basis, P, nullptr, done);
        scalar_slots(k_om_step2, 0, 0);  // coefficient rows of AR
        launch_update<double, double, double, double, false>(c, N, Y, ld, Pr, ld, 0, nullptr,
                                                             a.coefP, Pr, ld, s, nullptr, done,
                                                             2 * s * vb);
        launch_update<double, double, double, double, false>(
            c, N, (const double*)nullptr, 0, Y, ld, s + 1, nullptr, a.coefAP, APr, ld, s, nullptr,
            done, (2 * s + 1) * vb);
        if (mgs) orthogonalise(0);
    };

    true_residual();
    read_state();
    c.harvest(0);
    int status = SSTEP_NOT_CONVERGED, cycles = 0, matvecs = 1;
    const int batch = 8;
    while (true) {
        if (hs.err) { status = hs.err; break; }
        if (hs.conv) { status = SSTEP_OK; break; }
        if (hs.it >= max_iters) { status = SSTEP_NOT_CONVERGED; break; }
        // (re)start the recurrence from r = Y[:,0]
        ++cycles;
        start_recurrence();
        matvecs += s;
        int i = 0;
        bool stop = false;
        while (!stop) {
            const int it0 = hs.it;
            const int nb = std::min(batch, max_iters - it0);
            for (int b = 0; b < nb; ++b, ++i) {
                c.cur_block = b;
                const int slot = i % k, nslot = (i + 1) % k;
                const int nfill = std::min(i + 1, k);
                double* APi = APr + (long long)slot * s * ld;
                double* Pi = Pr + (long long)slot * s * ld;
                launch_gram<double>(c, APi, ld, s, APi, ld, s, Y, ld, 1, N, gpart, a.Gout, done,
                                    SSTEP_K_VEC);
                scalar(k_om_step1, 64, slot);
                launch_update<double, double, double, double, false>(
                    c, N, x, 0, Pi, ld, s, nullptr, dst->coef_x, x, 0, 1, nullptr, done,
                    (s + 2) * vb, SSTEP_K_VEC);
                launch_update<double, double, double, double, true>(
                    c, N, Y, 0, APi, ld, s, nullptr, dst->coef_r, Y, 0, 1, npart, done,
                    (s + 2) * vb, SSTEP_K_VEC);
                scalar(k_om_check, kThreads, (const double*)npart, nnpart);
                launch_mpk<double>(c, v, Y, ld, s, opt.basis, P, nullptr, done);
                launch_gram<double>(c, APr, ld, nfill * s, Y, ld, s + 1, (const double*)nullptr, 0,
                                    0, N, gpart, a.Gout, done);
                scalar_slots(k_om_step2, nfill, nfill);
                launch_update<double, double, double, double, false>(
                    c, N, Y, ld, Pr, ld, nfill * s, nullptr, a.coefP, Pr + (long long)nslot * s * ld,
                    ld, s, nullptr, done, (2 * s + nfill * s) * vb);
                launch_update<double, double, double, double, false>(
                    c, N, (const double*)nullptr, 0, Y, ld, s + 1 + nfill * s, nullptr, a.coefAP,
                    APr + (long long)nslot * s * ld, ld, s, nullptr, done,
                    (2 * s + 1 + nfill * s) * vb);
                if (mgs) orthogonalise(nslot);
            }
            read_state();
            const int ran = hs.it - it0;
            matvecs += ran * s;
            c.harvest(ran);
            if (hs.err) { stop = true; break; }
            if (hs.done) {
                // recurrence residual passed (or cap): confirm with the true residual
                true_residual();
                read_state();
                c.harvest(0);
                ++matvecs;
                stop = true;  // outer loop: converged, capped, or residual replacement
            }
        }
    }
    if (info) {
        info->iters = hs.it;
        info->cycles = cycles;
        info->matvecs = matvecs;
        info->rel_resid = hs.fnorm > 0 ? hs.rnorm / hs.fnorm : hs.rnorm;
        info->rel_resid_est = hs.fnorm > 0 ? hs.est / hs.fnorm : hs.est;
        info->sigma = P.sigma;
        info->cheb_centre = P.cc;
        info->cheb_half_width = P.cd;
    }
    return status;
}

}  // namespace sstep
