// capi.hip -- extern "C" entry points of libsstep.so: argument validation,
// workspace handling, timing, and the primitive kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/sstep.h"
#include "dense.hpp"
#include "launch.hpp"
#include "solvers.hpp"

using namespace sstep;

namespace {

bool stencil_ok(const sstep_stencil* A) {
    if (!A) return false;
    if (A->ndim != 2 && A->ndim != 3) return false;
    if (A->nx < 1 || A->ny < 1 || (A->ndim == 3 && A->nz < 1)) return false;
    const long long N = grid_points(*A);
    if (N > (1LL << 31) - 1) return false;
    if (!A->coef)
        for (int q = 0; q < 2 * A->ndim + 1; ++q)
            if (!std::isfinite(A->c[q])) return false;
    // rows of the grid are addressed by blockIdx (one workgroup per row segment)
    const long long rows = (long long)A->ny * (A->ndim == 3 ? A->nz : 1) * ((A->nx + 255) / 256);
    if (rows > 0x7fffffffLL) return false;
    return true;
}

int set_status(sstep_info* info, int st) {
    if (info) info->status = st;
    return st;
}

template <typename F>
int guarded(sstep_info* info, F&& fn) {
    try {
        return set_status(info, fn());
    } catch (const HipFailure&) {
        (void)hipGetLastError();
        return set_status(info, SSTEP_ERR_HIP);
    }
}

// Run a solver with workspace handling and total timing.
template <typename Solve>
int run_solver(const sstep_options* opt_in, size_t need, sstep_info* info, Solve&& solve) {
    sstep_options opt;
    if (opt_in) opt = *opt_in;
    else sstep_default_options(&opt);
    if (info) std::memset(info, 0, sizeof(*info));
    return guarded(info, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)opt.stream;
        c.profile = opt.profile != 0;
        void* ws = opt.workspace;
        size_t wsb = opt.workspace_bytes;
        bool owned = false;
        if (!ws) {
            if (hipMalloc(&ws, need) != hipSuccess) {
                (void)hipGetLastError();
                return SSTEP_ERR_NOMEM;
            }
            wsb = need;
            owned = true;
        } else if (wsb < need || ((uintptr_t)ws & 255u)) {
            return SSTEP_ERR_NOMEM;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int st = SSTEP_ERR_HIP;
        try {
            SSTEP_HIP(hipEventCreate(&e0));
            SSTEP_HIP(hipEventCreate(&e1));
            SSTEP_HIP(hipEventRecord(e0, c.st));
            st = solve(c, opt, ws, wsb);
            SSTEP_HIP(hipEventRecord(e1, c.st));
            SSTEP_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            SSTEP_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (info) {
                info->ms_total = ms;
                for (int k = 0; k < SSTEP_K_NCLASS; ++k) {
                    info->launches[k] = c.launches[k];
                    info->ms[k] = c.ms[k];
                    info->bytes[k] = c.bytes[k];
                }
            }
        } catch (...) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (owned) (void)hipFree(ws);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (owned) SSTEP_HIP(hipFree(ws));
        return st;
    });
}

bool precond_ok(const sstep_stencil* A, const sstep_options* opt, int prec, int basis) {
    if (!opt || opt->precond == SSTEP_PRECOND_NONE) return true;
    return opt->precond == SSTEP_PRECOND_ILU0 && ilu0_supported(*A) && prec == SSTEP_FP64 &&
           basis == SSTEP_BASIS_MONOMIAL;
}
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
size_t ilu0_sweep_bytes(const sstep_stencil& A) {
    // intermediate, right-hand side, 1/d and (per-point coefficients) four
    // neighbour coefficient planes
    return align256((size_t)ilu0_sweep_points(make_view(A)) * 8) * (A.coef ? 7 : 3);
}
size_t ilu0_workspace(const sstep_stencil& A) {
    return 4 * align256((size_t)grid_points(A) * 8) + ilu0_sweep_bytes(A) + 256;
}
// Right-preconditioned solve (Sec. 5): factor, u = M x, run the method on
// A M^{-1} u = f with the preconditioner attached to the context, x = M^{-1} u.
// pw: the preconditioner's part of the workspace (ilu0_workspace bytes).
template <typename Run>
int precond_solve(Ctx& c, const sstep_stencil& A, double* x, const sstep_options& o, char* pw,
                  Run&& run) {
    const StencilView v = make_view(A);
    const size_t vb = align256((size_t)v.N * 8);
    double* d = reinterpret_cast<double*>(pw);
    double* dinv = reinterpret_cast<double*>(pw + vb);
    double* u = reinterpret_cast<double*>(pw + 2 * vb);
    double* t = reinterpret_cast<double*>(pw + 3 * vb);
    const size_t sb = align256((size_t)ilu0_sweep_points(v) * 8);
    double* wsk = reinterpret_cast<double*>(pw + 4 * vb);
    double* rsk = reinterpret_cast<double*>(pw + 4 * vb + sb);
    double* sk = reinterpret_cast<double*>(pw + 4 * vb + 2 * sb);
    int* bad = reinterpret_cast<int*>(pw + 4 * vb + ilu0_sweep_bytes(A));
    ilu0_factor_launch(c, v, d, dinv, bad);
    int hb = 0;
    SSTEP_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, c.st));
    SSTEP_HIP(hipStreamSynchronize(c.st));
    if (hb) return SSTEP_ERR_BREAKDOWN;
    ilu0_skew_launch(c, v, dinv, sk);
    ilu0_mul_launch(c, v, d, dinv, x, u);
    sstep_options o2 = o;
    if (o2.sigma == 0.0) o2.sigma = 1.0;  // A M^{-1} is close to the identity
    const Ilu0 P{d, dinv, t, sk, wsk, rsk};
    c.pc = &P;
    int st;
    try {
        st = run(u, o2);
    } catch (...) {
        c.pc = nullptr;
        throw;
    }
    c.pc = nullptr;
    ilu0_solve_launch(c, v, sk, wsk, rsk, u, x, nullptr);
    return st;
}
}  // namespace

// Workspace of sstep_gmres_solve_noalloc: a static device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name
// as an address (on the host it is a stand-in, not a device pointer): the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and is what the kernels receive.
static __device__ __align__(256) unsigned char scratch[SSTEP_NOALLOC_MAX_WORKSPACE];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, null until set up

// Device address of the current device's scratch array (set up on first use).
int scratch_ptr(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return SSTEP_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SSTEP_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SSTEP_OK;
}
}  // namespace

extern "C" {

void sstep_default_options(sstep_options* opt) {
    if (opt) std::memset(opt, 0, sizeof(*opt));
}

const char* sstep_status_string(int status) {
    switch (status) {
        case SSTEP_OK: return "converged";
        case SSTEP_NOT_CONVERGED: return "not converged (iteration cap)";
        case SSTEP_ERR_ARG: return "invalid argument";
        case SSTEP_ERR_BREAKDOWN: return "breakdown (singular Gram matrix)";
        case SSTEP_ERR_NONFINITE: return "non-finite value";
        case SSTEP_ERR_HIP: return "HIP runtime error";
        case SSTEP_ERR_NOMEM: return "out of memory / workspace too small";
        default: return "unknown status";
    }
}

size_t sstep_workspace_bytes(const sstep_stencil* A, int method, int s, int k_or_m,
                             int precision) {
    if (!stencil_ok(A) || s < 1 || s > kMaxS || k_or_m < 1) return 0;
    if (method == SSTEP_METHOD_GMRES) {
        if ((long long)k_or_m * s > 2048) return 0;
        if (precision != SSTEP_FP64 && precision != SSTEP_MIXED) return 0;
        return gmres_workspace_bytes(*A, s, k_or_m, precision);
    }
    if (method == SSTEP_METHOD_OMIN) {
        if (k_or_m > 64 || precision != SSTEP_FP64) return 0;
        return omin_workspace_bytes(*A, s, k_or_m);
    }
    return 0;
}

static bool gmres_args_ok(const sstep_stencil* A, const double* f, const double* x, int s, int m,
                          double tol, const sstep_options* opt) {
    const int prec = opt ? opt->precision : SSTEP_FP64;
    const int basis = opt ? opt->basis : SSTEP_BASIS_MONOMIAL;
    return stencil_ok(A) && f && x && !((uintptr_t)f & 15u) && !((uintptr_t)x & 15u) && s >= 1 &&
           s <= kMaxS && m >= 1 && (long long)m * s <= 2048 && tol >= 0.0 &&
           (prec == SSTEP_FP64 || prec == SSTEP_MIXED) &&
           (basis == SSTEP_BASIS_MONOMIAL || basis == SSTEP_BASIS_CHEBYSHEV ||
            basis == SSTEP_BASIS_NEWTON) &&
           !(opt && (opt->max_iters < 0 || !(opt->sigma >= 0.0) || !(opt->inner_tol >= 0.0) ||
                     opt->orth != SSTEP_ORTH_CHOL)) &&
           precond_ok(A, opt, prec, basis);
}

// Workspace of an s-GMRES solve: the method's part, then the preconditioner's.
static size_t gmres_need(const sstep_stencil& A, int s, int m, const sstep_options* opt,
                         size_t* base) {
    *base = gmres_workspace_bytes(A, s, m, opt ? opt->precision : SSTEP_FP64);
    const bool pc = opt && opt->precond == SSTEP_PRECOND_ILU0;
    return *base + (pc ? ilu0_workspace(A) : 0);
}

static int gmres_dispatch(Ctx& c, const sstep_stencil& A, const double* f, double* x, int s, int m,
                          double tol, const sstep_options& o, sstep_info* info, void* ws,
                          size_t wsb, size_t base) {
    if (o.precond != SSTEP_PRECOND_ILU0) return gmres_solve_impl(c, A, f, x, s, m, tol, o, info, ws, wsb);
    return precond_solve(c, A, x, o, (char*)ws + base, [&](double* u, const sstep_options& o2) {
        return gmres_solve_impl(c, A, f, u, s, m, tol, o2, info, ws, base);
    });
}

int sstep_gmres_solve(const sstep_stencil* A, const double* f, double* x, int s, int m,
                      double tol, const sstep_options* opt, sstep_info* info) {
    if (!gmres_args_ok(A, f, x, s, m, tol, opt)) {
        if (info) std::memset(info, 0, sizeof(*info));
        return set_status(info, SSTEP_ERR_ARG);
    }
    size_t base = 0;
    const size_t need = gmres_need(*A, s, m, opt, &base);
    const sstep_stencil Acopy = *A;
    return run_solver(opt, need, info, [&](Ctx& c, const sstep_options& o, void* ws, size_t wsb) {
        return gmres_dispatch(c, Acopy, f, x, s, m, tol, o, info, ws, wsb, base);
    });
}

int sstep_gmres_solve_noalloc(const sstep_stencil* A, const double* f, double* x, int s, int m,
                              double tol, const sstep_options* opt, sstep_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (!gmres_args_ok(A, f, x, s, m, tol, opt) ||
        (opt && (opt->workspace || opt->profile || opt->graph)))
        return set_status(info, SSTEP_ERR_ARG);
    size_t base = 0;
    const size_t need = gmres_need(*A, s, m, opt, &base);
    if (need > SSTEP_NOALLOC_MAX_WORKSPACE) return set_status(info, SSTEP_ERR_NOMEM);
    sstep_options o;
    if (opt) o = *opt;
    else sstep_default_options(&o);
    const sstep_stencil Acopy = *A;
    return guarded(info, [&]() -> int {
        void* ws = nullptr;
        const int st = scratch_ptr(&ws);
        if (st != SSTEP_OK) return st;
        Ctx c;
        c.st = (hipStream_t)o.stream;
        c.profile = false;  // no timing events
        return gmres_dispatch(c, Acopy, f, x, s, m, tol, o, info, ws, SSTEP_NOALLOC_MAX_WORKSPACE,
                              base);
    });
}

int sstep_omin_solve(const sstep_stencil* A, const double* f, double* x, int s, int k, double tol,
                     const sstep_options* opt, sstep_info* info) {
    const int prec = opt ? opt->precision : SSTEP_FP64;
    const int basis = opt ? opt->basis : SSTEP_BASIS_MONOMIAL;
    if (!stencil_ok(A) || !f || !x || ((uintptr_t)f & 15u) || ((uintptr_t)x & 15u) || s < 1 ||
        s > kMaxS || k < 1 || k > 64 || !(tol >= 0.0) ||
        prec != SSTEP_FP64 ||
        (basis != SSTEP_BASIS_MONOMIAL && basis != SSTEP_BASIS_CHEBYSHEV &&
         basis != SSTEP_BASIS_NEWTON) ||
        (opt && (opt->max_iters < 0 || !(opt->sigma >= 0.0) ||
                 (opt->orth != SSTEP_ORTH_CHOL && opt->orth != SSTEP_ORTH_MGS))) ||
        !precond_ok(A, opt, prec, basis)) {
        if (info) std::memset(info, 0, sizeof(*info));
        return set_status(info, SSTEP_ERR_ARG);
    }
    const size_t base = omin_workspace_bytes(*A, s, k);
    const bool pc = opt && opt->precond == SSTEP_PRECOND_ILU0;
    const size_t need = base + (pc ? ilu0_workspace(*A) : 0);
    const sstep_stencil Acopy = *A;
    return run_solver(opt, need, info, [&](Ctx& c, const sstep_options& o, void* ws, size_t wsb) {
        if (!pc) return omin_solve_impl(c, Acopy, f, x, s, k, tol, o, info, ws, wsb);
        return precond_solve(c, Acopy, x, o, (char*)ws + base,
                             [&](double* u, const sstep_options& o2) {
                                 return omin_solve_impl(c, Acopy, f, u, s, k, tol, o2, info, ws,
                                                        base);
                             });
    });
}

size_t sstep_precond_workspace_bytes(const sstep_stencil* A, int precond) {
    if (precond != SSTEP_PRECOND_ILU0 || !stencil_ok(A) || !ilu0_supported(*A)) return 0;
    return ilu0_workspace(*A);
}

int sstep_ilu0_factor(const sstep_stencil* A, double* d, void* stream) {
    if (!stencil_ok(A) || !ilu0_supported(*A) || !d || ((uintptr_t)d & 7u)) return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        const StencilView v = make_view(*A);
        int* bad = nullptr;
        SSTEP_HIP(hipMallocAsync((void**)&bad, sizeof(int), c.st));
        ilu0_factor_launch(c, v, d, d + v.N, bad);
        int hb = 0;
        SSTEP_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, c.st));
        SSTEP_HIP(hipFreeAsync(bad, c.st));
        SSTEP_HIP(hipStreamSynchronize(c.st));
        return hb ? SSTEP_ERR_BREAKDOWN : SSTEP_OK;
    });
}

int sstep_ilu0_solve(const sstep_stencil* A, const double* d, const double* r, double* z,
                     void* stream) {
    if (!stencil_ok(A) || !ilu0_supported(*A) || !d || !r || !z || z == r ||
        ((uintptr_t)d & 7u) || ((uintptr_t)r & 7u) || ((uintptr_t)z & 7u))
        return SSTEP_ERR_ARG;
    const long long N = grid_points(*A);
    if ((z < d + 2 * N && d < z + N)) return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        const StencilView v = make_view(*A);
        // the sweeps read 1/d (and the coefficients) in their own layout
        const size_t sb = align256((size_t)ilu0_sweep_points(v) * 8);
        char* buf = nullptr;
        SSTEP_HIP(hipMallocAsync((void**)&buf, ilu0_sweep_bytes(*A), c.st));
        double* wsk = reinterpret_cast<double*>(buf);
        double* rsk = reinterpret_cast<double*>(buf + sb);
        double* sk = reinterpret_cast<double*>(buf + 2 * sb);
        ilu0_skew_launch(c, v, d + v.N, sk);
        ilu0_solve_launch(c, v, sk, wsk, rsk, r, z, nullptr);
        SSTEP_HIP(hipFreeAsync(buf, c.st));
        return SSTEP_OK;
    });
}

int sstep_ilu0_mul(const sstep_stencil* A, const double* d, const double* x, double* u,
                   void* stream) {
    if (!stencil_ok(A) || !ilu0_supported(*A) || !d || !x || !u || u == x ||
        ((uintptr_t)d & 7u) || ((uintptr_t)x & 7u) || ((uintptr_t)u & 7u))
        return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        const StencilView v = make_view(*A);
        ilu0_mul_launch(c, v, d, d + v.N, x, u);
        return SSTEP_OK;
    });
}

static int batch_args_ok(int nsys, const sstep_stencil* A, const double* const* f,
                         double* const* x, int s, int m, double tol, const sstep_options* opt) {
    if (nsys < 1 || !A || !f || !x || s < 1 || s > 8 || m < 1 || m > 128 || m * s > 512 ||
        !(tol >= 0.0))
        return 0;
    if (opt) {
        if (opt->precision != SSTEP_FP64 || opt->basis != SSTEP_BASIS_MONOMIAL ||
            opt->precond != SSTEP_PRECOND_NONE || opt->orth != SSTEP_ORTH_CHOL ||
            opt->max_iters < 0 || !(opt->sigma >= 0.0))
            return 0;
        if (opt->batch_threads != 0 && opt->batch_threads != 256 && opt->batch_threads != 512 &&
            opt->batch_threads != 1024)
            return 0;
        if (opt->batch_wgs_per_cu < 0 || opt->batch_wgs_per_cu > 4) return 0;
        if (opt->batch_team != 0 && opt->batch_team != 1 && opt->batch_team != 2 &&
            opt->batch_team != 4 && opt->batch_team != 8)
            return 0;
        const int gc = opt->batch_gram_cols;
        if (gc != 0 && !(s <= 4 ? (gc == 2 || gc == 4) : (gc == 1 || gc == 2))) return 0;
    }
    for (int i = 0; i < nsys; ++i) {
        if (!stencil_ok(&A[i]) || !f[i] || !x[i]) return 0;
        if (((uintptr_t)f[i] & 15) || ((uintptr_t)x[i] & 15) || ((uintptr_t)A[i].coef & 15)) return 0;
        if (grid_points(A[i]) > (1LL << 30)) return 0;
    }
    return 1;
}

size_t sstep_batch_workspace_bytes(int nsys, const sstep_stencil* A, int s, int m,
                                   const sstep_options* opt) {
    if (nsys < 1 || !A || s < 1 || s > 8 || m < 1 || m > 128 || m * s > 512) return 0;
    for (int i = 0; i < nsys; ++i)
        if (!stencil_ok(&A[i])) return 0;
    const int wpc = (opt && opt->batch_wgs_per_cu > 0) ? opt->batch_wgs_per_cu : 1;
    const int team = (opt && opt->batch_team > 0) ? opt->batch_team : 1;
    return batched_workspace_bytes(nsys, A, s, m, batched_slots(nsys, wpc, team));
}

int sstep_batch_plan_create(sstep_batch_plan* plan, int nsys, const sstep_stencil* A,
                            const double* const* f, double* const* x, int s, int m, double tol,
                            const sstep_options* opt) {
    if (!plan) return SSTEP_ERR_ARG;
    *plan = nullptr;
    if (!batch_args_ok(nsys, A, f, x, s, m, tol, opt)) return SSTEP_ERR_ARG;
    sstep_options o;
    if (opt) o = *opt;
    else sstep_default_options(&o);
    return guarded(nullptr, [&]() -> int {
        void* p = nullptr;
        const int st = batched_plan_create(&p, nsys, A, f, x, s, m, tol, o);
        *plan = (sstep_batch_plan)p;
        return st;
    });
}

int sstep_batch_plan_execute(sstep_batch_plan plan, sstep_info* info) {
    if (!plan) return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int { return batched_plan_execute(plan, info, nullptr); });
}

void sstep_batch_plan_destroy(sstep_batch_plan plan) { batched_plan_destroy(plan); }

int sstep_gmres_solve_batched(int nsys, const sstep_stencil* A, const double* const* f,
                              double* const* x, int s, int m, double tol,
                              const sstep_options* opt, sstep_info* info) {
    sstep_batch_plan plan = nullptr;
    int st = sstep_batch_plan_create(&plan, nsys, A, f, x, s, m, tol, opt);
    if (st != SSTEP_OK) return st;
    st = sstep_batch_plan_execute(plan, info);
    sstep_batch_plan_destroy(plan);
    return st;
}

int sstep_stencil_apply(const sstep_stencil* A, const double* x, double* y, void* stream) {
    if (!stencil_ok(A) || !x || !y || x == y) return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        const StencilView v = make_view(*A);
        launch_level<double>(c, v, x, nullptr, nullptr, nullptr, 1.0, 0.0, 0.0, y, nullptr, 0.0);
        return SSTEP_OK;
    });
}

int sstep_kernel_mpk(const sstep_stencil* A, double* Y, int64_t ldy, int s, int basis,
                     double in_scale, double sigma, double cheb_c, double cheb_d, void* stream) {
    if (!stencil_ok(A) || !Y || s < 1 || s > kMaxS || ldy < grid_points(*A) ||
        (basis != SSTEP_BASIS_MONOMIAL && basis != SSTEP_BASIS_CHEBYSHEV) ||
        !std::isfinite(in_scale) || (basis == SSTEP_BASIS_MONOMIAL && !(sigma != 0.0)) ||
        (basis == SSTEP_BASIS_CHEBYSHEV && !(cheb_d != 0.0)))
        return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        const StencilView v = make_view(*A);
        // the input scale lives in device memory for the solvers; stage it
        double* d = nullptr;
        SSTEP_HIP(hipMallocAsync((void**)&d, sizeof(double), c.st));
        SSTEP_HIP(hipMemcpyAsync(d, &in_scale, sizeof(double), hipMemcpyHostToDevice, c.st));
        OpParams P{sigma, cheb_c, cheb_d};
        launch_mpk<double>(c, v, Y, ldy, s, basis, P, d, nullptr, /*fused_only=*/true);
        SSTEP_HIP(hipFreeAsync(d, c.st));
        SSTEP_HIP(hipStreamSynchronize(c.st));
        return SSTEP_OK;
    });
}

int sstep_kernel_gram(const double* X, int64_t ldx, int ncx, const double* Z, int64_t ldz, int ncz,
                      int64_t N, double* G, void* stream) {
    if (!X || !Z || !G || N < 1 || ncx < 1 || ncz < 1 || ncz > 16 || ldx < N || ldz < N ||
        N > (1LL << 31) - 1 || ncx > 4096)
        return SSTEP_ERR_ARG;
    if (((uintptr_t)X & 15u) || ((uintptr_t)Z & 15u) || (ldx & 1) || (ldz & 1)) return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        double* part = nullptr;
        const size_t np = gram_partial_doubles(N, ncx, ncz);
        SSTEP_HIP(hipMallocAsync((void**)&part, sizeof(double) * np, c.st));
        launch_gram<double>(c, X, ldx, ncx, Z, ldz, ncz, (const double*)nullptr, 0, 0, N, part, G,
                            nullptr);
        SSTEP_HIP(hipFreeAsync(part, c.st));
        SSTEP_HIP(hipStreamSynchronize(c.st));
        return SSTEP_OK;
    });
}

int sstep_kernel_update(const double* X, int64_t ldx, int ncx, double* Y, int64_t ldy, int ncy,
                        const double* M, int64_t N, void* stream) {
    if ((ncx > 0 && (!X || !M || ldx < N)) || !Y || N < 1 || ncx < 0 || ncy < 1 || ncy > 16 ||
        ldy < N || N > (1LL << 31) - 1)
        return SSTEP_ERR_ARG;
    if ((ncx > 0 && (((uintptr_t)X & 15u) || (ldx & 1))) || ((uintptr_t)Y & 15u) || (ldy & 1))
        return SSTEP_ERR_ARG;
    return guarded(nullptr, [&]() -> int {
        Ctx c;
        c.st = (hipStream_t)stream;
        launch_update<double, double, double, double, false>(c, N, Y, ldy, X, ldx, ncx, nullptr, M,
                                                             Y, ldy, ncy, nullptr, nullptr, 0.0);
        return SSTEP_OK;
    });
}

}  // extern "C"
