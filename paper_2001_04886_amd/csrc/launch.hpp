// launch.hpp -- host-side launch helpers, per-launch profiling records,
// operator parameters (power scaling, Chebyshev interval) and workspace
// carving shared by the solver drivers.
#pragma once

#include <atomic>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/sstep.h"
#include "dense.hpp"
#include "gram_self.hpp"
#include "kernels.hpp"
#include "mpk.hpp"
#include "mpk3d.hpp"

namespace sstep {

#define SSTEP_HIP(call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) throw HipFailure{e_, #call}; \
    } while (0)

struct HipFailure {
    hipError_t err;
    const char* what;
};

inline long long round_up(long long v, long long a) { return (v + a - 1) / a * a; }

inline long long grid_points(const sstep_stencil& A) {
    return (long long)A.nx * A.ny * (A.ndim == 3 ? A.nz : 1);
}

inline StencilView make_view(const sstep_stencil& A) {
    StencilView v;
    v.ndim = A.ndim;
    v.nx = A.nx;
    v.ny = A.ny;
    v.nz = A.ndim == 3 ? A.nz : 1;
    v.N = grid_points(A);
    for (int q = 0; q < 7; ++q) v.c[q] = A.c[q];
    v.coef = A.coef;
    return v;
}

// Column stride of basis blocks: a multiple of 64 elements (256 bytes FP32,
// 512 bytes FP64) so every column starts aligned for 16-byte vector access,
// plus 256 elements.  Without the extra elements a power-of-two grid (256^3:
// 2^24 points) puts the same point of every column at addresses that agree in
// their low 27 bits, and the block Gram's hundreds of concurrent column
// streams crowd the same HBM channels: the Gram ran at 6.18 TB/s, with the
// padding at 6.49 (a 2 KiB offset per column; 256 bytes gave 6.32, 4 KiB was
// slower than none in the update).
inline long long col_stride(long long N) { return round_up(std::max(N, 1LL), 64) + 256; }

// One profiled launch: class, algorithmic bytes, the block of the restart
// cycle it belongs to (-1: always executed), and the event index before it.
struct LaunchRec {
    int cls;
    double bytes;
    int block;
    int ev;
};

// Sum of this thread's share of n partial sums (threads stride by kThreads),
// eight independent accumulators so that eight loads are in flight at once,
// combined in a fixed order.
__device__ __forceinline__ double strided_partial_sum(const double* __restrict__ part, int n) {
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 7 * kThreads < n; i += 8 * kThreads) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += part[i + u * kThreads];
    }
    for (; i < n; i += kThreads) acc[0] += part[i];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// ILU(0) right preconditioner of a 2-D five-point operator (Sec. 5): pivots,
// their reciprocals, and a scratch vector for M^{-1} of one vector.
struct Ilu0 {
    const double* d;
    const double* dinv;
    double* t;
    const double* sk;  // 1/d (and the four neighbour coefficients) in the sweep layout
    double* wsk;       // sweep intermediate in the sweep layout
    double* rsk;       // right-hand side of a solve in the sweep layout
};
constexpr int kIluMaxNx = 1024;

struct Ctx {
    hipStream_t st = nullptr;
    bool profile = false;
    std::vector<hipEvent_t> pool;
    int nev = 0;
    std::vector<LaunchRec> recs;
    int cur_block = -1;
    // set while a solve runs on the right-preconditioned operator A M^{-1}:
    // matrix powers and residuals apply M^{-1} first (FP64 only)
    const Ilu0* pc = nullptr;
    // totals
    long long launches[SSTEP_K_NCLASS] = {0};
    double ms[SSTEP_K_NCLASS] = {0};
    double bytes[SSTEP_K_NCLASS] = {0};

    ~Ctx() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t next_event() {
        if (nev == (int)pool.size()) {
            hipEvent_t e;
            SSTEP_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[nev++];
    }
    // call before a kernel launch
    void begin(int cls, double bytes_) {
        if (!profile) return;
        if (recs.empty() || recs.back().ev + 1 != nev) {
            SSTEP_HIP(hipEventRecord(next_event(), st));
        }
        recs.push_back({cls, bytes_, cur_block, nev - 1});
    }
    // call after a kernel launch
    void end() {
        if (!profile) return;
        SSTEP_HIP(hipEventRecord(next_event(), st));
    }
    // algorithmic bytes of a launch whose size was only known after it ran
    void add_bytes(int cls, double b) {
        if (profile) bytes[cls] += b;
    }
    // after a stream synchronize: fold records of executed blocks into totals
    // (blocks_done: blocks of the cycle that ran; launches of later blocks
    // exited at their first instruction and are not counted).
    void harvest(int blocks_done) {
        if (!profile) return;
        for (const auto& r : recs) {
            if (r.block >= 0 && r.block >= blocks_done) continue;
            float t = 0.f;
            SSTEP_HIP(hipEventElapsedTime(&t, pool[r.ev], pool[r.ev + 1]));
            launches[r.cls] += 1;
            ms[r.cls] += t;
            bytes[r.cls] += r.bytes;
        }
        recs.clear();
        nev = 0;
    }
};

// ---------------------------------------------------------------------------
// operator-derived parameters (host side)
// ---------------------------------------------------------------------------
inline double pow2_ceil(double b) {
    if (!(b > 0.0)) return 1.0;
    int e;
    const double m = std::frexp(b, &e);
    return m == 0.5 ? std::ldexp(1.0, e - 1) : std::ldexp(1.0, e);
}

// Gershgorin row-sum maximum and Chebyshev interval from device coefficients.
static __global__ __launch_bounds__(kThreads) void k_coef_bounds(StencilView A,
                                                                 double* __restrict__ part) {
    __shared__ double lds[4 * 3];
    const int nq = 2 * A.ndim + 1;
    double rmax = 0.0, lo = 1e300, hi = -1e300;
    for (long long p = (long long)blockIdx.x * kThreads + threadIdx.x; p < A.N;
         p += (long long)gridDim.x * kThreads) {
        double r = 0.0;
        for (int q = 1; q < nq; ++q) r += fabs(A.coef[q * A.N + p]);
        const double c0 = A.coef[p];
        rmax = fmax(rmax, r + fabs(c0));
        lo = fmin(lo, c0 - r);
        hi = fmax(hi, c0 + r);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
        lds[wave * 3 + 0] = rmax;
        lds[wave * 3 + 1] = lo;
        lds[wave * 3 + 2] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = lds[0], b = lds[1], c = lds[2];
        for (int w = 1; w < 4; ++w) {
            a = fmax(a, lds[w * 3]);
            b = fmin(b, lds[w * 3 + 1]);
            c = fmax(c, lds[w * 3 + 2]);
        }
        part[blockIdx.x * 3 + 0] = a;
        part[blockIdx.x * 3 + 1] = b;
        part[blockIdx.x * 3 + 2] = c;
    }
}

struct OpParams {
    double sigma, cc, cd;
    double th[kMaxS];  // Newton-basis shifts (SSTEP_BASIS_NEWTON)
};

// Newton-basis shifts: the s Chebyshev points cc + cd cos((2k+1) pi / (2s)) of
// the spectral interval in Leja order -- first the point of largest modulus,
// then each time the one maximising the product of distances to the points
// already taken (ties to the smaller k).
inline void newton_shifts(int s, double cc, double cd, double* th) {
    double pts[kMaxS];
    bool used[kMaxS] = {};
    for (int k = 0; k < s; ++k) pts[k] = cc + cd * std::cos((2.0 * k + 1.0) * M_PI / (2.0 * s));
    for (int n = 0; n < s; ++n) {
        int best = -1;
        double bv = -1.0;
        for (int k = 0; k < s; ++k) {
            if (used[k]) continue;
            double v = 1.0;
            if (n == 0) v = std::fabs(pts[k]);
            else
                for (int j = 0; j < n; ++j) v *= std::fabs(pts[k] - th[j]);
            if (v > bv) {
                bv = v;
                best = k;
            }
        }
        used[best] = true;
        th[n] = pts[best];
    }
}

// sigma: smallest power of two >= max_p sum_q |a_pq| (exact scaling);
// Chebyshev interval: for constant coefficients the spectrum of the symmetric
// part (per axis cos(pi/(n+1)) times |c_- + c_+|), else a Gershgorin interval.
inline OpParams op_params(const sstep_stencil& A, double sigma_opt, hipStream_t st,
                          double* dev_scratch /* >= 3*64 doubles */) {
    OpParams P{};
    const int nd = A.ndim == 3 ? 3 : 2;
    if (!A.coef) {
        double b = 0.0;
        for (int q = 0; q < 2 * nd + 1; ++q) b += std::fabs(A.c[q]);
        P.sigma = pow2_ceil(b);
        const int n[3] = {A.nx, A.ny, A.ndim == 3 ? A.nz : 1};
        double hw = 0.0;
        for (int a = 0; a < nd; ++a)
            hw += std::fabs(A.c[1 + 2 * a] + A.c[2 + 2 * a]) * std::cos(M_PI / (n[a] + 1));
        P.cc = A.c[0];
        P.cd = hw;
    } else {
        const StencilView v = make_view(A);
        hipLaunchKernelGGL(k_coef_bounds, dim3(64), dim3(kThreads), 0, st, v, dev_scratch);
        SSTEP_HIP(hipGetLastError());
        double h[64 * 3];
        SSTEP_HIP(hipMemcpyAsync(h, dev_scratch, sizeof(h), hipMemcpyDeviceToHost, st));
        SSTEP_HIP(hipStreamSynchronize(st));
        double a = 0.0, lo = 1e300, hi = -1e300;
        for (int b = 0; b < 64; ++b) {
            a = std::max(a, h[3 * b]);
            lo = std::min(lo, h[3 * b + 1]);
            hi = std::max(hi, h[3 * b + 2]);
        }
        P.sigma = pow2_ceil(a);
        P.cc = 0.5 * (lo + hi);
        P.cd = 0.5 * (hi - lo);
    }
    if (!(P.cd > 0.0)) P.cd = std::fabs(P.cc) > 0.0 ? std::fabs(P.cc) : 1.0;
    if (sigma_opt > 0.0) P.sigma = sigma_opt;
    return P;
}

// Basis change B ((s+1) x s, column-major ld s+1): A Y[:, 0:s] = Y B.
inline void basis_matrix(int s, int basis, const OpParams& P, double* B) {
    std::memset(B, 0, sizeof(double) * (s + 1) * s);
    for (int j = 0; j < s; ++j) {
        if (basis == SSTEP_BASIS_NEWTON) {  // A y_j = cd y_{j+1} + th_j y_j
            B[j + j * (s + 1)] = P.th[j];
            B[(j + 1) + j * (s + 1)] = P.cd;
        } else if (basis == SSTEP_BASIS_CHEBYSHEV) {
            if (j == 0) {
                B[0] = P.cc;
                B[1] = P.cd;
            } else {
                B[(j - 1) + j * (s + 1)] = 0.5 * P.cd;
                B[j + j * (s + 1)] = P.cc;
                B[(j + 1) + j * (s + 1)] = 0.5 * P.cd;
            }
        } else {
            B[(j + 1) + j * (s + 1)] = P.sigma;
        }
    }
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
inline int stencil_segments(const StencilView& v) { return (v.nx + kThreads - 1) / kThreads; }
inline long long stencil_blocks(const StencilView& v) {
    return (long long)stencil_segments(v) * v.ny * v.nz;
}

template <typename T>
inline void launch_level(Ctx& c, const StencilView& v, const T* in, const double* in_scale,
                         const T* prev, const double* prev_scale, double alpha, double beta,
                         double gam, T* out, const int* skip, double bytes) {
    c.begin(SSTEP_K_MPK, bytes);
    const int nseg = stencil_segments(v);
    hipLaunchKernelGGL(k_stencil_level<T>, dim3((unsigned)stencil_blocks(v)), dim3(kThreads), 0,
                       c.st, v, nseg, in, in_scale, prev, prev_scale, alpha, beta, gam, out, skip);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

// Compute units of the current device (cached per device).
inline int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

// Fused matrix-powers geometry: plane tiles (exact interiors of 32 x 32
// points in 3-D, 256-point row segments in 2-D) times chunks of the march
// axis; each chunk also computes L planes on either side.  3-D: the chunk
// count minimises (rounds of workgroups per compute unit) x (planes marched
// per workgroup), the time of the most loaded compute unit -- on a 256^3 grid
// that is one 64-plane chunk per compute unit.  2-D (short workgroups that
// need company on a compute unit to cover memory latency): about 1024
// workgroups.
struct MpkGeom {
    int ntx, nty, zchunk, nzc;
    long long wgs() const { return (long long)ntx * nty * nzc; }
};
inline MpkGeom mpk_geometry(const StencilView& v, int L) {
    const bool d3 = v.ndim == 3;
    const int IX = d3 ? 32 : 256, IY = d3 ? 32 : 1;
    MpkGeom g;
    g.ntx = (v.nx + IX - 1) / IX;
    g.nty = d3 ? (v.ny + IY - 1) / IY : 1;
    const int nmarch = d3 ? v.nz : v.ny;
    const long long tiles = (long long)g.ntx * g.nty;
    const int minchunk = (d3 ? 2 : 4) * L;
    if (d3) {
        const long long ncu = device_cus();
        long long best = -1;
        g.zchunk = nmarch;
        for (int n = 1; n <= std::max(1, nmarch / minchunk); ++n) {
            const int zc = (nmarch + n - 1) / n;
            const long long nz = (nmarch + zc - 1) / zc;
            const long long cost = ((tiles * nz + ncu - 1) / ncu) * (zc + 2 * L);
            if (best < 0 || cost < best) {
                best = cost;
                g.zchunk = zc;
            }
        }
    } else {
        const long long nch = std::max<long long>(1, (1024 + tiles - 1) / tiles);
        g.zchunk = (int)std::max<long long>(minchunk, (nmarch + nch - 1) / nch);
    }
    g.nzc = (nmarch + g.zchunk - 1) / g.zchunk;
    return g;
}

// Grids too small for a fused pass: even with the shortest chunks it would
// have fewer than 512 workgroups (a few hundred rows; their vectors sit in L2).
inline bool mpk_small_grid(const StencilView& v, int L) {
    const bool d3 = v.ndim == 3;
    const int IX = d3 ? 32 : 256, IY = d3 ? 32 : 1;
    const long long tiles = (long long)((v.nx + IX - 1) / IX) * (d3 ? (v.ny + IY - 1) / IY : 1);
    const int nmarch = d3 ? v.nz : v.ny, minchunk = (d3 ? 2 : 4) * L;
    return tiles * ((nmarch + minchunk - 1) / minchunk) < 512;
}

// The fused kernel addresses one plane of a vector (and of a coefficient
// field, FP64) with 32-bit byte offsets.
inline bool mpk_fused_fits(const StencilView& v) {
    const long long plane = v.ndim == 3 ? (long long)v.nx * v.ny : v.nx;
    return plane * 8 < (1LL << 31);
}

template <typename T, int DIM, int L>
inline void mpk_go(Ctx& c, const StencilView& v, T* out0, long long ldo, const T* in,
                   const double* in_scale, const T* prev, const double* prev_scale,
                   const MpkLevels& lv, const int* skip) {
    const MpkGeom g = mpk_geometry(v, L);
    const dim3 grid((unsigned)g.wgs()), block(MpkTile<DIM, L>::THREADS);
    if (v.coef)
        hipLaunchKernelGGL((k_mpk_fused<T, DIM, L, true>), grid, block, 0, c.st, v, out0, ldo, in,
                           in_scale, prev, prev_scale, lv, g.ntx, g.nty, g.zchunk, skip);
    else
        hipLaunchKernelGGL((k_mpk_fused<T, DIM, L, false>), grid, block, 0, c.st, v, out0, ldo, in,
                           in_scale, prev, prev_scale, lv, g.ntx, g.nty, g.zchunk, skip);
}

// 3-D constant-coefficient matrix powers (mpk3d.hpp): up to kMpk3L levels per
// pass on tiles of 64 x 64 points (56 x 56 exact).  Tile shape per variant:
// 4 rows x 16 waves, or 4 rows x 8 waves when the first level also reads
// y_{-1} (more registers per row).
constexpr int kMpk3L = 4;
using Mpk3Geom = Mpk3Tile<kMpk3L, 4, 16>;
static_assert(Mpk3Tile<kMpk3L, 4, 8>::IX == Mpk3Geom::IX, "same x interior");

inline bool mpk3_applies(const StencilView& v) { return v.ndim == 3 && !v.coef && mpk_fused_fits(v); }

// Grids too small for the register-tile kernel: fewer than 128 workgroups even
// with the shortest chunks.
inline bool mpk3_small_grid(const StencilView& v) {
    const long long tiles = (long long)((v.nx + Mpk3Geom::IX - 1) / Mpk3Geom::IX) *
                            ((v.ny + Mpk3Geom::IY - 1) / Mpk3Geom::IY);
    return tiles * ((v.nz + 2 * kMpk3L - 1) / (2 * kMpk3L)) < 128;
}

template <typename T, int L, int POS, int W, bool PREV, bool UNI, bool BETA, bool GAM>
inline void mpk3_launch(Ctx& c, const StencilView& v, T* out0, long long ldo, const T* in,
                        const double* in_scale, const T* prev, const double* prev_scale,
                        const MpkLevels& lv, const int* skip) {
    using G = Mpk3Tile<L, POS, W>;
    const auto kern = k_mpk3d<T, L, POS, W, PREV, UNI, BETA, GAM>;
    const int ntx = (v.nx + G::IX - 1) / G::IX, nty = (v.ny + G::IY - 1) / G::IY;
    const long long tiles = (long long)ntx * nty;
    // chunks along z: minimise (rounds of resident workgroups) x (steps per
    // workgroup), the time of the most loaded compute unit
    static const int occ = [&] {  // resident workgroups per compute unit, queried once
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, G::THREADS, 0) != hipSuccess)
            n = 1;
        return std::max(1, n);
    }();
    const long long slots = (long long)device_cus() * occ;
    int zchunk = v.nz;
    long long best = -1;
    for (int n = 1; n <= std::max(1, v.nz / (2 * L)); ++n) {
        const int zc = (v.nz + n - 1) / n;
        const long long nzc = (v.nz + zc - 1) / zc;
        const long long cost = ((tiles * nzc + slots - 1) / slots) * (zc + 2 * L);
        if (best < 0 || cost < best) {
            best = cost;
            zchunk = zc;
        }
    }
    const int nzc = (v.nz + zchunk - 1) / zchunk;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * nzc)), dim3(G::THREADS), 0, c.st, v, out0,
                       ldo, in, in_scale, prev, prev_scale, lv, ntx, nty, zchunk, skip);
}

template <typename T, int L>
inline void mpk3_go(Ctx& c, const StencilView& v, T* out0, long long ldo, const T* in,
                    const double* in_scale, const T* prev, const double* prev_scale,
                    const MpkLevels& lv, const int* skip) {
    bool uni = true, beta = false, gam = false;
    for (int j = 0; j < L; ++j) {
        uni = uni && lv.alpha[j] == lv.alpha[0];
        beta = beta || lv.beta[j] != 0.0;
        gam = gam || lv.gam[j] != 0.0;
    }
    const bool pv = prev != nullptr && lv.gam[0] != 0.0;
    constexpr int WP = sizeof(T) == 8 ? 8 : 16;  // waves with y_{-1}
#define SSTEP_MPK3(W_, PV, UN, BE, GA) \
    mpk3_launch<T, L, 4, W_, PV, UN, BE, GA>(c, v, out0, ldo, in, in_scale, prev, prev_scale, lv, skip)
    if (pv && !uni) throw HipFailure{hipErrorInvalidValue, "mpk3 level scales"};
    if (pv) SSTEP_MPK3(WP, true, true, true, true);                      // three-term, continued
    else if (!beta && !gam && uni) SSTEP_MPK3(16, false, true, false, false);  // monomial
    else if (!gam && uni) SSTEP_MPK3(16, false, true, true, false);            // Newton
    else if (!gam) SSTEP_MPK3(16, false, false, true, false);  // two-term, scales differ
    else SSTEP_MPK3(16, false, false, true, true);             // three-term, first pass
#undef SSTEP_MPK3
}

// Level coefficients of the monomial / Chebyshev recurrence at global level
// lev = 1..s: y_lev = alpha A y_{lev-1} + beta y_{lev-1} + gam y_{lev-2}.
inline void mpk_level_coefs(int lev, int basis, const OpParams& P, double* a, double* b,
                            double* g) {
    if (basis == SSTEP_BASIS_NEWTON) {  // y_lev = (A - th_{lev-1}) y_{lev-1} / cd
        *a = 1.0 / P.cd;
        *b = -P.th[lev - 1] / P.cd;
        *g = 0.0;
    } else if (basis == SSTEP_BASIS_CHEBYSHEV) {
        *a = (lev == 1 ? 1.0 : 2.0) / P.cd;
        *b = -(lev == 1 ? 1.0 : 2.0) * P.cc / P.cd;
        *g = lev == 1 ? 0.0 : -1.0;
    } else {
        *a = 1.0 / P.sigma;
        *b = 0.0;
        *g = 0.0;
    }
}

// ILU(0) kernels (ilu.hip).
bool ilu0_supported(const sstep_stencil& A);
void ilu0_factor_launch(Ctx& c, const StencilView& v, double* d, double* dinv, int* bad);
long long ilu0_sweep_points(const StencilView& v);
void ilu0_skew_launch(Ctx& c, const StencilView& v, const double* dinv, double* sk);
void ilu0_solve_launch(Ctx& c, const StencilView& v, const double* sk, double* wsk,
                       double* rsk, const double* r, double* z, const int* skip);
void ilu0_mul_launch(Ctx& c, const StencilView& v, const double* d, const double* dinv,
                     const double* x, double* u);
void ilu0_level_launch(Ctx& c, const StencilView& v, const double* in, const double* in_scale,
                       const double* prev, const double* prev_scale, double alpha, double beta,
                       double gam, const double* t, double* out, const int* skip, double bytes);

// Matrix powers of column 0 of Y into columns 1..s: fused launches of at
// most kMpkMaxL levels each.  Column 0 is read with in_scale applied.  Grids
// too small to give a fused launch 512 workgroups (a few hundred rows) run one
// stencil launch per level instead (unless fused_only): their vectors sit in
// L2, and a fused pass would march few workgroups through many halo rows.
// So do planes of 2^28 points or more, which the fused kernel cannot address.
template <typename T>
inline void launch_mpk(Ctx& c, const StencilView& v, T* Y, long long ldy, int s, int basis,
                       const OpParams& P, const double* in_scale, const int* skip,
                       bool fused_only = false) {
    const double vb = (double)v.N * sizeof(T);
    if constexpr (std::is_same<T, double>::value) {
        if (c.pc) {
            // right-preconditioned operator: per level t = M^{-1} y_{lev-1},
            // then the level's stencil on t
            for (int lev = 1; lev <= s; ++lev) {
                double a, b, g;
                mpk_level_coefs(lev, basis, P, &a, &b, &g);
                const double* in = Y + (long long)(lev - 1) * ldy;
                const double* prev = lev >= 2 ? Y + (long long)(lev - 2) * ldy : nullptr;
                ilu0_solve_launch(c, v, c.pc->sk, c.pc->wsk, c.pc->rsk, in, c.pc->t, skip);
                ilu0_level_launch(c, v, in, lev == 1 ? in_scale : nullptr, prev,
                                  lev == 2 ? in_scale : nullptr, a, b, g, c.pc->t,
                                  Y + (long long)lev * ldy, skip, vb * (lev == 1 ? 2.0 : 1.0));
            }
            return;
        }
    }
    const bool r3 = mpk3_applies(v);
    const int L0 = v.ndim == 3 ? std::min(s, 2) : (s >= 8 ? 8 : (s >= 6 ? 6 : (s >= 4 ? 4 : s)));
    const bool small = r3 ? mpk3_small_grid(v) : mpk_small_grid(v, L0);
    if ((!fused_only && small) || !mpk_fused_fits(v)) {
        for (int lev = 1; lev <= s; ++lev) {
            double a, b, g;
            mpk_level_coefs(lev, basis, P, &a, &b, &g);
            const T* in = Y + (long long)(lev - 1) * ldy;
            const T* prev = lev >= 2 ? Y + (long long)(lev - 2) * ldy : nullptr;
            // algorithmic bytes of the whole call: read 1, write s
            launch_level<T>(c, v, in, lev == 1 ? in_scale : nullptr, prev,
                            lev == 2 ? in_scale : nullptr, a, b, g, Y + (long long)lev * ldy,
                            skip, vb * (lev == 1 ? 2.0 : 1.0));
        }
        return;
    }
    int j0 = 0;
    while (j0 < s) {
        const int left = s - j0;
        // 2-D: up to 8 levels per pass; 3-D constant coefficients: up to 4
        // (mpk3d.hpp); 3-D variable coefficients: 2 (seven coefficient planes
        // per level are loaded too)
        const int L = r3 ? std::min(left, kMpk3L)
                         : v.ndim == 3 ? std::min(left, 2)
                                       : (left >= 8 ? 8 : (left >= 6 ? 6 : (left >= 4 ? 4 : left)));
        MpkLevels lv;
        for (int j = 0; j < L; ++j)  // global level index j0 + j + 1
            mpk_level_coefs(j0 + j + 1, basis, P, &lv.alpha[j], &lv.beta[j], &lv.gam[j]);
        const T* in = Y + (long long)j0 * ldy;
        const double* isc = j0 == 0 ? in_scale : nullptr;
        const T* prev = j0 >= 1 ? Y + (long long)(j0 - 1) * ldy : nullptr;
        const double* psc = j0 == 1 ? in_scale : nullptr;
        T* out0 = Y + (long long)(j0 + 1) * ldy;
        // algorithmic bytes of the whole MPK call: read 1, write s
        c.begin(SSTEP_K_MPK, vb * (L + (j0 == 0 ? 1.0 : 0.0)));
#define SSTEP_MPK(D, LL) mpk_go<T, D, LL>(c, v, out0, ldy, in, isc, prev, psc, lv, skip)
        if (r3) {
            switch (L) {
                case 4: mpk3_go<T, 4>(c, v, out0, ldy, in, isc, prev, psc, lv, skip); break;
                case 3: mpk3_go<T, 3>(c, v, out0, ldy, in, isc, prev, psc, lv, skip); break;
                case 2: mpk3_go<T, 2>(c, v, out0, ldy, in, isc, prev, psc, lv, skip); break;
                default: mpk3_go<T, 1>(c, v, out0, ldy, in, isc, prev, psc, lv, skip); break;
            }
        } else if (v.ndim == 3) {
            if (L == 2) SSTEP_MPK(3, 2);
            else SSTEP_MPK(3, 1);
        } else {
            switch (L) {
                case 8: SSTEP_MPK(2, 8); break;
                case 6: SSTEP_MPK(2, 6); break;
                case 4: SSTEP_MPK(2, 4); break;
                case 3: SSTEP_MPK(2, 3); break;
                case 2: SSTEP_MPK(2, 2); break;
                default: SSTEP_MPK(2, 1); break;
            }
        }
#undef SSTEP_MPK
        SSTEP_HIP(hipGetLastError());
        c.end();
        j0 += L;
    }
}

template <typename TR>
inline void launch_residual(Ctx& c, const StencilView& v, const double* f, const double* x, TR* r,
                            double* part) {
    if (c.pc) {  // x is the preconditioned unknown u: the residual is f - A M^{-1} u
        ilu0_solve_launch(c, v, c.pc->sk, c.pc->wsk, c.pc->rsk, x, c.pc->t, nullptr);
        x = c.pc->t;
    }
    c.begin(SSTEP_K_RESID, (double)v.N * (16.0 + sizeof(TR)));
    const int nseg = stencil_segments(v);
    hipLaunchKernelGGL(k_residual<TR>, dim3((unsigned)stencil_blocks(v)), dim3(kThreads), 0, c.st,
                       v, nseg, f, x, r, part);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

// Gram geometry: column-tile width for a given Z width, and the point chunk.
// X columns per wave of the Gram kernel (a workgroup takes 4 waves' worth)
constexpr int gram_ca_c(int kz) { return kz <= 9 ? 4 : 2; }
inline int gram_ca(int kz) { return gram_ca_c(kz); }
inline int gram_kz(int nz) {
    static const int ks[] = {1, 2, 4, 8, 9, 12, 13, 16, 17};
    for (int k : ks)
        if (nz <= k) return k;
    return -1;
}
inline void gram_geometry(long long N, int ncx, int nz, int* KZ, int* CA, int* nct, int* nchunk,
                          long long* chunk) {
    *KZ = gram_kz(nz);
    *CA = gram_ca(*KZ);
    *nct = (ncx + 4 * *CA - 1) / (4 * *CA);
    // chunks of at least 2048 points (16 steps of the kernel), about 2048
    // workgroups in all on large grids
    long long nch = std::min<long long>((N + 2047) / 2048, std::max(1, 2048 / *nct));
    nch = std::max<long long>(1, std::min<long long>(nch, 512));
    long long ck = round_up((N + nch - 1) / nch, 512);
    nch = (N + ck - 1) / ck;
    *nchunk = (int)std::max<long long>(nch, 1);
    *chunk = ck;
}
inline size_t gram_partial_doubles(long long N, int ncx, int nz) {
    int KZ, CA, nct, nchunk;
    long long chunk;
    gram_geometry(N, ncx, nz, &KZ, &CA, &nct, &nchunk, &chunk);
    return (size_t)nchunk * ncx * KZ;
}

template <typename T, int CA, int KZ>
inline void gram_go(Ctx& c, const T* X, long long ldx, int ncx, const T* Z1, long long ldz1,
                    int nz1, const T* Z2, long long ldz2, int nz2, long long N, long long chunk,
                    int nct, int nchunk, double* part, const int* skip) {
    hipLaunchKernelGGL((k_gram_partial<T, CA, KZ>), dim3((unsigned)(nct * nchunk)),
                       dim3(kThreads), 0, c.st, X, ldx, ncx, Z1, ldz1, nz1, Z2, ldz2, nz2, N, chunk,
                       nct, part, skip);
}

// G (ncx x (nz1+nz2), row-major) = X^T [Z1 | Z2]
template <typename T>
inline void launch_gram(Ctx& c, const T* X, long long ldx, int ncx, const T* Z1, long long ldz1,
                        int nz1, const T* Z2, long long ldz2, int nz2, long long N, double* part,
                        double* G, const int* skip, int cls = SSTEP_K_GRAM, bool reduce = true) {
    const int nz = nz1 + nz2;
    int KZ, CA, nct, nchunk;
    long long chunk;
    gram_geometry(N, ncx, nz, &KZ, &CA, &nct, &nchunk, &chunk);
    // algorithmic bytes: every distinct column read once
    const int ncols = (Z1 == X && ldz1 == ldx) ? std::max(ncx, nz1) + nz2 : ncx + nz;
    c.begin(cls, (double)N * sizeof(T) * ncols);  // one record: partial + reduce
    if (Z1 == X && ldz1 == ldx && nz2 == 0 && ncx == nz1 && ncx <= 9) {
        // a block against itself: one pass over its columns (same chunking,
        // so the partials fit the space sized by gram_partial_doubles)
        const dim3 g((unsigned)nchunk), b(kThreads);
        if (ncx <= 3)
            hipLaunchKernelGGL((k_gram_self<T, 3>), g, b, 0, c.st, X, ldx, ncx, N, chunk, KZ, part, skip);
        else if (ncx <= 5)
            hipLaunchKernelGGL((k_gram_self<T, 5>), g, b, 0, c.st, X, ldx, ncx, N, chunk, KZ, part, skip);
        else
            hipLaunchKernelGGL((k_gram_self<T, 9>), g, b, 0, c.st, X, ldx, ncx, N, chunk, KZ, part, skip);
        SSTEP_HIP(hipGetLastError());
        if (reduce)
            hipLaunchKernelGGL(k_gram_reduce, dim3((ncx * nz + 63) / 64), dim3(kThreads), 0, c.st,
                               part, nchunk, ncx, KZ, nz, G, skip);
        SSTEP_HIP(hipGetLastError());
        c.end();
        return;
    }
    if (!Z2) Z2 = Z1;
#define SSTEP_GRAM_CASE(K)                                                                      \
    case K:                                                                                     \
        gram_go<T, gram_ca_c(K), K>(c, X, ldx, ncx, Z1, ldz1, nz1, Z2, ldz2, nz2, N, chunk, nct, \
                                    nchunk, part, skip);                                        \
        break;
    switch (KZ) {
        SSTEP_GRAM_CASE(1)
        SSTEP_GRAM_CASE(2)
        SSTEP_GRAM_CASE(4)
        SSTEP_GRAM_CASE(8)
        SSTEP_GRAM_CASE(9)
        SSTEP_GRAM_CASE(12)
        SSTEP_GRAM_CASE(13)
        SSTEP_GRAM_CASE(16)
        SSTEP_GRAM_CASE(17)
        default:
            throw HipFailure{hipErrorInvalidValue, "gram width"};
    }
#undef SSTEP_GRAM_CASE
    SSTEP_HIP(hipGetLastError());
    const int nout = ncx * nz;
    if (reduce)
        hipLaunchKernelGGL(k_gram_reduce, dim3((nout + 63) / 64), dim3(kThreads), 0, c.st, part,
                           nchunk, ncx, KZ, nz, G, skip);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

// points per thread of the update kernel for a type combination
template <typename TV, typename TB, typename TO>
constexpr int update_ppt() {
    constexpr int PA = 16 / sizeof(TV), PB = 16 / sizeof(TB), PO = 16 / sizeof(TO);
    return PA > PB ? (PA > PO ? PA : PO) : (PB > PO ? PB : PO);
}
template <typename TV, typename TB, typename TO>
inline long long update_blocks_t(long long N) {
    const long long per = (long long)kThreads * update_ppt<TV, TB, TO>();
    return (N + per - 1) / per;
}
// upper bound over all type combinations (sizing of norm partials)
inline long long update_blocks(long long N) { return (N + 2 * kThreads - 1) / (2 * kThreads); }

// out[:, l] = base[:, l] + sum_c V[:, c] M[c*nout + l], nout = 1..16
template <typename TV, typename TB, typename TO, typename TA, bool NORM>
inline void launch_update(Ctx& c, long long N, const TB* base, long long ldb, const TV* V,
                          long long ldv, int n2, const int* n2_dev, const double* M, TO* out,
                          long long ldo, int nout, double* part, const int* skip, double bytes,
                          int cls = SSTEP_K_UPDATE) {
    c.begin(cls, bytes);
    // 4-wave workgroups: with non-temporal output stores they stream 0.5-1.5%
    // faster than 2-wave ones at every width from 40 to 312 columns (8 outputs
    // of 2^24 doubles).  FP64 updates of 4 or more outputs against 128 or more
    // stored columns on large grids take 16-wave workgroups: 2.3-2.7% faster at
    // 160 and 312 columns, even at 80 and 7% slower at 40; on small grids (2^16
    // points: 32 such workgroups) they are 45% slower.
    constexpr int UT = kThreads, UTW = 1024;
    const bool wide = !NORM && sizeof(TV) == 8 && n2 >= 128 && N >= (1LL << 22);
    const auto grid = [&](int ut) {
        const long long per = (long long)ut * update_ppt<TV, TB, TO>();
        return dim3((unsigned)((N + per - 1) / per));
    };
#define SSTEP_UPD(K)                                                                         \
    case K:                                                                                  \
        if constexpr (K >= 4 && !NORM && sizeof(TV) == 8) {                                  \
            if (wide) {                                                                      \
                hipLaunchKernelGGL((k_update<TV, TB, TO, TA, K, false, UTW>), grid(UTW),     \
                                   dim3(UTW), 0, c.st, N, base, ldb, V, ldv, n2, n2_dev, M,  \
                                   out, ldo, part, skip);                                    \
                break;                                                                       \
            }                                                                                \
        }                                                                                    \
        hipLaunchKernelGGL((k_update<TV, TB, TO, TA, K, NORM && (K == 1), UT>), grid(UT),    \
                           dim3(UT), 0, c.st, N, base, ldb, V, ldv, n2, n2_dev, M, out, ldo, \
                           part, skip);                                                      \
        break;
    switch (nout) {
        SSTEP_UPD(1) SSTEP_UPD(2) SSTEP_UPD(3) SSTEP_UPD(4) SSTEP_UPD(5) SSTEP_UPD(6)
        SSTEP_UPD(7) SSTEP_UPD(8) SSTEP_UPD(9) SSTEP_UPD(10) SSTEP_UPD(11) SSTEP_UPD(12)
        SSTEP_UPD(13) SSTEP_UPD(14) SSTEP_UPD(15) SSTEP_UPD(16)
        default:
            throw HipFailure{hipErrorInvalidValue, "update width"};
    }
#undef SSTEP_UPD
    SSTEP_HIP(hipGetLastError());
    c.end();
}

inline int norm_blocks(long long N) {
    return (int)std::min<long long>(1024, (N + kThreads - 1) / kThreads);
}
inline void launch_norm2(Ctx& c, long long N, const double* v, double* part) {
    c.begin(SSTEP_K_VEC, 8.0 * N);
    hipLaunchKernelGGL(k_norm2, dim3(norm_blocks(N)), dim3(kThreads), 0, c.st, N, v, part);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

}  // namespace sstep
