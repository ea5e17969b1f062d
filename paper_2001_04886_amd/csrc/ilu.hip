// ilu.hip -- ILU(0) right preconditioning (Sec. 5) of a 2-D five-point
// stencil: factorisation, preconditioner solve and product.
//
// For a five-point matrix in the natural ordering the only fill that
// elimination creates lies at columns p -+ (nx - 1) and ILU(0) drops it, so
// the factors keep A's off-diagonal entries and only the pivots change:
//   M = (D + Lo) D^{-1} (D + Up),
//   d_p = a_pp - a_{p,p-nx} a_{p-nx,p} / d_{p-nx} - a_{p,p-1} a_{p-1,p} / d_{p-1},
// Lo / Up the strictly lower (south, west) / upper (east, north) parts of A.
// (L = I + Lo D^{-1} and U = D + Up are the unit-lower / upper ILU(0)
// factors.)
//
// Point (i, j) of a forward sweep depends on (i-1, j) and (i, j-1), so the
// sweeps run over the anti-diagonals i + j (the hyperplane order that makes
// the preconditioner vectorise): a point is reached one step after its west
// and its south neighbour.  The factorisation (once per solve) runs on one
// wave whose lanes own CPL adjacent columns each; the preconditioner solve
// (once per matrix-powers level) spreads the columns over up to 16 waves, one
// column per lane.  Neighbour values move between lanes by whole-wave DPP
// shifts, loads are issued several steps ahead of use (register ring), and
// every load and store is a raw buffer access whose out-of-grid lanes read 0
// / write nothing, so the sweeps have no branches around memory operations
// and no wait for loads still in flight.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/sstep.h"
#include "kernels.hpp"
#include "launch.hpp"
#include "mpk.hpp"

namespace sstep {

namespace {

constexpr int kIluLanes = 64;

// Value of the same register in lane l - 1 (lane 0: 0) / lane l + 1 (lane 63: 0).
__device__ __forceinline__ double from_lane_below(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)b, 0x138, 0xf, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(b >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | lo);
}
__device__ __forceinline__ double from_lane_above(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)b, 0x130, 0xf, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | lo);
}

// Store through the caches (no nontemporal hint): the sweeps read back what
// they wrote, and a store's completion gates the wait for every later load.
__device__ __forceinline__ void ilu_st(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
}

// Buffer resource over coefficient plane q of a variable-coefficient stencil
// (or an empty one: every access out of range).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t coef_rsrc(const StencilView& A, int q) {
    return A.coef ? mpk_rsrc(A.coef + (long long)q * A.N, (unsigned)(A.N * 8))
                  : mpk_rsrc(A.coef, 0u);
}

// Byte offset of (i, j) or kMpkOff when ok is false.
__device__ __forceinline__ unsigned ofs(bool ok, int i, int j, int nx) {
    return ok ? (unsigned)((j * nx + i) * 8) : kMpkOff;
}

// Number of lanes that own at least one column.
__host__ __device__ __forceinline__ int ilu_lanes(int nx, int cpl) { return (nx + cpl - 1) / cpl; }

// ---------------------------------------------------------------------------
// Pivots: d[p] and dinv[p] = 1 / d[p]; *bad = 1 if a pivot is zero or not
// finite, else 0 (always written).
// ---------------------------------------------------------------------------
template <int CPL, int D, bool VC>
__global__ __launch_bounds__(kIluLanes) void k_ilu0_factor(StencilView A, double* __restrict__ d,
                                                           double* __restrict__ dinv,
                                                           int* __restrict__ bad) {
    const int nx = A.nx, ny = A.ny, lane = threadIdx.x, i0 = lane * CPL;
    const int nl = ilu_lanes(nx, CPL), T = ny + nl - 1;
    const __amdgpu_buffer_rsrc_t rc0 = coef_rsrc(A, 0), rw = coef_rsrc(A, 1), re = coef_rsrc(A, 2),
                                 rs = coef_rsrc(A, 3), rn = coef_rsrc(A, 4);
    const __amdgpu_buffer_rsrc_t rd = mpk_rsrc(d, (unsigned)(A.N * 8)),
                                 ri = mpk_rsrc(dinv, (unsigned)(A.N * 8));
    // per point of a step: centre, (west coef) x (east coef of the west
    // point), (south coef) x (north coef of the south point)
    double cc[D][CPL], kw[D][CPL], ks[D][CPL];
    auto fetch = [&](int t, double (&c0)[CPL], double (&w)[CPL], double (&s)[CPL]) {
        const int j = t - lane;
        const bool row = j >= 0 && j < ny;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int i = i0 + c;
            const bool in = row && i < nx;
            if constexpr (VC) {
                c0[c] = mpk_ld<double>(rc0, ofs(in, i, j, nx));
                w[c] = mpk_ld<double>(rw, ofs(in && i > 0, i, j, nx)) *
                       mpk_ld<double>(re, ofs(in && i > 0, i - 1, j, nx));
                s[c] = mpk_ld<double>(rs, ofs(in && j > 0, i, j, nx)) *
                       mpk_ld<double>(rn, ofs(in && j > 0, i, j - 1, nx));
            } else {
                c0[c] = in ? A.c[0] : 1.0;
                w[c] = (in && i > 0) ? A.c[1] * A.c[2] : 0.0;
                s[c] = (in && j > 0) ? A.c[3] * A.c[4] : 0.0;
            }
        }
    };
    // the loop starts D steps early on zeros (rows < 0: nothing stored), so
    // no load is in flight when it is entered and every entry to its head
    // sees the same loads outstanding
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
        for (int c = 0; c < CPL; ++c) cc[u][c] = kw[u][c] = ks[u][c] = 0.0;
    double south[CPL];  // 1 / d of the point below each owned column
#pragma unroll
    for (int c = 0; c < CPL; ++c) south[c] = 0.0;
    double last = 0.0;  // 1 / d of this lane's last column, previous step
    bool fail = false;
    for (int t0 = -D; t0 < T; t0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int t = t0 + u;
            const int j = t - lane;
            const bool row = j >= 0 && j < ny;
            double west = from_lane_below(last);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int i = i0 + c;
                const bool in = row && i < nx;
                const double piv = cc[u][c] - ks[u][c] * south[c] - kw[u][c] * west;
                const double r = 1.0 / piv;
                fail |= in && !(std::isfinite(piv) && piv != 0.0 && std::isfinite(r));
                const double rv = in ? r : 0.0;
                ilu_st(piv, rd, ofs(in, i, j, nx));
                ilu_st(rv, ri, ofs(in, i, j, nx));
                south[c] = rv;
                west = rv;
            }
            last = west;
            fetch(t + D, cc[u], kw[u], ks[u]);
        }
    }
    const bool any = __any(fail);
    if (lane == 0) *bad = any ? 1 : 0;
}

// ---------------------------------------------------------------------------
// z = M^{-1} r.  Forward: (D + Lo) w = r; backward: (D + Up) z = D w, i.e.
// z_p = w_p - (a_e z_{p+1} + a_n z_{p+nx}) / d_p.  One workgroup of
// ceil(nx / 64) waves, one column per lane: wave w owns columns
// [64 w, 64 w + 64).  Inside a wave the west (east) value comes from the
// neighbour lane by a DPP shift; between waves lane 63 (lane 0) leaves it in
// an LDS ring that the next wave reads two steps before it needs it.  Wave w
// runs kIluLag steps behind wave w - 1 (64 for the wavefront, kIluK + 1 more
// so that a barrier, taken every kIluK steps, always separates the ring
// write from that read), and loads run kIluK steps ahead of use.
//
// Sweep layout: the lanes of a wave sit on an anti-diagonal, 64 different
// rows, so natural-order arrays cost a cache line per lane and access.
// 1/d, the coefficients and the intermediate w are therefore kept with point
// (i, j) at ((w * (ny + 63) + j + l) * 64 + l), i = 64 w + l: at every step
// of either sweep the 64 lanes of a wave read one contiguous 512-byte row of
// it.  r is copied into this layout and z out of it by two grid-wide kernels
// around the sweeps (the backward sweep overwrites w with z in place).
// Slots that are no grid point hold 0, and points outside the grid compute
// 0, so the coefficients need no boundary masks: every neighbour value a
// boundary coefficient meets is 0.
// ---------------------------------------------------------------------------
constexpr int kIluK = 8;              // steps between barriers = prefetch depth
constexpr int kIluRing = 32;          // exchange slots per wave (>= 2 kIluK + 2)
constexpr int kIluLag = 64 + kIluK + 1;  // steps between neighbouring waves
constexpr int kIluMaxWaves = 16;

__host__ __device__ __forceinline__ int sweep_rows(int ny) { return ny + 63; }

// 1/d and (VC) the west, south, east, north coefficients into the sweep
// layout: sk[k * P + slot], P = ilu0_sweep_points, k = 0..4.
template <bool VC>
__global__ __launch_bounds__(kThreads) void k_ilu0_skew(StencilView A, long long P,
                                                        const double* __restrict__ dinv,
                                                        double* __restrict__ sk) {
    const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (s >= P) return;
    const int l = (int)(s & 63);
    const long long q = s >> 6;
    const int TS = sweep_rows(A.ny);
    const int tr = (int)(q % TS), w = (int)(q / TS);
    const int j = tr - l, i = 64 * w + l;
    const bool ok = j >= 0 && j < A.ny && i < A.nx;
    const long long p = ok ? (long long)j * A.nx + i : 0;
    sk[s] = ok ? dinv[p] : 0.0;
    if constexpr (VC) {
#pragma unroll
        for (int k = 1; k <= 4; ++k) sk[k * P + s] = ok ? A.coef[k * A.N + p] : 0.0;
    }
}

// x (natural order) into the sweep layout, 0 where a slot is no grid point.
__global__ __launch_bounds__(kThreads) void k_ilu0_to_sweep(StencilView A, long long P,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ xs,
                                                            const int* __restrict__ skip) {
    if (skip && *skip) return;
    const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (s >= P) return;
    const int l = (int)(s & 63);
    const long long q = s >> 6;
    const int TS = sweep_rows(A.ny);
    const int j = (int)(q % TS) - l, i = 64 * (int)(q / TS) + l;
    xs[s] = (j >= 0 && j < A.ny && i < A.nx) ? x[(long long)j * A.nx + i] : 0.0;
}

// The sweep layout back to natural order, one thread per grid point.
__global__ __launch_bounds__(kThreads) void k_ilu0_from_sweep(StencilView A,
                                                              const double* __restrict__ xs,
                                                              double* __restrict__ x,
                                                              const int* __restrict__ skip) {
    if (skip && *skip) return;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= A.N) return;
    const int i = (int)(p % A.nx), j = (int)(p / A.nx), l = i & 63;
    x[p] = xs[((long long)(i >> 6) * sweep_rows(A.ny) + j + l) * 64 + l];
}

template <bool VC>
__global__ __launch_bounds__(64 * kIluMaxWaves) void k_ilu0_solve(
    StencilView A, long long P, const double* __restrict__ sk, const double* __restrict__ rsk,
    double* __restrict__ wsk, const int* __restrict__ skip) {
    if (skip && *skip) return;
    // ring row kIluMaxWaves stays 0 (the west of wave 0 / east of the last
    // wave); lanes that publish nothing write their own dummy slot instead
    __shared__ double xch[kIluMaxWaves + 1][kIluRing];
    __shared__ double dummy[kIluMaxWaves * 64];
    const int ny = A.ny, nw = blockDim.x >> 6, TS = sweep_rows(ny);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int T = ny + 63 + (nw - 1) * kIluLag;
    const unsigned pb = (unsigned)(P * 8);
    const __amdgpu_buffer_rsrc_t rr = mpk_rsrc(rsk, pb);
    const __amdgpu_buffer_rsrc_t rd = mpk_rsrc(sk, pb), rws = mpk_rsrc(wsk, pb);
    // coefficient planes in stencil order: 1 west, 2 east, 3 south, 4 north
    const __amdgpu_buffer_rsrc_t rcw = mpk_rsrc(sk + (VC ? P : 0), VC ? pb : 0u),
                                 rce = mpk_rsrc(sk + (VC ? 2 * P : 0), VC ? pb : 0u),
                                 rcs = mpk_rsrc(sk + (VC ? 3 * P : 0), VC ? pb : 0u),
                                 rcn = mpk_rsrc(sk + (VC ? 4 * P : 0), VC ? pb : 0u);
    // sweep-layout offset of sweep row tr of this wave
    const unsigned sbase = (unsigned)((w * TS * 64 + l) * 8);
    auto sat = [&](int tr) {
        return (unsigned)tr < (unsigned)TS ? sbase + (unsigned)tr * 512u : kMpkOff;
    };
    auto clear_ring = [&]() {
        for (int k = threadIdx.x; k < (kIluMaxWaves + 1) * kIluRing; k += blockDim.x)
            (&xch[0][0])[k] = 0.0;
        __syncthreads();
    };

    double v[kIluK], dv[kIluK], a1[kIluK], a2[kIluK];
    auto fetch_f = [&](int j, int u) {
        const unsigned o = sat(j + l);
        v[u] = mpk_ld<double>(rr, o);
        dv[u] = mpk_ld<double>(rd, o);
        if constexpr (VC) {
            a1[u] = mpk_ld<double>(rcw, o);
            a2[u] = mpk_ld<double>(rcs, o);
        } else {
            a1[u] = A.c[1];  // times a neighbour value that is 0 off the grid
            a2[u] = A.c[3];
        }
    };
    auto fetch_b = [&](int j, int u) {
        const unsigned o = sat(j + l);
        v[u] = mpk_ld<double>(rws, o);
        dv[u] = mpk_ld<double>(rd, o);
        if constexpr (VC) {
            a1[u] = mpk_ld<double>(rce, o);
            a2[u] = mpk_ld<double>(rcn, o);
        } else {
            a1[u] = A.c[2];
            a2[u] = A.c[4];
        }
    };
    // both sweeps start kIluK steps early on zeros: no load is in flight when
    // a loop is entered, and every entry to its head sees the same loads
    auto zero_ring = [&]() {
#pragma unroll
        for (int u = 0; u < kIluK; ++u) v[u] = dv[u] = a1[u] = a2[u] = 0.0;
    };

    // forward sweep: wave w, lane l at step t is on row j = t - l - w kIluLag,
    // sweep row j + l = t - w kIluLag
    clear_ring();
    zero_ring();
    {
        const int off = l + w * kIluLag;
        double* const pub = l == 63 ? &xch[w][0] : &dummy[threadIdx.x];
        const int pmask = l == 63 ? kIluRing - 1 : 0;
        const double* const sub = &xch[w > 0 ? w - 1 : kIluMaxWaves][0];
        double below = 0.0, edge = 0.0, xp = 0.0, xq = 0.0;
        for (int t0 = -kIluK; t0 < T; t0 += kIluK) {
#pragma unroll
            for (int u = 0; u < kIluK; ++u) {
                const int t = t0 + u, j = t - off;
                const double dn = from_lane_below(edge);
                const double west = l == 0 ? xp : dn;
                const double val = (v[u] - a2[u] * below - a1[u] * west) * dv[u];
                ilu_st(val, rws, sat(j + l));
                below = val;
                edge = val;
                pub[j & pmask] = val;
                fetch_f(j + kIluK, u);
                // lane 0: the previous wave's value for the row two steps on
                xp = xq;
                xq = sub[(t + 2 - w * kIluLag) & (kIluRing - 1)];
            }
            __syncthreads();
        }
    }
    // the backward sweep reads the forward result of the lane's own points;
    // the wait also drains the forward sweep's last (out-of-range) loads
    __threadfence_block();
    clear_ring();
    zero_ring();
    // backward sweep, mirrored: wave w, lane l at step t is on row
    // j = ny - 1 - (t - (63 - l) - (nw - 1 - w) kIluLag)
    {
        const int wm = nw - 1 - w, off = (63 - l) + wm * kIluLag;
        double* const pub = l == 0 ? &xch[w][0] : &dummy[threadIdx.x];
        const int pmask = l == 0 ? kIluRing - 1 : 0;
        const double* const sub = &xch[w < nw - 1 ? w + 1 : kIluMaxWaves][0];
        double above = 0.0, edge = 0.0, xp = 0.0, xq = 0.0;
        for (int t0 = -kIluK; t0 < T; t0 += kIluK) {
#pragma unroll
            for (int u = 0; u < kIluK; ++u) {
                const int t = t0 + u, j = ny - 1 - (t - off);
                const double up = from_lane_above(edge);
                const double east = l == 63 ? xp : up;
                const double val = v[u] - dv[u] * (a1[u] * east + a2[u] * above);
                ilu_st(val, rws, sat(j + l));
                above = val;
                edge = val;
                pub[j & pmask] = val;
                fetch_b(j - kIluK, u);
                // lane 63: the next wave's value for the row two steps on
                xp = xq;
                xq = sub[(ny - 1 - (t + 2 - wm * kIluLag)) & (kIluRing - 1)];
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// u = M x = (D + Lo) D^{-1} (D + Up) x, one thread per point:
//   y_q = d_q x_q + a_e(q) x_{q+1} + a_n(q) x_{q+nx}     (q = p, p-1, p-nx)
//   u_p = y_p + a_w(p) y_{p-1} / d_{p-1} + a_s(p) y_{p-nx} / d_{p-nx}
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_ilu0_mul(StencilView A, const double* __restrict__ d,
                                                       const double* __restrict__ dinv,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ u) {
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= A.N) return;
    const int nx = A.nx, ny = A.ny;
    const int i = (int)(p % nx), j = (int)(p / nx);
    auto cf = [&](int q, long long pt) { return A.coef ? A.coef[q * A.N + pt] : A.c[q]; };
    auto y = [&](long long q, int iq, int jq) {
        double v = d[q] * x[q];
        if (iq < nx - 1) v += cf(2, q) * x[q + 1];
        if (jq < ny - 1) v += cf(4, q) * x[q + nx];
        return v;
    };
    double r = y(p, i, j);
    if (j > 0) r += cf(3, p) * dinv[p - nx] * y(p - nx, i, j - 1);
    if (i > 0) r += cf(1, p) * dinv[p - 1] * y(p - 1, i - 1, j);
    u[p] = r;
}

// ---------------------------------------------------------------------------
// One level of matrix powers of the right-preconditioned operator:
//   out = alpha * si * A(t) + beta * si * in + gam * sp * prev,  t = M^{-1} in
// (si, sp: optional device scales of in / prev, nullptr = 1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_ilu0_level(
    StencilView A, const double* __restrict__ in, const double* __restrict__ in_scale,
    const double* __restrict__ prev, const double* __restrict__ prev_scale, double alpha,
    double beta, double gam, const double* __restrict__ t, double* __restrict__ out,
    const int* __restrict__ skip) {
    if (skip && *skip) return;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= A.N) return;
    const int nx = A.nx, ny = A.ny;
    const int i = (int)(p % nx), j = (int)(p / nx);
    auto cf = [&](int q) { return A.coef ? A.coef[q * A.N + p] : A.c[q]; };
    double acc = 0.0;
    if (i > 0) acc += cf(1) * t[p - 1];
    if (i < nx - 1) acc += cf(2) * t[p + 1];
    if (j > 0) acc += cf(3) * t[p - nx];
    if (j < ny - 1) acc += cf(4) * t[p + nx];
    acc += cf(0) * t[p];
    const double si = in_scale ? *in_scale : 1.0;
    double r = alpha * si * acc;
    if (beta != 0.0) r += beta * si * in[p];
    if (gam != 0.0) r += gam * (prev_scale ? *prev_scale : 1.0) * prev[p];
    out[p] = r;
}

// columns per lane for a row of nx points (nx <= 64 * 16)
int ilu_cpl(int nx) {
    if (nx <= 64) return 1;
    if (nx <= 128) return 2;
    if (nx <= 256) return 4;
    if (nx <= 512) return 8;
    return 16;
}

}  // namespace

bool ilu0_supported(const sstep_stencil& A) {
    // byte offsets of the natural and of the sweep layout fit 31 bits
    return A.ndim == 2 && A.nx >= 1 && A.ny >= 1 && A.nx <= kIluMaxNx &&
           (long long)A.nx * A.ny * 8 < (1LL << 31) &&
           (long long)((A.nx + 63) / 64) * 64 * (A.ny + 63) * 8 < (1LL << 31);
}

// Factorisation prefetch depth D (steps) per columns-per-lane and coefficient
// kind: the memory operations of D steps (about 7 per point with coefficient
// fields, 2 without) must fit the 63 the wait counter tracks.
#define SSTEP_ILU_CASES(X) X(1, 8, 8) X(2, 4, 8) X(4, 2, 4) X(8, 1, 2) X(16, 1, 1)

void ilu0_factor_launch(Ctx& c, const StencilView& v, double* d, double* dinv, int* bad) {
    c.begin(SSTEP_K_MPK, (double)v.N * 8.0 * (v.coef ? 7.0 : 2.0));
    switch (ilu_cpl(v.nx)) {
#define SSTEP_F(C, DV, DC)                                                                        \
    case C:                                                                                       \
        if (v.coef)                                                                               \
            hipLaunchKernelGGL((k_ilu0_factor<C, DV, true>), dim3(1), dim3(kIluLanes), 0, c.st, v, \
                               d, dinv, bad);                                                     \
        else                                                                                      \
            hipLaunchKernelGGL((k_ilu0_factor<C, DC, false>), dim3(1), dim3(kIluLanes), 0, c.st,  \
                               v, d, dinv, bad);                                                  \
        break;
        SSTEP_ILU_CASES(SSTEP_F)
#undef SSTEP_F
    }
    SSTEP_HIP(hipGetLastError());
    c.end();
}

long long ilu0_sweep_points(const StencilView& v) {
    return (long long)((v.nx + 63) / 64) * sweep_rows(v.ny) * 64;
}

void ilu0_skew_launch(Ctx& c, const StencilView& v, const double* dinv, double* sk) {
    const long long P = ilu0_sweep_points(v);
    c.begin(SSTEP_K_MPK, (double)P * 8.0 * (v.coef ? 10.0 : 2.0));
    const dim3 grid((unsigned)((P + kThreads - 1) / kThreads));
    if (v.coef)
        hipLaunchKernelGGL(k_ilu0_skew<true>, grid, dim3(kThreads), 0, c.st, v, P, dinv, sk);
    else
        hipLaunchKernelGGL(k_ilu0_skew<false>, grid, dim3(kThreads), 0, c.st, v, P, dinv, sk);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

void ilu0_solve_launch(Ctx& c, const StencilView& v, const double* sk, double* wsk,
                       double* rsk, const double* r, double* z, const int* skip) {
    // algorithmic bytes: r, 1/d (twice), the four neighbour coefficients, the
    // intermediate written and read, z written
    c.begin(SSTEP_K_MPK, (double)v.N * 8.0 * (v.coef ? 10.0 : 6.0));
    const long long P = ilu0_sweep_points(v);
    hipLaunchKernelGGL(k_ilu0_to_sweep, dim3((unsigned)((P + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, c.st, v, P, r, rsk, skip);
    const dim3 block(64 * ((v.nx + 63) / 64));
    if (v.coef)
        hipLaunchKernelGGL(k_ilu0_solve<true>, dim3(1), block, 0, c.st, v, P, sk, rsk, wsk, skip);
    else
        hipLaunchKernelGGL(k_ilu0_solve<false>, dim3(1), block, 0, c.st, v, P, sk, rsk, wsk, skip);
    hipLaunchKernelGGL(k_ilu0_from_sweep, dim3((unsigned)((v.N + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, c.st, v, wsk, z, skip);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

void ilu0_mul_launch(Ctx& c, const StencilView& v, const double* d, const double* dinv,
                     const double* x, double* u) {
    c.begin(SSTEP_K_MPK, (double)v.N * 8.0 * (v.coef ? 7.0 : 4.0));
    hipLaunchKernelGGL(k_ilu0_mul, dim3((unsigned)((v.N + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, c.st, v, d, dinv, x, u);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

void ilu0_level_launch(Ctx& c, const StencilView& v, const double* in, const double* in_scale,
                       const double* prev, const double* prev_scale, double alpha, double beta,
                       double gam, const double* t, double* out, const int* skip, double bytes) {
    c.begin(SSTEP_K_MPK, bytes);
    hipLaunchKernelGGL(k_ilu0_level, dim3((unsigned)((v.N + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, c.st, v, in, in_scale, prev, prev_scale, alpha, beta,
                       gam, t, out, skip);
    SSTEP_HIP(hipGetLastError());
    c.end();
}

}  // namespace sstep
