// batched.hip -- many independent s-step GMRES(m) solves (Sec. 4, Alg. 4.2)
// in one persistent launch.
//
// The grid holds exactly as many workgroups as can be resident at once.
// Systems are split by size into two queues, each ordered largest first:
//   * phase 1 (teams): workgroups are grouped in teams of T (members share an
//     XCD).  A team takes the next large system and solves it cooperatively:
//     each member owns a contiguous range of grid rows of every vector; the
//     partial sums of every reduction are published per member and summed in
//     rank order after a team barrier, so each member holds bit-identical
//     totals and repeats the small FP64 work itself; matrix-powers levels and
//     the assembly are separated by team barriers because the stencil reads
//     rows of neighbouring members;
//   * phase 2: every workgroup takes the next small system alone.
// Team barriers are counters advanced with atomics, with a bounded spin: on a
// time-out the launch is aborted and the affected systems report
// SSTEP_ERR_HIP.  Where the hardware reports one XCD for every member of a
// team (the usual case) the members share an L2 and a barrier costs only the
// wait for their stores and an L1 invalidation; otherwise it takes agent-scope
// release/acquire (the L2 written back and invalidated).  The grid size is
// checked against the occupancy of the kernel, so every member of a team is
// resident.
//
// Per block the arithmetic is the same as in gmres.hip (normalised start
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

constexpr int kMaxTeam = 8;
constexpr int kPartLen = 512 * 8 + 64;  // largest reduction: c0 * s (Gram) + scalars

struct BatchSys {
    StencilView A;
    const double* f;
    double* x;
    double* ws;        // this system's basis region: (m*s+1) columns of ld doubles
    long long ld;
    double sigma;
    int status, blocks, cycles, team;
    double rel_resid;
    long long ticks[SSTEP_K_NCLASS];  // wall-clock ticks of the (lead) workgroup per class
};

// per-workgroup scratch for the small dense state (sized for m*s <= 512)
struct BatchSlot {
    double G[513 * 512];   // Hessenberg, column-major, ld = K+1
    double R[513 * 512];   // rotated L G
    double cs[513], sn[513], rhs[513], y[513];
    double T[512 * 17];    // projection coefficients [row][s+1]
    double C[512 * 16];    // Gram (team total)
    double part[2][kPartLen];  // this workgroup's partial sums, double-buffered
    GramFactor Wf[128];
    double nu[129], inv_nu[129];
};

struct BatchArgs {
    BatchSys* sys;
    const int* order_big;    // solved by teams, largest first
    const int* order_small;  // solved by one workgroup each, largest first
    int nbig, nsmall;
    int s, m;
    double tol;
    int max_blocks;
    double rank_tol, lucky_tol;
    BatchSlot* slots;
    int* queue;              // [0] big-system queue, [1] small-system queue, [2] abort flag
    unsigned* team_sync;     // per team 64 words: [0] barrier counter, [32] mailbox,
                             // [40 + rank] XCD of each member plus one
    int team;                // workgroups per team (1: no phase 1)
    long long spin_limit;
};

// A workgroup's team (kept in LDS).  T == 1: the workgroup alone.
struct Team {
    int T, rank, parity, failed;
    int local;  // every member runs on the same XCD (one L2)
    unsigned target;
    unsigned* cnt;
    int* mailbox;
    int* abort;
    long long limit;
    BatchSlot* member[kMaxTeam];
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

// XCD (accelerator complex) the calling workgroup runs on.
__device__ __forceinline__ unsigned xcd_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 0xfu;
}

// Thread 0 arrives at the team's counter and waits for every member (bounded).
__device__ __forceinline__ void team_arrive_wait(Team& tm, int order) {
    tm.target += tm.T;
    if (order == __ATOMIC_RELEASE)
        __hip_atomic_fetch_add(tm.cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_fetch_add(tm.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long long spins = 0;
    while (__hip_atomic_load(tm.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tm.target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > tm.limit ||
            __hip_atomic_load(tm.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            tm.failed = 1;
            __hip_atomic_store(tm.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
    }
}

// Team barrier: every member's global writes before it are visible to every
// member after it.  Returns false (and marks the team failed) on a time-out or
// an abort raised elsewhere; later barriers then return at once.
//   * members on one XCD share its L2, and the per-CU vector L1 is write-
//     through: each wave waits until its stores are acknowledged (by the L2),
//     and after the arrival of every member the CU's L1 is invalidated so
//     later loads see the other members' lines;
//   * otherwise agent-scope release / acquire (the L2 is written back and
//     invalidated as well, since the XCDs' L2s are not coherent).
__device__ bool team_barrier(Team& tm) {
    if (tm.T == 1) {
        __syncthreads();
        return true;
    }
    if (tm.local) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0 && !tm.failed) {
            team_arrive_wait(tm, __ATOMIC_RELAXED);
            asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
        }
        __syncthreads();
        return !tm.failed;
    }
    // every wave publishes its own stores (agent-scope release: wait for them
    // and write the XCD's L2 back); __syncthreads alone does not wait for them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0 && !tm.failed) {
        team_arrive_wait(tm, __ATOMIC_RELEASE);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return !tm.failed;
}

// out[0..n) = sum over members (rank order) of their part[parity][0..n); each
// member first wrote its own partials there.  T == 1: out = own partials.
template <int NT>
__device__ void team_combine(Team& tm, BatchSlot& W, int n, double* out) {
    const int buf = tm.parity;
    if (tm.T == 1) {
        if (out != W.part[buf])
            for (int i = threadIdx.x; i < n; i += NT) out[i] = W.part[buf][i];
        __syncthreads();
        return;
    }
    team_barrier(tm);
    for (int i = threadIdx.x; i < n; i += NT) {
        double t = 0.0;
        for (int r = 0; r < tm.T; ++r) t += tm.member[r]->part[buf][i];
        out[i] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) tm.parity ^= 1;
    __syncthreads();
}

// a scalar reduction over the team: v is this workgroup's total
template <int NT>
__device__ double team_scalar(Team& tm, BatchSlot& W, double v, double* lds1) {
    if (tm.T == 1) return v;
    if (threadIdx.x == 0) W.part[tm.parity][0] = v;
    team_combine<NT>(tm, W, 1, lds1);
    return lds1[0];
}

// Phase timer of the (lead) workgroup: thread 0 reads the constant-rate wall
// clock after the barrier that closes a phase and charges the interval to one
// kernel class.  Accumulators in LDS (slot SSTEP_K_NCLASS: last reading).
struct PhaseClock {
    long long* acc;
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
// streamed once (stored basis columns): non-temporal, so they do not push the
// lines that are reused (Z tiles, stencil neighbours) out of the caches
__device__ __forceinline__ d2v ld2nt(const double* p) {
    return __builtin_nontemporal_load((const SSTEP_GLOBAL d2v*)p);
}
__device__ __forceinline__ void st2(double* p, d2v v) { *(SSTEP_GLOBAL d2v*)p = v; }
__device__ __forceinline__ void st2nt(double* p, d2v v) {
    __builtin_nontemporal_store(v, (SSTEP_GLOBAL d2v*)p);
}
__device__ __forceinline__ double ldg(const double* p) { return *(const SSTEP_GLOBAL double*)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(SSTEP_GLOBAL double*)p = v; }
__device__ __forceinline__ double lds(const double* p) { return *(const SSTEP_LDS double*)p; }

// Point range [P0, P1) of a workgroup: pairs [pa, pb) with even ends (16-byte
// loads) and at most two single points (e0 at the front, e1 at the back).
struct Range {
    long long P0, P1, pa, pb, e0, e1;
    __device__ Range(long long p0, long long p1) : P0(p0), P1(p1) {
        pa = (p0 + 1) & ~1LL;
        pb = p1 & ~1LL;
        if (pb < pa) pb = pa;
        e0 = (p0 < pa && p0 < p1) ? p0 : -1;
        e1 = (pb < p1 && pb >= pa) ? pb : -1;
    }
};

// Grid coordinates of the points a thread visits (p = p0, p0 + step, ...),
// advanced without divisions.
struct Walker {
    int i, j, l, di, dj, dl, nx, ny;
    __device__ Walker(int nx_, int ny_, long long p0, int step) {
        nx = nx_;
        ny = ny_;
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

// Bits 1..6 of a grid point: its -x, +x, -y, +y, -z, +z neighbour lies inside.
__device__ __forceinline__ unsigned grid_bits(int i, int j, int l, int nx, int ny, int nz) {
    return (unsigned)(i > 0) << 1 | (unsigned)(i < nx - 1) << 2 | (unsigned)(j > 0) << 3 |
           (unsigned)(j < ny - 1) << 4 | (unsigned)(l > 0) << 5 | (unsigned)(l < nz - 1) << 6;
}

// One stencil row of a point from its seven values (order -x, +x, -y, +y, -z,
// +z, centre; neighbours outside the grid weighted 0).
__device__ __forceinline__ double stencil_point(unsigned b, const double (&c)[7], double vxm,
                                                double vxp, double vym, double vyp, double vzm,
                                                double vzp, double vc) {
    double acc = 0.0;
    acc = fma((b >> 1 & 1u) ? c[1] : 0.0, vxm, acc);
    acc = fma((b >> 2 & 1u) ? c[2] : 0.0, vxp, acc);
    acc = fma((b >> 3 & 1u) ? c[3] : 0.0, vym, acc);
    acc = fma((b >> 4 & 1u) ? c[4] : 0.0, vyp, acc);
    acc = fma((b >> 5 & 1u) ? c[5] : 0.0, vzm, acc);
    acc = fma((b >> 6 & 1u) ? c[6] : 0.0, vzp, acc);
    return fma(c[0], vc, acc);
}

// Constant coefficients: the same pass over point pairs [R.pa, R.pb) (16-byte
// centre loads and stores, SP pairs per thread and step, 2 NT points apart),
// then the (at most two) single points at the ends of the range.  Each point's
// arithmetic is the one of the general pass below.
template <int NT, bool D3>
__device__ __forceinline__ double wg_stencil_pairs(const StencilView& Ad, const double (&c)[7],
                                                   const double* in, double* out, double sc,
                                                   const double* f, const Range& R) {
    constexpr int SP = 4;
    const int nx = Ad.nx, ny = Ad.ny, nz = Ad.nz;
    const long long sy = nx, sz = (long long)nx * ny;
    const SSTEP_GLOBAL double* gin = (const SSTEP_GLOBAL double*)in;
    const SSTEP_GLOBAL double* gf = (const SSTEP_GLOBAL double*)f;
    double sq = 0.0;
    Walker w(nx, ny, R.pa + 2 * (long long)threadIdx.x, 2 * NT);
    for (long long q0 = R.pa + 2 * (long long)threadIdx.x; q0 < R.pb; q0 += 2LL * SP * NT) {
        long long pp[SP];
        unsigned m0[SP], m1[SP];  // grid bits of the pair's two points
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            const long long p = q0 + 2LL * u * NT;
            const bool ok = p < R.pb;
            pp[u] = ok ? p : q0;
            unsigned a = 0, b = 0;
            if (ok) {
                int i1 = w.i + 1, j1 = w.j, l1 = w.l;
                if (i1 == nx) {
                    i1 = 0;
                    if (++j1 == ny) {
                        j1 = 0;
                        ++l1;
                    }
                }
                a = grid_bits(w.i, w.j, w.l, nx, ny, nz);
                b = grid_bits(i1, j1, l1, nx, ny, nz);
            }
            m0[u] = a;
            m1[u] = b;
            w.next();
        }
        // every load of the SP pairs before any arithmetic; a neighbour outside
        // the grid is read at its own point (valid) and weighted 0
        d2v ctr[SP], fp[SP];
        double xm[SP], xp[SP], y0m[SP], y0p[SP], y1m[SP], y1p[SP];
        double z0m[D3 ? SP : 1], z0p[D3 ? SP : 1], z1m[D3 ? SP : 1], z1p[D3 ? SP : 1];
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            const long long p = pp[u];
            const unsigned a = m0[u], b = m1[u];
            ctr[u] = ld2(in + p);
            xm[u] = gin[(a >> 1 & 1u) ? p - 1 : p];
            xp[u] = gin[(b >> 2 & 1u) ? p + 2 : p + 1];
            y0m[u] = gin[(a >> 3 & 1u) ? p - sy : p];
            y0p[u] = gin[(a >> 4 & 1u) ? p + sy : p];
            y1m[u] = gin[(b >> 3 & 1u) ? p + 1 - sy : p + 1];
            y1p[u] = gin[(b >> 4 & 1u) ? p + 1 + sy : p + 1];
            if constexpr (D3) {
                z0m[u] = gin[(a >> 5 & 1u) ? p - sz : p];
                z0p[u] = gin[(a >> 6 & 1u) ? p + sz : p];
                z1m[u] = gin[(b >> 5 & 1u) ? p + 1 - sz : p + 1];
                z1p[u] = gin[(b >> 6 & 1u) ? p + 1 + sz : p + 1];
            }
            if (f) fp[u] = ld2(f + p);
        }
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            const unsigned a = m0[u], b = m1[u];
            // +x of the first point is the second, -x of the second the first
            double r0 = stencil_point(a, c, xm[u], ctr[u].y, y0m[u], y0p[u], D3 ? z0m[u] : 0.0,
                                      D3 ? z0p[u] : 0.0, ctr[u].x);
            double r1 = stencil_point(b, c, ctr[u].x, xp[u], y1m[u], y1p[u], D3 ? z1m[u] : 0.0,
                                      D3 ? z1p[u] : 0.0, ctr[u].y);
            r0 = f ? fp[u].x - r0 : sc * r0;
            r1 = f ? fp[u].y - r1 : sc * r1;
            if (q0 + 2LL * u * NT < R.pb) {
                st2(out + pp[u], d2v{r0, r1});
                sq += r0 * r0 + r1 * r1;
            }
        }
    }
    const long long pe = threadIdx.x == 0 ? R.e0 : (threadIdx.x == 1 ? R.e1 : -1);
    if (pe >= 0) {
        const long long rest = pe / nx;
        const int i = (int)(pe - rest * nx), j = (int)(rest % ny), l = (int)(rest / ny);
        const unsigned b = grid_bits(i, j, l, nx, ny, nz);
        double r = stencil_point(b, c, gin[(b >> 1 & 1u) ? pe - 1 : pe], gin[(b >> 2 & 1u) ? pe + 1 : pe],
                                 gin[(b >> 3 & 1u) ? pe - sy : pe], gin[(b >> 4 & 1u) ? pe + sy : pe],
                                 D3 ? gin[(b >> 5 & 1u) ? pe - sz : pe] : 0.0,
                                 D3 ? gin[(b >> 6 & 1u) ? pe + sz : pe] : 0.0, gin[pe]);
        r = f ? gf[pe] - r : sc * r;
        stg(out + pe, r);
        sq += r * r;
    }
    return sq;
}

// One stencil pass over points [P0, P1): out = sc * (A in), or with f given
// r = f - A in into out; returns this thread's share of sum(out^2).
// Neighbours are summed in the order -x, +x, -y, +y, -z, +z, then the centre
// (outside the grid = Dirichlet 0).  Constant coefficients take the paired
// pass above; per-point coefficients: a thread takes SU points per step (NT
// apart) and issues the loads of all of them before the arithmetic, so SU
// points' worth of loads are in flight per thread; a neighbour outside the
// grid is read at the point itself (always valid) and enters with weight 0,
// which leaves the sum bit-identical to skipping it.  The operator's scalars
// are copied to registers first (the descriptor sits in LDS).  Out of line:
// inlined, its registers pushed the solve's long-lived state into scratch
// inside the Gram and update loops.
template <int NT>
__device__ __noinline__ double wg_stencil(const StencilView& Ad, const double* in, double* out, double sc,
                             const double* f, long long P0, long long P1) {
    constexpr int SU = 4;
    const int nx = Ad.nx, ny = Ad.ny, nz = Ad.nz;
    const bool d3 = Ad.ndim == 3;
    const long long N = Ad.N, sy = nx, sz = (long long)nx * ny;
    const double* coef = Ad.coef;
    double c[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) c[q] = Ad.c[q];
    if (!coef) {
        const Range R(P0, P1);
        return d3 ? wg_stencil_pairs<NT, true>(Ad, c, in, out, sc, f, R)
                  : wg_stencil_pairs<NT, false>(Ad, c, in, out, sc, f, R);
    }
    const SSTEP_GLOBAL double* gin = (const SSTEP_GLOBAL double*)in;
    SSTEP_GLOBAL double* gout = (SSTEP_GLOBAL double*)out;
    const SSTEP_GLOBAL double* gf = (const SSTEP_GLOBAL double*)f;
    const SSTEP_GLOBAL double* gc = (const SSTEP_GLOBAL double*)coef;
    Walker w(nx, ny, P0 + threadIdx.x, NT);
    double sq = 0.0;
    for (long long pb = P0 + threadIdx.x; pb < P1; pb += (long long)SU * NT) {
        long long pp[SU];
        unsigned in_grid[SU];  // bit q: neighbour q (1 -x, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z) inside
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const long long p = pb + (long long)u * NT;
            const bool ok = p < P1;
            pp[u] = ok ? p : pb;
            unsigned b = 0;
            if (ok) {
                b = (unsigned)(w.i > 0) << 1 | (unsigned)(w.i < nx - 1) << 2 |
                    (unsigned)(w.j > 0) << 3 | (unsigned)(w.j < ny - 1) << 4 |
                    (unsigned)(w.l > 0) << 5 | (unsigned)(w.l < nz - 1) << 6;
            }
            in_grid[u] = b;
            w.next();
        }
        double v[SU][7], cc[SU][7], fv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const long long p = pp[u];
            const unsigned b = in_grid[u];
            v[u][0] = gin[p];
            v[u][1] = gin[(b >> 1 & 1u) ? p - 1 : p];
            v[u][2] = gin[(b >> 2 & 1u) ? p + 1 : p];
            v[u][3] = gin[(b >> 3 & 1u) ? p - sy : p];
            v[u][4] = gin[(b >> 4 & 1u) ? p + sy : p];
            if (d3) {
                v[u][5] = gin[(b >> 5 & 1u) ? p - sz : p];
                v[u][6] = gin[(b >> 6 & 1u) ? p + sz : p];
            } else {
                v[u][5] = v[u][6] = 0.0;
            }
            if (coef) {
#pragma unroll
                for (int q = 0; q < 7; ++q) cc[u][q] = (q < 5 || d3) ? gc[q * N + p] : 0.0;
            } else {
#pragma unroll
                for (int q = 0; q < 7; ++q) cc[u][q] = c[q];
            }
            fv[u] = f ? gf[p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const unsigned b = in_grid[u];
            double acc = 0.0;
#pragma unroll
            for (int q = 1; q < 7; ++q) acc = fma((b >> q & 1u) ? cc[u][q] : 0.0, v[u][q], acc);
            acc = fma(cc[u][0], v[u][0], acc);
            const double r = f ? fv[u] - acc : sc * acc;
            if (pb + (long long)u * NT < P1) {
                gout[pp[u]] = r;
                sq += r * r;
            }
        }
    }
    return sq;
}

// Y[:, l] += sum_{c < nc} V[:, c] M[c * ldm + l] for l < nout <= NMAX (M in LDS)
// over the points of R; returns this thread's share of ||Y[:, 0]||^2 after the
// update when norm.  Threads own point pairs (16-byte loads); eight columns of
// V are loaded while the previous eight are summed; the sum over c runs in
// column order.  Lanes
// l >= nout compute on clamped (valid) columns and are never stored, so the
// loops have no data-dependent branches.
template <int NT, int NMAX>
__device__ double wg_lincomb(const double* V, long long ld, int nc, const double* M, int ldm,
                             double* Y, long long ldy, int nout, const Range& R, bool norm) {
    double nacc = 0.0;
    int lc[NMAX];
#pragma unroll
    for (int l = 0; l < NMAX; ++l) lc[l] = l < nout ? l : nout - 1;
    for (long long p = R.pa + 2 * threadIdx.x; p < R.pb; p += 2 * NT) {
        d2v a[NMAX];
#pragma unroll
        for (int l = 0; l < NMAX; ++l) a[l] = ld2nt(Y + lc[l] * ldy + p);
        int c = 0;
        // software pipeline: the next eight columns load while these FMAs run
        d2v vn[8];
        if (8 <= nc) {
#pragma unroll
            for (int u = 0; u < 8; ++u) vn[u] = ld2nt(V + (long long)u * ld + p);
        }
        for (; c + 8 <= nc; c += 8) {
            d2v v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = vn[u];
            if (c + 16 <= nc) {
#pragma unroll
                for (int u = 0; u < 8; ++u) vn[u] = ld2nt(V + (long long)(c + 8 + u) * ld + p);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int l = 0; l < NMAX; ++l) {
                    const double mm = lds(M + (c + u) * ldm + lc[l]);
                    a[l].x = fma(v[u].x, mm, a[l].x);
                    a[l].y = fma(v[u].y, mm, a[l].y);
                }
        }
        // the last nc mod 8 columns: four at a time with their loads issued
        // together, then one at a time, summed in column order
        for (; c + 4 <= nc; c += 4) {
            d2v v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = ld2nt(V + (long long)(c + u) * ld + p);
#pragma unroll
            for (int u = 0; u < 4; ++u)
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
            if (l < nout) st2nt(Y + l * ldy + p, a[l]);
        if (norm) nacc += a[0].x * a[0].x + a[0].y * a[0].y;
    }
    // the (at most two) single points of the range
    const long long pe = threadIdx.x == 0 ? R.e0 : (threadIdx.x == 1 ? R.e1 : -1);
    if (pe >= 0) {
        double a[NMAX];
#pragma unroll
        for (int l = 0; l < NMAX; ++l) a[l] = ldg(Y + lc[l] * ldy + pe);
        for (int c = 0; c < nc; ++c) {
            const double v = ldg(V + (long long)c * ld + pe);
#pragma unroll
            for (int l = 0; l < NMAX; ++l) a[l] = fma(v, lds(M + c * ldm + lc[l]), a[l]);
        }
#pragma unroll
        for (int l = 0; l < NMAX; ++l)
            if (l < nout) stg(Y + l * ldy + pe, a[l]);
        if (norm) nacc += a[0] * a[0];
    }
    return nacc;
}

// out[a * nz + j] = sum_{p in R} X[:, a][p] Z[:, j][p] (a < ncx, j < nz <= KZ).
// The waves of the workgroup walk the same 256 points per step, each lane two
// point pairs 128 points apart, wave w taking CAW columns of X in the current
// pass (CAW NT/64 columns per pass; CAW is chosen by the caller to cover the
// columns of X with few passes within the register budget).  The step's Z tile (KZ columns x 128 pairs x 16 bytes) is loaded once
// for the workgroup, two steps ahead, into a three-deep LDS ring (ztile: 3
// tiles of KZ*128 + 1 pairs; the extra pair takes the loads of threads without
// a tile slot), so Z is read once per pass rather than once per few columns of
// X.  X is loaded one step ahead.  The step loop is unrolled by two with named
// register sets and every load in it is unconditional (addresses past the
// range clamp to its last step).  Each lane sums its pairs in point order.
// Each wave reduces its own columns.  Columns past ncx / nz are clamped to
// valid ones and their sums dropped.
template <int KZ>
constexpr int gram_ztile_pairs() { return 3 * (KZ * 128 + 1); }

template <int NT, int KZ, int CAW>
__device__ void wg_gram(const double* X, long long ldx, int ncx, const double* Z, long long ldz,
                        int nz, const Range& R, double* out /* [ncx][nz] */, d2v* ztile) {
    constexpr int STEP = 256, TP = KZ * 128, TS = TP + 1,
                  NSL = (TP + NT - 1) / NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    SSTEP_LDS d2v* zt = (SSTEP_LDS d2v*)ztile;
    const double* zq[NSL];
    int zd[NSL];
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
        const int q = threadIdx.x + NT * i;
        const bool slot = q < TP;
        const int j0 = slot ? q / 128 : 0;
        const int j = j0 < nz ? j0 : nz - 1;
        zq[i] = Z + (long long)j * ldz + (slot ? (q % 128) * 2 : 0);
        zd[i] = slot ? q : TP;
    }
    const long long nstep = (R.pb - R.pa) / STEP;
    auto at = [&](long long st) { return R.pa + (st < nstep ? st : nstep - 1) * STEP; };
    for (int c0 = 0; c0 < ncx; c0 += (NT / 64) * CAW) {
        const int cw = c0 + wave * CAW;
        const double* xc[CAW];
#pragma unroll
        for (int a = 0; a < CAW; ++a) xc[a] = X + (long long)(cw + a < ncx ? cw + a : ncx - 1) * ldx;
        double acc[CAW][KZ];
#pragma unroll
        for (int a = 0; a < CAW; ++a)
#pragma unroll
            for (int j = 0; j < KZ; ++j) acc[a][j] = 0.0;
        if (nstep > 0) {
            // step st: issue X(st+1), Z(st+2); FMAs on X(st) and tile st mod 3;
            // store the Z loaded at step st-1 into tile (st+1) mod 3 (last read
            // at step st-2); barrier
            auto half = [&](long long st, d2v (&xcur)[CAW][2], d2v (&xnext)[CAW][2],
                            d2v (&zload)[NSL], const d2v (&zstore)[NSL]) {
                const long long px = at(st + 1) + 2 * lane, pz = at(st + 2);
#pragma unroll
                for (int a = 0; a < CAW; ++a) {
                    xnext[a][0] = ld2nt(xc[a] + px);
                    xnext[a][1] = ld2nt(xc[a] + px + 128);
                }
#pragma unroll
                for (int i = 0; i < NSL; ++i) zload[i] = ld2(zq[i] + pz);
                __builtin_amdgcn_sched_barrier(0);  // the loads go out before the FMAs
                const SSTEP_LDS d2v* tile = zt + (int)(st % 3) * TS;
#pragma unroll
                for (int j = 0; j < KZ; ++j) {
                    const d2v z0 = tile[j * 128 + lane], z1 = tile[j * 128 + 64 + lane];
#pragma unroll
                    for (int a = 0; a < CAW; ++a) {
                        acc[a][j] = fma(xcur[a][0].y, z0.y, fma(xcur[a][0].x, z0.x, acc[a][j]));
                        acc[a][j] = fma(xcur[a][1].y, z1.y, fma(xcur[a][1].x, z1.x, acc[a][j]));
                    }
                }
                SSTEP_LDS d2v* w = zt + (int)((st + 1) % 3) * TS;
#pragma unroll
                for (int i = 0; i < NSL; ++i) w[zd[i]] = zstore[i];
                __syncthreads();
            };
            d2v xa[CAW][2], xb[CAW][2], za[NSL], zb[NSL];
#pragma unroll
            for (int i = 0; i < NSL; ++i) {
                zt[zd[i]] = ld2(zq[i] + at(0));
                zb[i] = ld2(zq[i] + at(1));
            }
#pragma unroll
            for (int a = 0; a < CAW; ++a) {
                xa[a][0] = ld2nt(xc[a] + at(0) + 2 * lane);
                xa[a][1] = ld2nt(xc[a] + at(0) + 2 * lane + 128);
            }
            __syncthreads();
            long long st = 0;
            for (; st + 2 <= nstep; st += 2) {
                half(st, xa, xb, za, zb);
                half(st + 1, xb, xa, zb, za);
            }
            if (st < nstep) half(st, xa, xb, za, zb);
        }
        // pairs after the last whole step (one per lane per 128 points, in
        // point order), then the (at most two) single points
        for (long long p = R.pa + nstep * STEP + 2 * lane; p < R.pb; p += 128) {
            d2v x[CAW];
#pragma unroll
            for (int a = 0; a < CAW; ++a) x[a] = ld2(xc[a] + p);
#pragma unroll
            for (int j = 0; j < KZ; ++j) {
                const d2v zv = ld2(Z + (long long)(j < nz ? j : nz - 1) * ldz + p);
#pragma unroll
                for (int a = 0; a < CAW; ++a)
                    acc[a][j] = fma(x[a].y, zv.y, fma(x[a].x, zv.x, acc[a][j]));
            }
        }
        const long long pe = lane == 0 ? R.e0 : (lane == 1 ? R.e1 : -1);
        if (pe >= 0) {
#pragma unroll
            for (int a = 0; a < CAW; ++a) {
                const double xv = ldg(xc[a] + pe);
#pragma unroll
                for (int j = 0; j < KZ; ++j)
                    acc[a][j] = fma(xv, ldg(Z + (long long)(j < nz ? j : nz - 1) * ldz + pe), acc[a][j]);
            }
        }
#pragma unroll
        for (int a = 0; a < CAW; ++a)
#pragma unroll
            for (int j = 0; j < KZ; ++j) {
                const double t = wave_sum(acc[a][j]);
                if (lane == 0 && cw + a < ncx && j < nz) out[(cw + a) * nz + j] = t;
            }
        __syncthreads();  // the next pass rewrites tiles 0 and 1
    }
}

// Symmetric block Gram out[a * k + b] = sum_{p in R} Y[:, a][p] Y[:, b][p]
// (a, b < k <= KMAX), every column read once (the general Gram would read
// each column twice, as X and as Z).  Threads own point pairs (16-byte loads,
// 2 NT points apart; with KMAX <= 5 the next pair's columns load while the
// current pair's products are summed) and keep the upper triangle; the sums
// are reduced over each wave, then over the waves in wave order through
// scratch, an LDS area of NT / 64 * KMAX (KMAX + 1) / 2 doubles.  Columns past
// k are clamped to valid ones and their sums dropped.  Out of line, like the
// stencil pass, so its registers do not push the solve's state into scratch
// inside the other streaming loops.
template <int NT, int KMAX>
__device__ __noinline__ void wg_gram_sym(const double* Y, long long ld, int k, const Range& R, double* out,
                            double* scratch) {
    constexpr int NT2 = KMAX * (KMAX + 1) / 2;
    constexpr bool PF = KMAX <= 5;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    SSTEP_LDS double* sc = (SSTEP_LDS double*)scratch;
    const double* yc[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) yc[c] = Y + (long long)(c < k ? c : k - 1) * ld;
    double acc[NT2];
#pragma unroll
    for (int t = 0; t < NT2; ++t) acc[t] = 0.0;
    auto accum = [&](const d2v (&v)[KMAX]) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < KMAX; ++a)
#pragma unroll
            for (int b = a; b < KMAX; ++b, ++t)
                acc[t] = fma(v[a].y, v[b].y, fma(v[a].x, v[b].x, acc[t]));
    };
    long long p = R.pa + 2 * (long long)threadIdx.x;
    if constexpr (PF) {
        d2v cur[KMAX], nxt[KMAX];
        if (p < R.pb) {
#pragma unroll
            for (int c = 0; c < KMAX; ++c) cur[c] = ld2(yc[c] + p);
        }
        for (; p < R.pb; p += 2 * NT) {
            const long long pn = p + 2 * NT;
            if (pn < R.pb) {
#pragma unroll
                for (int c = 0; c < KMAX; ++c) nxt[c] = ld2(yc[c] + pn);
            }
            accum(cur);
#pragma unroll
            for (int c = 0; c < KMAX; ++c) cur[c] = nxt[c];
        }
    } else {
        for (; p < R.pb; p += 2 * NT) {
            d2v v[KMAX];
#pragma unroll
            for (int c = 0; c < KMAX; ++c) v[c] = ld2(yc[c] + p);
            accum(v);
        }
    }
    // the (at most two) single points of the range
    const long long pe = threadIdx.x == 0 ? R.e0 : (threadIdx.x == 1 ? R.e1 : -1);
    if (pe >= 0) {
        double v[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) v[c] = ldg(yc[c] + pe);
        int t = 0;
#pragma unroll
        for (int a = 0; a < KMAX; ++a)
#pragma unroll
            for (int b = a; b < KMAX; ++b, ++t) acc[t] = fma(v[a], v[b], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < NT2; ++t) {
        const double w = wave_sum(acc[t]);
        if (lane == 0) sc[wave * NT2 + t] = w;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < k * k; q += NT) {
        const int a = q / k, b = q % k;
        const int i = a < b ? a : b, j = a < b ? b : a;
        const int t = i * KMAX - i * (i - 1) / 2 + (j - i);
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) sum += sc[w * NT2 + t];
        out[a * k + b] = sum;
    }
    __syncthreads();
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

// LDS state of a workgroup handed to the solve.
struct WgShared {
    double* red;
    d2v* ztile;  // Z tiles of the block Gram: 3 x ((KZ + 1) * 128 + 1) pairs
    double* sh;
    double* lw;
    GramFactor* lf;
    double* lm;
    double* l1;
    long long* clk;
};

// The whole restarted s-step GMRES for one system, by a team (T >= 1).
template <int NT, int GC, int KZ>
__device__ void solve_sys(const BatchArgs& args, BatchSys& S, BatchSlot& W, const WgShared& L,
                          const StencilView& A, Team& tm) {
    const int s = args.s, m = args.m, K = m * s, ldg_ = K + 1, s1 = s + 1;
    const long long N = A.N, ld = S.ld;
    double* V = S.ws;
    const int tid = threadIdx.x;
    const double sigma = S.sigma;
    // this member's rows of the grid
    const long long rows = (long long)A.ny * A.nz;
    const long long r0 = rows * tm.rank / tm.T, r1 = rows * (tm.rank + 1) / tm.T;
    const Range R(r0 * A.nx, r1 * A.nx);
    double* red = L.red;
    d2v* ztile = L.ztile;
    double* sh = L.sh;
    double* lm = L.lm;

    PhaseClock pc{L.clk};
    pc.start();
    // ||f||
    double acc = 0.0;
    for (long long p = R.P0 + tid; p < R.P1; p += NT) {
        const double v = ldg(S.f + p);
        acc += v * v;
    }
    const double fnorm = sqrt(team_scalar<NT>(tm, W, wg_sum<NT>(acc, red), L.l1));
    pc.lap(SSTEP_K_VEC);
    const double tol_abs = args.tol * fnorm;
    int blocks = 0, cycles = 0, status = SSTEP_NOT_CONVERGED;
    double beta = 0.0;
    for (;;) {
        // r = f - A x into column 0, beta = ||r||
        acc = wg_stencil<NT>(A, S.x, V, 1.0, S.f, R.P0, R.P1);
        beta = sqrt(team_scalar<NT>(tm, W, wg_sum<NT>(acc, red), L.l1));
        pc.lap(SSTEP_K_RESID);
        if (tm.failed) { status = SSTEP_ERR_HIP; break; }
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
            // matrix powers: y_j = A y_{j-1} / sigma, y_0 = stored column * inv_nu;
            // the next level reads neighbouring members' rows
            for (int jl = 1; jl <= s; ++jl) {
                const double* in = Yk + (long long)(jl - 1) * ld;
                double* out = Yk + (long long)jl * ld;
                const double sc = (jl == 1 ? W.inv_nu[kb] : 1.0) / sigma;
                (void)wg_stencil<NT>(A, in, out, sc, nullptr, R.P0, R.P1);
                team_barrier(tm);
            }
            pc.lap(SSTEP_K_MPK);
            if (kb > 0) {
                // C = V_prev^T [y_1..y_s]
                double* gout = tm.T == 1 ? W.C : W.part[tm.parity];
                // the stored blocks: many columns of X, GC per wave and pass
                wg_gram<NT, KZ, GC>(V, ld, c0, Yk + ld, ld, s, R, gout, ztile);
                if (tm.T > 1) team_combine<NT>(tm, W, c0 * s, W.C);
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
                // y_j -= sum_c V_c coefM[c][j]  (coefficients in LDS, own rows only)
                wg_lincomb<NT, KZ>(V, ld, c0, lm, s, Yk + ld, ld, s, R, false);
                __syncthreads();
                pc.lap(SSTEP_K_UPDATE);
            }
            // block Gram of [w_k, y_1..y_s]
            {
                double* gout = tm.T == 1 ? W.C : W.part[tm.parity];
                // symmetric: each column read once; the Z-tile area is the
                // reduction scratch (free between the Gram passes)
                wg_gram_sym<NT, KZ + 1>(Yk, ld, s1, R, gout, reinterpret_cast<double*>(ztile));
                if (tm.T > 1) team_combine<NT>(tm, W, s1 * s1, W.C);
            }
            pc.lap(SSTEP_K_GRAM);
            if (tid == 0) scalar_factor(W, kb, s, args.rank_tol, L.lw, L.lf, sh);
            __syncthreads();
            {
                const double* src = reinterpret_cast<const double*>(L.lf);
                double* dst = reinterpret_cast<double*>(&W.Wf[kb]);
                for (int i = tid; i < (int)(sizeof(GramFactor) / sizeof(double)); i += NT) dst[i] = src[i];
            }
            __syncthreads();
            pc.lap(SSTEP_K_SCALAR);
            const int q = W.Wf[kb].rank;
            if (q == 0 || tm.failed) { err = true; break; }
            double nu = 0.0;
            if (q == s) {
                // w_hat = Yhat_s - V_k g, nu^2 (the next matrix powers read it)
                double* ys = Yk + (long long)s * ld;
                acc = wg_lincomb<NT, 1>(Yk, ld, s, sh + s, 1, ys, ld, 1, R, true);
                nu = sqrt(team_scalar<NT>(tm, W, wg_sum<NT>(acc, red), L.l1));
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
                    // four steps' loads issued together (the G entries are read
                    // whether or not their coefficient is 0; all lie inside G)
                    int cp = r > 0 ? r - 1 : 0;
                    for (; cp + 4 <= c0; cp += 4) {
                        double tv[4], gv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            tv[u] = W.T[(cp + u) * s1 + j];
                            gv[u] = W.G[r + (cp + u) * ldg_];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (tv[u] != 0.0) val -= gv[u] * tv[u];
                    }
                    for (; cp < c0; ++cp) {
                        const double t = W.T[cp * s1 + j];
                        if (t != 0.0) val -= W.G[r + cp * ldg_] * t;
                    }
                }
                W.G[r + (c0 + j) * ldg_] = val;
            }
            __syncthreads();
            for (int idx = tid; idx < q * (c0 + q + 1); idx += NT) {
                const int j = idx / (c0 + q + 1), r = idx % (c0 + q + 1);
                const double* gc = W.G + (c0 + j) * ldg_;
                double val;
                if (r == c0 + q) {
                    val = gc[r];
                } else {
                    const int i = r / s, pp = r % s;
                    const int qi = (i < kb) ? s : q;
                    val = 0.0;
                    for (int b = pp; b < qi; ++b) val += gram_L(W.Wf[i], pp, b) * gc[i * s + b];
                }
                W.R[r + (c0 + j) * ldg_] = val;
            }
            __syncthreads();
            if (tid < q) {
                // the earlier rotations on the new columns, one thread per
                // column; eight rotations' operands loaded together (each
                // col[i + 1] is read before col[i + 1] is rewritten, as in the
                // one-at-a-time order)
                double* col = W.R + (c0 + tid) * ldg_;
                double x0 = col[0];
                int i = 0;
                for (; i + 8 <= c0; i += 8) {
                    double cv[8], sv[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        cv[u] = W.cs[i + u];
                        sv[u] = W.sn[i + u];
                        xv[u] = col[i + u + 1];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        col[i + u] = cv[u] * x0 + sv[u] * xv[u];
                        x0 = -sv[u] * x0 + cv[u] * xv[u];
                    }
                }
                for (; i < c0; ++i) {
                    const double cth = W.cs[i], sth = W.sn[i], x1 = col[i + 1];
                    col[i] = cth * x0 + sth * x1;
                    x0 = -sth * x0 + cth * x1;
                }
                col[c0] = x0;
            }
            __syncthreads();
            if (tid == 0) scalar_givens(W, kb, c0, q, ldg_, nu, sh);
            __syncthreads();
            pc.lap(SSTEP_K_SCALAR);
            ncols = c0 + q;
            ++blocks;
            const double est = sh[2 * kMaxS + 1];
            if (!isfinite(est)) { err = true; break; }
            if (est <= tol_abs || lucky || q < s) break;
        }
        if (err) { status = tm.failed ? SSTEP_ERR_HIP : SSTEP_ERR_NONFINITE; break; }
        // y = R^{-1} rhs, assembly x += V y on own rows; the residual that
        // follows reads neighbouring members' rows of x
        if (tid == 0) scalar_ysolve(W, ncols, s, ldg_, lm);
        __syncthreads();
        wg_lincomb<NT, 1>(V, ld, ncols, lm, 1, S.x, N, 1, R, false);
        team_barrier(tm);
        pc.lap(SSTEP_K_UPDATE);
    }
    if (tid == 0 && tm.rank == 0) {
        S.status = status;
        S.blocks = blocks;
        S.cycles = cycles;
        S.team = tm.T;
        S.rel_resid = fnorm > 0.0 ? beta / fnorm : beta;
        for (int c = 0; c < SSTEP_K_NCLASS; ++c) S.ticks[c] = L.clk[c];
    }
    __syncthreads();
}

// NT threads per workgroup, GC stored-block columns per wave in the block
// Gram, KZ = 4 (s <= 4) or 8 (s <= 8)
template <int NT, int GC, int KZ>
__global__ __launch_bounds__(NT) void k_batched_gmres(BatchArgs args) {
    __shared__ double red[NT / 64];
    __shared__ d2v ztile[gram_ztile_pairs<KZ + 1>()];
    // the symmetric block Gram reduces its per-wave sums through this area
    static_assert((NT / 64) * (KZ + 1) * (KZ + 2) / 2 * sizeof(double) <= sizeof(ztile),
                  "Z-tile area too small for the symmetric Gram's reduction");
    __shared__ double sh[3 * kMaxS + 4];
    __shared__ double lw[kMaxS * kMaxS];
    __shared__ GramFactor lf;
    __shared__ double lm[512 * 8];  // update / assembly coefficients
    __shared__ double l1[2];
    __shared__ StencilView sA;      // the current system's operator
    __shared__ long long clk[SSTEP_K_NCLASS + 1];
    __shared__ Team tm;
    __shared__ int next;
    // filled member by member: a braced initializer of LDS addresses would be
    // folded into a static initializer the compiler cannot emit
    WgShared L;
    L.red = red;
    L.ztile = ztile;
    L.sh = sh;
    L.lw = lw;
    L.lf = &lf;
    L.lm = lm;
    L.l1 = l1;
    L.clk = clk;
    BatchSlot& W = args.slots[blockIdx.x];
    int* abort = args.queue + 2;

    // phase 1: large systems, teams of args.team workgroups on one XCD
    if (args.team > 1 && args.nbig > 0) {
        if (threadIdx.x == 0) {
            const int T = args.team, G = gridDim.x, b = blockIdx.x;
            const int per_xcd = G / 8, tpx = per_xcd / T;
            const int x = b % 8, k = b / 8;
            const int id = x * tpx + k / T;
            tm.T = T;
            tm.rank = k % T;
            tm.parity = 0;
            tm.failed = 0;
            tm.local = 0;
            tm.target = 0;
            tm.cnt = args.team_sync + (size_t)id * 64;
            tm.mailbox = (int*)(args.team_sync + (size_t)id * 64 + 32);
            tm.abort = abort;
            tm.limit = args.spin_limit;
            for (int r = 0; r < T; ++r) tm.member[r] = args.slots + ((k / T) * T + r) * 8 + x;
            // publish this member's XCD (words 40.. of the team's block)
            __hip_atomic_store((int*)(tm.cnt + 40 + tm.rank), (int)xcd_id() + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        // the cheaper barrier only where the hardware reports one XCD for the
        // whole team (the grouping by blockIdx.x mod 8 is the usual dispatch)
        if (team_barrier(tm) && threadIdx.x == 0) {
            int same = 1;
            const int x0 = __hip_atomic_load((int*)(tm.cnt + 40), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int r = 1; r < tm.T; ++r)
                same &= __hip_atomic_load((int*)(tm.cnt + 40 + r), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) == x0;
            tm.local = same && x0 > 0;
        }
        __syncthreads();
        for (;;) {
            if (tm.rank == 0 && threadIdx.x == 0) {
                const int k = atomicAdd(args.queue + 0, 1);
                __hip_atomic_store(tm.mailbox, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (!team_barrier(tm)) break;
            if (threadIdx.x == 0)
                next = __hip_atomic_load(tm.mailbox, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int k = next;
            if (k >= args.nbig) break;
            BatchSys& S = args.sys[args.order_big[k]];
            if (threadIdx.x == 0) sA = S.A;
            __syncthreads();
            solve_sys<NT, GC, KZ>(args, S, W, L, sA, tm);
            if (tm.failed) break;
        }
        __syncthreads();
    }
    // phase 2: small systems, one workgroup each
    if (threadIdx.x == 0) {
        tm.T = 1;
        tm.rank = 0;
        tm.parity = 0;
        tm.failed = 0;
    }
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0)
            next = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       ? args.nsmall
                       : atomicAdd(args.queue + 1, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();
        if (k >= args.nsmall) break;
        BatchSys& S = args.sys[args.order_small[k]];
        if (threadIdx.x == 0) sA = S.A;
        __syncthreads();
        solve_sys<NT, GC, KZ>(args, S, W, L, sA, tm);
    }
}

// queue words, abort flag and team counters, cleared by a kernel (recorded as
// a kernel node in the graph: no memset node)
static __global__ void k_batch_reset(int* queue, unsigned* team_sync, int nwords) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4) queue[i] = 0;
    if (i < nwords) team_sync[i] = 0u;
}

// ---------------------------------------------------------------------------
// host side: a plan uploads the system table once, captures the reset and the
// persistent launch in a hipGraph, and replays it per execution.
// ---------------------------------------------------------------------------
struct BatchPlan {
    int nsys = 0, s = 0, m = 0, threads = 512, wgs_per_cu = 1, nslots = 0, team = 1, nteam_words = 0;
    int gram_cols = 0;  // 0: the default Gram column tile
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

// Calls f(kernel) with the instance for (threads, s, Gram column tile);
// gram_cols 0 = the default tile.
template <typename F>
static void with_batch_kernel(int threads, int s, int gram_cols, F&& f) {
#define SSTEP_BK(NT, GC, KZ) f(reinterpret_cast<const void*>(&k_batched_gmres<NT, GC, KZ>))
    if (s <= 4) {
        const bool narrow = gram_cols == 2;
        if (threads == 256) { if (narrow) SSTEP_BK(256, 2, 4); else SSTEP_BK(256, 4, 4); }
        else if (threads == 512) { if (narrow) SSTEP_BK(512, 2, 4); else SSTEP_BK(512, 4, 4); }
        else { if (narrow) SSTEP_BK(1024, 2, 4); else SSTEP_BK(1024, 4, 4); }
    } else {
        const bool narrow = gram_cols == 1;
        if (threads == 256) { if (narrow) SSTEP_BK(256, 1, 8); else SSTEP_BK(256, 2, 8); }
        else if (threads == 512) { if (narrow) SSTEP_BK(512, 1, 8); else SSTEP_BK(512, 2, 8); }
        else { if (narrow) SSTEP_BK(1024, 1, 8); else SSTEP_BK(1024, 2, 8); }
    }
#undef SSTEP_BK
}

static const void* batch_kernel_for(int threads, int s, int gram_cols) {
    const void* k = nullptr;
    with_batch_kernel(threads, s, gram_cols, [&](const void* kern) { k = kern; });
    return k;
}

static void batch_enqueue(const BatchPlan& P, hipStream_t s) {
    const int nw = std::max(P.nteam_words, 4);
    hipLaunchKernelGGL(k_batch_reset, dim3((nw + 255) / 256), dim3(256), 0, s, P.args.queue,
                       P.args.team_sync, P.nteam_words);
    BatchArgs args = P.args;
    void* params[] = {&args};
    const void* k = batch_kernel_for(P.threads, P.s, P.gram_cols);
    SSTEP_HIP(hipLaunchKernel(k, dim3(P.nslots), dim3(P.threads), params, 0, s));
}

// slots: compute units x workgroups per CU (every workgroup resident); without
// teams no more workgroups than systems
int batched_slots(int nsys, int wgs_per_cu, int team) {
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int full = std::max(1, ncu) * wgs_per_cu;
    return team > 1 ? full : std::min(nsys, full);
}

size_t batched_workspace_bytes(int nsys, const sstep_stencil* A, int s, int m, int nslots) {
    size_t tot = 0;
    for (int i = 0; i < nsys; ++i)
        tot += ((size_t)(m * s + 1) * col_stride(grid_points(A[i])) * sizeof(double) + 255) / 256 * 256;
    tot += (sizeof(BatchSlot) * (size_t)nslots + 255) / 256 * 256 + 4096 +
           (sizeof(unsigned) * 64 * (size_t)nslots + 255) / 256 * 256 +
           (sizeof(BatchSys) * (size_t)nsys + 255) / 256 * 256 +
           2 * ((sizeof(int) * (size_t)nsys + 255) / 256 * 256);
    return tot;
}

int batched_plan_create(void** out, int nsys, const sstep_stencil* A, const double* const* f,
                        double* const* x, int s, int m, double tol, const sstep_options& opt) {
    BatchPlan* P = new BatchPlan();
    P->nsys = nsys;
    P->s = s;
    P->m = m;
    P->threads = opt.batch_threads > 0 ? opt.batch_threads : 512;
    P->wgs_per_cu = opt.batch_wgs_per_cu > 0 ? opt.batch_wgs_per_cu : 1;
    P->team = opt.batch_team > 0 ? opt.batch_team : 1;
    P->gram_cols = opt.batch_gram_cols;
    P->nslots = batched_slots(nsys, P->wgs_per_cu, P->team);
    P->st = (hipStream_t)opt.stream;
    {
        int dev = 0, khz = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            P->tick_khz = khz;
        else
            (void)hipGetLastError();
    }
    // teams need every workgroup resident and whole teams inside each XCD
    if (P->team > 1) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_kernel_for(P->threads, s, P->gram_cols),
                                                         P->threads, 0) != hipSuccess) {
            (void)hipGetLastError();
            occ = 0;
        }
        if (occ < P->wgs_per_cu || P->nslots % (8 * P->team) != 0) {
            P->team = 1;
            P->nslots = batched_slots(nsys, P->wgs_per_cu, 1);
        }
    }
    P->nteam_words = P->nslots * 64;
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
        unsigned* team_sync = (unsigned*)take(sizeof(unsigned) * 64 * (size_t)P->nslots);
        P->dsys = (BatchSys*)take(sizeof(BatchSys) * nsys);
        int* dbig = (int*)take(sizeof(int) * nsys);
        int* dsmall = (int*)take(sizeof(int) * nsys);
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
            // scanned on the device; the queue words are free scratch until launch)
            b.sigma = op_params(A[i], opt.sigma, P->st, (double*)queue).sigma;
        }
        std::vector<int> order(nsys);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return P->hs[a].A.N > P->hs[b].A.N; });
        // large systems go to the teams: at least 16384 points and 4 grid rows
        // per member
        std::vector<int> big, small;
        for (int i : order) {
            const long long rows = (long long)P->hs[i].A.ny * P->hs[i].A.nz;
            const bool is_big = P->team > 1 && P->hs[i].A.N >= (long long)P->team * 16384 &&
                                rows >= 4LL * P->team;
            (is_big ? big : small).push_back(i);
        }
        if (!big.empty())
            SSTEP_HIP(hipMemcpyAsync(dbig, big.data(), sizeof(int) * big.size(),
                                     hipMemcpyHostToDevice, P->st));
        if (!small.empty())
            SSTEP_HIP(hipMemcpyAsync(dsmall, small.data(), sizeof(int) * small.size(),
                                     hipMemcpyHostToDevice, P->st));
        SSTEP_HIP(hipMemcpyAsync(P->dsys, P->hs.data(), sizeof(BatchSys) * nsys,
                                 hipMemcpyHostToDevice, P->st));
        SSTEP_HIP(hipStreamSynchronize(P->st));
        BatchArgs& args = P->args;
        args.sys = P->dsys;
        args.order_big = dbig;
        args.order_small = dsmall;
        args.nbig = (int)big.size();
        args.nsmall = (int)small.size();
        args.s = s;
        args.m = m;
        args.tol = tol;
        args.max_blocks = opt.max_iters > 0 ? opt.max_iters : 10000;
        args.rank_tol = 1e-14;
        args.lucky_tol = 1e-14;
        args.slots = slots;
        args.queue = queue;
        args.team_sync = team_sync;
        args.team = P->team;
        args.spin_limit = 1LL << 22;  // seconds of polling per barrier before giving up
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
            info[i].matvecs = b.team;  // workgroups that solved this system
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
