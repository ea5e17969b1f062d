// kernels.hpp -- HIP kernels (gfx950) for the data-parallel part of the
// s-step methods: stencil operator, matrix powers, true residual, block Gram
// (all inner products of one s-step), block updates (linear combinations).
//
// Memory layout: every vector is one column of N elements; a block of
// columns has a column stride ld (a multiple of 64 elements, so each column
// starts 256-byte aligned).  Reductions are deterministic: per-workgroup
// partial sums in a fixed order, then a fixed-order second pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace sstep {

constexpr int kThreads = 256;  // 4 wave64 per workgroup

struct StencilView {
    int ndim, nx, ny, nz;
    long long N;
    double c[7];
    const double* coef;  // [7][N] or nullptr
};

// Workgroup b is dispatched to XCD (b mod 8).  Give every XCD a contiguous
// range of logical tiles so that neighbouring tiles (stencil halos, the
// shared right-hand block of a Gram) meet in the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
    const unsigned nfull = nb & ~7u;
    if (b >= nfull) return b;
    return (b & 7u) * (nfull >> 3) + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV per-thread values over the workgroup.  Result valid in out[0..NV)
// for threads 0..NV-1 (written by those threads only).  lds: >= 4*NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum(const double (&v)[NV], double* lds, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = wave_sum(v[k]);
        if (lane == 0) lds[wave * NV + k] = t;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NV; k += kThreads)
        out[k] = (lds[k] + lds[NV + k]) + (lds[2 * NV + k] + lds[3 * NV + k]);
}

template <typename T>
__device__ __forceinline__ double to_f64(T v) { return static_cast<double>(v); }

// ---------------------------------------------------------------------------
// Stencil level: out = alpha * A(y) + beta * y + gam * z,
//   y = in * in_scale, z = prev * prev_scale  (scales from device pointers,
//   nullptr = 1).  One workgroup per 256-point row segment; rows are mapped
//   XCD-contiguously.  Neighbour order -x, +x, -y, +y, -z, +z, then centre.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_stencil_level(
    StencilView A, int nseg, const T* __restrict__ in, const double* __restrict__ in_scale,
    const T* __restrict__ prev, const double* __restrict__ prev_scale, double alpha, double beta,
    double gam, T* __restrict__ out, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int seg = t % nseg;
    const unsigned row = t / nseg;
    const int j = row % A.ny, l = row / A.ny;
    const int i = seg * kThreads + threadIdx.x;
    if (i >= A.nx) return;
    const long long sy = A.nx, sz = (long long)A.nx * A.ny;
    const long long p = i + sy * j + sz * l;
    T c[7];
    if (A.coef) {
#pragma unroll
        for (int q = 0; q < 7; ++q) c[q] = (q < 2 * A.ndim + 1) ? (T)A.coef[q * A.N + p] : T(0);
    } else {
#pragma unroll
        for (int q = 0; q < 7; ++q) c[q] = (T)A.c[q];
    }
    T acc = 0;
    if (i > 0) acc += c[1] * in[p - 1];
    if (i < A.nx - 1) acc += c[2] * in[p + 1];
    if (j > 0) acc += c[3] * in[p - sy];
    if (j < A.ny - 1) acc += c[4] * in[p + sy];
    if (A.ndim == 3) {
        if (l > 0) acc += c[5] * in[p - sz];
        if (l < A.nz - 1) acc += c[6] * in[p + sz];
    }
    const T xc = in[p];
    acc += c[0] * xc;
    const T si = in_scale ? (T)*in_scale : T(1);
    T r = (T)alpha * si * acc;
    if (beta != 0.0) r += (T)beta * si * xc;
    if (gam != 0.0) {
        const T sp = prev_scale ? (T)*prev_scale : T(1);
        r += (T)gam * sp * prev[p];
    }
    out[p] = r;
}

// ---------------------------------------------------------------------------
// True residual r = f - A x in FP64 (x, f FP64); r stored as TR; per
// workgroup partial sum of r^2 (FP64, before rounding to TR).
// ---------------------------------------------------------------------------
template <typename TR>
__global__ __launch_bounds__(kThreads) void k_residual(StencilView A, int nseg,
                                                       const double* __restrict__ f,
                                                       const double* __restrict__ x,
                                                       TR* __restrict__ r, double* __restrict__ part) {
    __shared__ double lds[4];
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int seg = t % nseg;
    const unsigned row = t / nseg;
    const int j = row % A.ny, l = row / A.ny;
    const int i = seg * kThreads + threadIdx.x;
    double rr = 0.0;
    if (i < A.nx) {
        const long long sy = A.nx, sz = (long long)A.nx * A.ny;
        const long long p = i + sy * j + sz * l;
        double c[7];
#pragma unroll
        for (int q = 0; q < 7; ++q)
            c[q] = A.coef ? ((q < 2 * A.ndim + 1) ? A.coef[q * A.N + p] : 0.0) : A.c[q];
        double acc = 0.0;
        if (i > 0) acc += c[1] * x[p - 1];
        if (i < A.nx - 1) acc += c[2] * x[p + 1];
        if (j > 0) acc += c[3] * x[p - sy];
        if (j < A.ny - 1) acc += c[4] * x[p + sy];
        if (A.ndim == 3) {
            if (l > 0) acc += c[5] * x[p - sz];
            if (l < A.nz - 1) acc += c[6] * x[p + sz];
        }
        acc += c[0] * x[p];
        const double v = f[p] - acc;
        r[p] = (TR)v;
        rr = v * v;
    }
    double v1[1] = {rr}, o[1];
    block_sum<1>(v1, lds, o);
    if (threadIdx.x == 0) part[t] = o[0];
}

// ---------------------------------------------------------------------------
// 16-byte vector access helpers.  NT: non-temporal (streamed once; keeps the
// L2 for data that is re-read).
// ---------------------------------------------------------------------------
template <typename T, int PPT, bool NT>
__device__ __forceinline__ void load_pts(const T* __restrict__ p, T (&v)[PPT]) {
    constexpr int E = 16 / sizeof(T);
    static_assert(PPT % E == 0, "points per thread must fill 16-byte loads");
    typedef T vt __attribute__((ext_vector_type(E)));
#pragma unroll
    for (int q = 0; q < PPT / E; ++q) {
        vt t;
        if constexpr (NT) t = __builtin_nontemporal_load(reinterpret_cast<const vt*>(p + q * E));
        else t = *reinterpret_cast<const vt*>(p + q * E);
#pragma unroll
        for (int e = 0; e < E; ++e) v[q * E + e] = t[e];
    }
}
// The store goes through an explicit global-address-space pointer and p has
// no __restrict__: otherwise the compiler's rewriting of the inlined store
// can drop its non-temporal bit (a plain global_store; block updates measured
// 3-9% slower).
template <typename T, int PPT>
__device__ __forceinline__ void store_pts_nt(T* p, const T (&v)[PPT]) {
    constexpr int E = 16 / sizeof(T);
    typedef T vt __attribute__((ext_vector_type(E)));
#pragma unroll
    for (int q = 0; q < PPT / E; ++q) {
        vt t;
#pragma unroll
        for (int e = 0; e < E; ++e) t[e] = v[q * E + e];
        __builtin_nontemporal_store(t, (__attribute__((address_space(1))) vt*)(p + q * E));
    }
}
template <typename T, int PPT>
__device__ __forceinline__ void store_pts(T* __restrict__ p, const T (&v)[PPT]) {
    constexpr int E = 16 / sizeof(T);
    typedef T vt __attribute__((ext_vector_type(E)));
#pragma unroll
    for (int q = 0; q < PPT / E; ++q) {
        vt t;
#pragma unroll
        for (int e = 0; e < E; ++e) t[e] = v[q * E + e];
        *reinterpret_cast<vt*>(p + q * E) = t;
    }
}

// ---------------------------------------------------------------------------
// Block Gram, stage 1: for a point chunk and a group of 4*CAW columns of X,
//   partial[chunk][c][j] = sum_{p in chunk} X[c][p] * Z[j][p],  j < KZ
// Z = [Z1 (nz1 columns) | Z2 (nz2 columns)], nz1 + nz2 <= KZ.  Accumulation
// in FP64.  The four waves of a workgroup walk the same points, each with
// its own CAW columns of X (streamed with non-temporal 16-byte loads); the Z
// tile of a step (KZ columns x 64 lanes x 16 bytes) is loaded once per
// workgroup, two steps ahead, and read by all four waves from LDS, so Z costs
// one L2 read per 4*CAW columns of X and few registers.  The next step's X and
// the Z tile two steps ahead are in flight while the FMAs of the current step
// run.  Every load in the loop is issued unconditionally (addresses past the
// chunk clamp to its last step), so no branch makes the compiler wait for
// loads in flight.  Each wave reduces its own partials (no cross-wave sum is
// needed).
// ---------------------------------------------------------------------------
template <typename T, int CAW, int KZ>
__global__ __launch_bounds__(kThreads) void k_gram_partial(
    const T* __restrict__ X, long long ldx, int ncx, const T* __restrict__ Z1, long long ldz1,
    int nz1, const T* __restrict__ Z2, long long ldz2, int nz2, long long N, long long chunk,
    int nct, double* __restrict__ part, const int* __restrict__ skip) {
    if (skip && *skip) return;
    constexpr int PPT = 16 / sizeof(T);  // points per lane per step (one 16-byte load)
    constexpr int STEP = 64 * PPT;       // points per step (all four waves share them)
    constexpr int NSL = (KZ * 64 + kThreads - 1) / kThreads;  // Z slots per thread
    typedef T vt __attribute__((ext_vector_type(PPT)));
    // three Z tiles: step s is read from tile s mod 3 while step s+2 is written
    __shared__ vt zs[3][NSL * kThreads];
    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int ct = b % nct;
    const long long ch = b / nct;
    const long long p0 = ch * chunk;
    const long long p1 = (p0 + chunk < N) ? p0 + chunk : N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = ct * 4 * CAW + wave * CAW;
    const int nz = nz1 + nz2;
    // columns beyond ncx / nz alias valid ones; their sums are discarded
    const T* xc[CAW];
#pragma unroll
    for (int a = 0; a < CAW; ++a) xc[a] = X + (long long)(c0 + a < ncx ? c0 + a : ncx - 1) * ldx;
    // this thread's Z slots: slot q holds lane q%64's points of column q/64
    // (slots past KZ*64 load a valid column into the tile's padding)
    const T* zq[NSL];
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
        const int q = threadIdx.x + kThreads * i;
        const int j0 = q / 64;
        const int j = j0 < nz ? j0 : nz - 1;
        zq[i] = (j < nz1 ? Z1 + (long long)j * ldz1 : Z2 + (long long)(j - nz1) * ldz2) +
                (q % 64) * PPT;
    }
    double acc[CAW][KZ];
#pragma unroll
    for (int a = 0; a < CAW; ++a)
#pragma unroll
        for (int j = 0; j < KZ; ++j) acc[a][j] = 0.0;

    const long long nstep = (p1 - p0) / STEP;
    if (nstep > 0) {
        auto at = [&](long long st) { return p0 + (st < nstep ? st : nstep - 1) * STEP; };
        // Step st: issue X(st+1) and Z(st+2), run the FMAs of step st on X
        // registers and Z tile st mod 3, then store the Z registers loaded at
        // step st-1 into tile (st+1) mod 3 (last read at step st-2) and
        // synchronise.  The loop is unrolled by two with named register sets,
        // so every value is loaded in one half and consumed in the other
        // (no copies of loaded registers that would wait for the loads).
        auto half = [&](long long st, vt (&xcur)[CAW], vt (&xnext)[CAW], vt (&zload)[NSL],
                        const vt (&zstore)[NSL]) {
            const long long px = at(st + 1) + lane * PPT, pz = at(st + 2);
#pragma unroll
            for (int a = 0; a < CAW; ++a)
                xnext[a] = __builtin_nontemporal_load(reinterpret_cast<const vt*>(xc[a] + px));
#pragma unroll
            for (int i = 0; i < NSL; ++i) zload[i] = *reinterpret_cast<const vt*>(zq[i] + pz);
            __builtin_amdgcn_sched_barrier(0);  // the loads go out before the FMAs
            const vt* zt = zs[st % 3];
#pragma unroll
            for (int j = 0; j < KZ; ++j) {
                const vt zv = zt[j * 64 + lane];
#pragma unroll
                for (int a = 0; a < CAW; ++a)
#pragma unroll
                    for (int e = 0; e < PPT; ++e)
                        acc[a][j] = fma((double)xcur[a][e], (double)zv[e], acc[a][j]);
            }
            vt* zw = zs[(st + 1) % 3];
#pragma unroll
            for (int i = 0; i < NSL; ++i) zw[threadIdx.x + kThreads * i] = zstore[i];
            __syncthreads();
        };
        vt xa[CAW], xb[CAW], za[NSL], zb[NSL];
#pragma unroll
        for (int i = 0; i < NSL; ++i) {
            zs[0][threadIdx.x + kThreads * i] = *reinterpret_cast<const vt*>(zq[i] + at(0));
            zb[i] = *reinterpret_cast<const vt*>(zq[i] + at(1));
        }
#pragma unroll
        for (int a = 0; a < CAW; ++a)
            xa[a] = __builtin_nontemporal_load(reinterpret_cast<const vt*>(xc[a] + at(0) + lane * PPT));
        __syncthreads();
        long long st = 0;
        for (; st + 2 <= nstep; st += 2) {
            half(st, xa, xb, za, zb);
            half(st + 1, xb, xa, zb, za);
        }
        if (st < nstep) half(st, xa, xb, za, zb);
    }
    // ragged tail of the chunk: lanes over points, Z read directly
    for (long long q = p0 + nstep * STEP + lane; q < p1; q += 64) {
        double xq[CAW];
#pragma unroll
        for (int a = 0; a < CAW; ++a) xq[a] = to_f64(xc[a][q]);
#pragma unroll
        for (int j = 0; j < KZ; ++j) {
            const int jj = j < nz ? j : nz - 1;
            const T* zc = jj < nz1 ? Z1 + (long long)jj * ldz1 : Z2 + (long long)(jj - nz1) * ldz2;
            const double zv = to_f64(zc[q]);
#pragma unroll
            for (int a = 0; a < CAW; ++a) acc[a][j] = fma(xq[a], zv, acc[a][j]);
        }
    }
#pragma unroll
    for (int a = 0; a < CAW; ++a)
#pragma unroll
        for (int j = 0; j < KZ; ++j) {
            const double t = wave_sum(acc[a][j]);
            if (lane == 0 && c0 + a < ncx && j < nz) part[(ch * ncx + c0 + a) * KZ + j] = t;
        }
}

// Block Gram, stage 2: G[c*nz + j] = sum over chunks in a fixed order.
// 64 outputs per workgroup, 4 threads per output each summing a fixed
// quarter of the chunks, combined in a fixed order.
static __global__ __launch_bounds__(kThreads) void k_gram_reduce(const double* __restrict__ part,
                                                                 int nchunk, int ncx, int KZ,
                                                                 int nz, double* __restrict__ G,
                                                                 const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double lds[4][64];
    const int lo = threadIdx.x & 63, qd = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lo;
    double s = 0.0;
    if (o < ncx * nz) {
        const int c = o / nz, jz = o % nz;
        const int per = (nchunk + 3) / 4;
        const int ch0 = qd * per, ch1 = min(nchunk, ch0 + per);
        // even chunks into s0, odd ones into s1, each in chunk order; eight
        // chunks' loads are issued before their sums (the order of the
        // additions, and so the result, does not depend on the batching)
        const long long str = (long long)ncx * KZ;
        const double* pp = part + ((long long)ch0 * ncx + c) * KZ + jz;
        double s0 = 0.0, s1 = 0.0;
        int ch = ch0;
        for (; ch + 8 <= ch1; ch += 8, pp += 8 * str) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = pp[u * str];
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                s0 += a[u];
                s1 += a[u + 1];
            }
        }
        for (; ch + 1 < ch1; ch += 2, pp += 2 * str) {
            s0 += pp[0];
            s1 += pp[str];
        }
        if (ch < ch1) s0 += pp[0];
        s = s0 + s1;
    }
    lds[qd][lo] = s;
    __syncthreads();
    if (qd == 0 && o < ncx * nz) G[o] = (lds[0][lo] + lds[1][lo]) + (lds[2][lo] + lds[3][lo]);
}

// ---------------------------------------------------------------------------
// Block update (tall-skinny linear combination):
//   out[:, l] = base[:, l] + sum_{c < n2} V[:, c] * M[c * NOUT + l],  l < NOUT
// base has type TB (nullptr: zero).  base may alias out and out may alias
// columns of V: every thread reads all inputs of its points before writing.
// n2 may come from device memory (n2_dev) so a launch can cover a column count
// that is only known on the device.  Arithmetic in TA.  V is streamed with
// non-temporal loads and out written with non-temporal stores; consecutive
// point ranges go to the same XCD.  NORM: per-workgroup partial sum of
// out[:,0]^2 (FP64), indexed by point range.  UT threads per workgroup.
// ---------------------------------------------------------------------------
template <typename TV, typename TB, typename TO, typename TA, int NOUT, bool NORM, int UT>
__global__ __launch_bounds__(UT) void k_update(
    long long N, const TB* base, long long ldb, const TV* V, long long ldv, int n2,
    const int* __restrict__ n2_dev, const double* __restrict__ M, TO* out, long long ldo,
    double* __restrict__ part, const int* __restrict__ skip) {
    if (skip && *skip) return;
    static_assert(!NORM || UT == kThreads, "the norm partials use the 4-wave block sum");
    constexpr int PA = 16 / sizeof(TV), PB = 16 / sizeof(TB), PO = 16 / sizeof(TO);
    constexpr int PPT = PA > PB ? (PA > PO ? PA : PO) : (PB > PO ? PB : PO);
    const int nc = n2_dev ? *n2_dev : n2;
    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const long long p = ((long long)b * UT + threadIdx.x) * PPT;
    double nrm = 0.0;
    if (p + PPT <= N) {
        TA acc[NOUT][PPT];
#pragma unroll
        for (int l = 0; l < NOUT; ++l) {
            if (base) {
                TB t[PPT];
                load_pts<TB, PPT, false>(base + l * ldb + p, t);
#pragma unroll
                for (int e = 0; e < PPT; ++e) acc[l][e] = (TA)t[e];
            } else {
#pragma unroll
                for (int e = 0; e < PPT; ++e) acc[l][e] = TA(0);
            }
        }
        int c = 0;
        constexpr int UNR = 4;
        // software pipeline: the next UNR columns load while this batch's FMAs run
        TV vn[UNR][PPT];
        if (UNR <= nc) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) load_pts<TV, PPT, true>(V + (long long)u * ldv + p, vn[u]);
        }
        for (; c + UNR <= nc; c += UNR) {
            TV v[UNR][PPT];
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int e = 0; e < PPT; ++e) v[u][e] = vn[u][e];
            if (c + 2 * UNR <= nc) {
#pragma unroll
                for (int u = 0; u < UNR; ++u)
                    load_pts<TV, PPT, true>(V + (long long)(c + UNR + u) * ldv + p, vn[u]);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int l = 0; l < NOUT; ++l) {
                    const TA m = (TA)M[(c + u) * NOUT + l];
#pragma unroll
                    for (int e = 0; e < PPT; ++e) acc[l][e] = fma((TA)v[u][e], m, acc[l][e]);
                }
        }
        for (; c < nc; ++c) {
            TV v[PPT];
            load_pts<TV, PPT, true>(V + (long long)c * ldv + p, v);
#pragma unroll
            for (int l = 0; l < NOUT; ++l) {
                const TA m = (TA)M[c * NOUT + l];
#pragma unroll
                for (int e = 0; e < PPT; ++e) acc[l][e] = fma((TA)v[e], m, acc[l][e]);
            }
        }
#pragma unroll
        for (int l = 0; l < NOUT; ++l) {
            // stored straight from the accumulators: a local copy in between
            // lets the compiler drop the non-temporal bit when NOUT = 1
            if constexpr (std::is_same_v<TA, TO>) {
                store_pts_nt<TO, PPT>(out + l * ldo + p, acc[l]);
            } else {
                TO t[PPT];
#pragma unroll
                for (int e = 0; e < PPT; ++e) t[e] = (TO)acc[l][e];
                store_pts_nt<TO, PPT>(out + l * ldo + p, t);
            }
        }
        if (NORM) {
#pragma unroll
            for (int e = 0; e < PPT; ++e) nrm += (double)acc[0][e] * (double)acc[0][e];
        }
    } else if (p < N) {  // ragged tail: element by element
        for (long long q = p; q < N; ++q) {
            TA acc[NOUT];
#pragma unroll
            for (int l = 0; l < NOUT; ++l) acc[l] = base ? (TA)base[l * ldb + q] : TA(0);
            for (int c = 0; c < nc; ++c) {
                const TA v = (TA)V[(long long)c * ldv + q];
#pragma unroll
                for (int l = 0; l < NOUT; ++l) acc[l] = fma(v, (TA)M[c * NOUT + l], acc[l]);
            }
#pragma unroll
            for (int l = 0; l < NOUT; ++l) out[l * ldo + q] = (TO)acc[l];
            if (NORM) nrm += (double)acc[0] * (double)acc[0];
        }
    }
    if (NORM) {
        __shared__ double lds[4];
        double v1[1] = {nrm}, o[1];
        block_sum<1>(v1, lds, o);
        if (threadIdx.x == 0) part[b] = o[0];
    }
}

// Squared norm partials of an FP64 vector (one value per workgroup).
static __global__ __launch_bounds__(kThreads) void k_norm2(long long N, const double* __restrict__ v,
                                                           double* __restrict__ part) {
    __shared__ double lds[4];
    double s = 0.0;
    for (long long p = (long long)blockIdx.x * kThreads + threadIdx.x; p < N;
         p += (long long)gridDim.x * kThreads)
        s += v[p] * v[p];
    double v1[1] = {s}, o[1];
    block_sum<1>(v1, lds, o);
    if (threadIdx.x == 0) part[blockIdx.x] = o[0];
}

}  // namespace sstep
