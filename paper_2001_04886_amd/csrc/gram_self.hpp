// gram_self.hpp -- the Gram matrix of a block with itself, X^T X for up to
// NC columns, in one pass: each point's NC values are loaded once and all
// NC (NC + 1) / 2 products of the upper triangle are accumulated.  This is the
// block's own Gram of s-step GMRES (W_k and V_k^T Yhat_s, Sec. 4, eqs. 6-7),
// which the general tiled kernel would otherwise stream CA columns at a time
// (re-reading the block once per tile).  Partials use the layout of
// k_gram_partial (full, mirrored matrix per chunk) so k_gram_reduce finishes it.
#pragma once

#include "kernels.hpp"

namespace sstep {

template <typename T, int NC>
__global__ __launch_bounds__(kThreads) void k_gram_self(const T* __restrict__ X, long long ldx,
                                                        int nc, long long N, long long chunk,
                                                        int KZ, double* __restrict__ part,
                                                        const int* __restrict__ skip) {
    if (skip && *skip) return;
    constexpr int PPT = 16 / sizeof(T);  // points per thread per step (one 16-byte load)
    constexpr int STEP = PPT * kThreads;
    constexpr int NP = NC * (NC + 1) / 2;
    __shared__ double lds[4][NP];
    __shared__ double tot[NP];
    const long long ch = xcd_remap(blockIdx.x, gridDim.x);
    const long long p0 = ch * chunk;
    const long long p1 = (p0 + chunk < N) ? p0 + chunk : N;
    // columns beyond nc alias the last one; their sums are discarded
    const T* xc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) xc[a] = X + (long long)(a < nc ? a : nc - 1) * ldx;
    double acc[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = 0.0;

    // full vectors (chunk starts are multiples of 512 points), next step's
    // loads in flight during this step's products
    const long long pv1 = p0 + (p1 - p0) / PPT * PPT;
    long long p = p0 + (long long)PPT * threadIdx.x;
    T xn[NC][PPT];
    if (p < pv1) {
#pragma unroll
        for (int a = 0; a < NC; ++a) load_pts<T, PPT, true>(xc[a] + p, xn[a]);
    }
    for (; p < pv1; p += STEP) {
        T xv[NC][PPT];
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int e = 0; e < PPT; ++e) xv[a][e] = xn[a][e];
        const long long pn = p + STEP;
        if (pn < pv1) {
#pragma unroll
            for (int a = 0; a < NC; ++a) load_pts<T, PPT, true>(xc[a] + pn, xn[a]);
        }
        int k = 0;
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = a; b < NC; ++b, ++k)
#pragma unroll
                for (int e = 0; e < PPT; ++e)
                    acc[k] = fma((double)xv[a][e], (double)xv[b][e], acc[k]);
    }
    for (long long q = pv1 + threadIdx.x; q < p1; q += kThreads) {  // ragged tail
        double x0[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) x0[a] = to_f64(xc[a][q]);
        int k = 0;
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = a; b < NC; ++b, ++k) acc[k] = fma(x0[a], x0[b], acc[k]);
    }
    // workgroup sums (wave shuffles, then four wave partials in a fixed order)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double t = wave_sum(acc[k]);
        if (lane == 0) lds[wave][k] = t;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NP; k += kThreads)
        tot[k] = (lds[0][k] + lds[1][k]) + (lds[2][k] + lds[3][k]);
    __syncthreads();
    // full matrix, mirrored: entry (a, b) is product k(min, max)
    for (int o = threadIdx.x; o < nc * nc; o += kThreads) {
        const int a = o / nc, b = o % nc;
        const int i = a < b ? a : b, j = a < b ? b : a;
        const int k = i * NC - i * (i - 1) / 2 + (j - i);
        part[(ch * nc + a) * KZ + b] = tot[k];
    }
}

}  // namespace sstep
