// mpk.hpp -- fused matrix-powers kernel: L levels of a 5-/7-point stencil in
// one pass over memory (the s directions of Sec. 3-4 from one vector).
//
// Each workgroup owns a tile of the grid "plane" (x-y in 3-D, x in 2-D)
// extended by a halo of L points on every side, and marches along the slowest
// axis (z in 3-D, y in 2-D) over a chunk of planes extended by L planes on
// each side.  At step t the input plane t enters level 0; level j is then
// computed on plane t - j from level j-1.  Every thread keeps, for each level,
// the three most recent planes of its own column in registers (the
// neighbours along the march axis); the in-plane neighbours of level j-1 are
// exchanged through one plane of LDS.  Level j is exact on the tile shrunk by
// j, so after L levels the tile interior is exact; only interior points of
// the chunk's own planes are written.  HBM traffic per launch: the input read
// once (halos come from L2) and L output columns written.
//
// Level recurrence (per level j = 1..L, coefficients from the host):
//   y_j = alpha_j * A y_{j-1} + beta_j * y_{j-1} + gam_j * y_{j-2}
// with y_0 = in * in_scale and y_{-1} = prev * prev_scale (first level only).
#pragma once

#include "kernels.hpp"

namespace sstep {

constexpr int kMpkMaxL = 8;

struct MpkLevels {
    double alpha[kMpkMaxL], beta[kMpkMaxL], gam[kMpkMaxL];
};

// Plane tile: 32 x 32 in 3-D, a 256-point row segment in 2-D; POS positions
// per thread.
template <int DIM, int POS_>
struct MpkTile {
    static constexpr int PX = DIM == 3 ? 32 : 256, PY = DIM == 3 ? 32 : 1;
    static constexpr int POS = POS_, THREADS = PX * PY / POS_;
};

template <typename T, int DIM, int L, int POSN>
__global__ __launch_bounds__((MpkTile<DIM, POSN>::THREADS)) void k_mpk_fused(
    StencilView A, T* __restrict__ out0, long long ldo, const T* __restrict__ in,
    const double* __restrict__ in_scale, const T* __restrict__ prev,
    const double* __restrict__ prev_scale, MpkLevels lv, int ntx, int nty, int zchunk,
    const int* __restrict__ skip) {
    if (skip && *skip) return;
    constexpr int PX = MpkTile<DIM, POSN>::PX, PY = MpkTile<DIM, POSN>::PY;
    constexpr int NT = MpkTile<DIM, POSN>::THREADS, POS = POSN;
    constexpr int IX = PX - 2 * L, IY = (DIM == 3) ? PY - 2 * L : 1;
    // two plane buffers used alternately by consecutive levels (also across
    // steps), so one barrier per level suffices
    __shared__ T plane[2][PX * PY];

    const int nx = A.nx, ny = A.ny;
    const int nmarch = (DIM == 3) ? A.nz : ny;
    const long long smarch = (DIM == 3) ? (long long)nx * ny : nx;

    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % ntx;
    const int ty = (b / ntx) % nty;
    const int zc = b / (ntx * nty);
    const int z0 = zc * zchunk;
    const int z1 = min(nmarch, z0 + zchunk);
    const int zs = z0 - L;
    const int nsteps = (z1 - z0) + 2 * L;

    int pos[POS], px[POS], gx[POS], gy[POS];
    bool inxy[POS], interior[POS];
    long long pxy[POS];
#pragma unroll
    for (int e = 0; e < POS; ++e) {
        pos[e] = threadIdx.x + NT * e;
        px[e] = pos[e] % PX;
        const int py = pos[e] / PX;
        gx[e] = tx * IX - L + px[e];
        gy[e] = (DIM == 3) ? ty * IY - L + py : 0;
        inxy[e] = gx[e] >= 0 && gx[e] < nx && (DIM == 2 || (gy[e] >= 0 && gy[e] < ny));
        interior[e] = px[e] >= L && px[e] < PX - L && (DIM == 2 || (py >= L && py < PY - L));
        pxy[e] = (DIM == 3) ? (long long)gx[e] + (long long)nx * gy[e] : gx[e];
    }

    T c[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) c[q] = (T)A.c[q];
    const T sin0 = in_scale ? (T)*in_scale : T(1);
    const T sprev = prev_scale ? (T)*prev_scale : T(1);

    T ring[L + 1][3][POS];
#pragma unroll
    for (int j = 0; j <= L; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int e = 0; e < POS; ++e) ring[j][k][e] = T(0);

    for (int t = 0; t < nsteps; ++t) {
        const int zl = zs + t;  // level 0 enters this plane
        const bool zl_ok = zl >= 0 && zl < nmarch;
#pragma unroll
        for (int e = 0; e < POS; ++e) {
            ring[0][0][e] = ring[0][1][e];
            ring[0][1][e] = ring[0][2][e];
            ring[0][2][e] = (inxy[e] && zl_ok) ? in[pxy[e] + smarch * zl] * sin0 : T(0);
        }
#pragma unroll
        for (int j = 1; j <= L; ++j) {
            const int zj = zs + t - j;  // plane computed by level j at this step
            const bool zj_ok = zj >= 0 && zj < nmarch;
            T* buf = plane[(t * L + j) & 1];  // alternates across steps too
#pragma unroll
            for (int e = 0; e < POS; ++e) buf[pos[e]] = ring[j - 1][1][e];
            __syncthreads();
            T val[POS];
#pragma unroll
            for (int e = 0; e < POS; ++e) {
                val[e] = T(0);
                if (inxy[e] && zj_ok) {
                    const T ctr = ring[j - 1][1][e];
                    T cc[7];
                    if (A.coef) {
                        const long long p = pxy[e] + smarch * zj;
#pragma unroll
                        for (int q = 0; q < 7; ++q)
                            cc[q] = (q < 2 * DIM + 1) ? (T)A.coef[q * A.N + p] : T(0);
                    } else {
#pragma unroll
                        for (int q = 0; q < 7; ++q) cc[q] = c[q];
                    }
                    const int ps = pos[e];
                    T acc = T(0);
                    if (px[e] > 0 && gx[e] > 0) acc += cc[1] * buf[ps - 1];
                    if (px[e] < PX - 1 && gx[e] < nx - 1) acc += cc[2] * buf[ps + 1];
                    if (DIM == 3) {
                        if (ps >= PX && gy[e] > 0) acc += cc[3] * buf[ps - PX];
                        if (ps < PX * (PY - 1) && gy[e] < ny - 1) acc += cc[4] * buf[ps + PX];
                        acc += cc[5] * ring[j - 1][0][e];
                        acc += cc[6] * ring[j - 1][2][e];
                    } else {
                        acc += cc[3] * ring[j - 1][0][e];
                        acc += cc[4] * ring[j - 1][2][e];
                    }
                    acc += cc[0] * ctr;
                    T v = (T)lv.alpha[j - 1] * acc;
                    if (lv.beta[j - 1] != 0.0) v += (T)lv.beta[j - 1] * ctr;
                    if (lv.gam[j - 1] != 0.0) {
                        const T pv = (j == 1) ? (prev ? prev[pxy[e] + smarch * zj] * sprev : T(0))
                                              : ring[j - 2 > 0 ? j - 2 : 0][0][e];
                        v += (T)lv.gam[j - 1] * pv;
                    }
                    val[e] = v;
                }
            }
#pragma unroll
            for (int e = 0; e < POS; ++e) {
                ring[j][0][e] = ring[j][1][e];
                ring[j][1][e] = ring[j][2][e];
                ring[j][2][e] = val[e];
                if (interior[e] && inxy[e] && zj >= z0 && zj < z1)
                    out0[(j - 1) * ldo + pxy[e] + smarch * zj] = val[e];
            }
        }
    }
}

}  // namespace sstep
