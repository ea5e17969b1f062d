// mpk3d.hpp -- fused matrix powers of a constant-coefficient 7-point stencil
// on a 3-D grid (the s directions of Sec. 3-4 from one vector): L levels per
// pass over memory, with the tile's in-plane neighbours held in registers.
//
// Tile: 64 points along x (one per lane of a wave; lanes L..63-L are exact
// after L levels) times W*POS rows along y (each wave owns POS consecutive
// rows; rows L..W*POS-1-L are exact).  The workgroup marches along z over a
// chunk of planes extended by L planes on either side; at step t the input
// plane t enters level 0 and level j is computed on plane t - j from three
// planes of level j - 1 kept in a per-level ring of registers.  Neighbours:
//   x +- 1 : the same register of the adjacent lane (whole-wave DPP shift;
//            lanes 0 and 63 receive 0, they are halo lanes),
//   y +- 1 : the thread's own registers, except above the wave's first and
//            below its last row: those two rows are exchanged between
//            neighbouring waves through LDS (one barrier per level),
//   z +- 1 : the ring.
// The step loop is unrolled by three so the ring rotates by renaming
// registers.  A level runs only on the planes a later level or the output
// needs (planes z0 - (L - j) .. z1 - 1 + (L - j)); planes outside the grid
// are zero.  With the same scale on every level (monomial and Newton bases)
// the scale carries the out-of-grid mask (alpha or 0 per row).  Loads and
// stores are raw buffer accesses whose out-of-range lanes read 0 / write
// nothing, with no branch around them; the next input plane is loaded one
// step ahead; stores are nontemporal.  HBM traffic per launch: the input
// read once (the x-y halo of a tile comes mostly from the caches) and L
// output columns written.
//
// Level recurrence (as in mpk.hpp):
//   y_j = alpha_j A y_{j-1} + beta_j y_{j-1} + gam_j y_{j-2},
// y_0 = in * in_scale, y_{-1} = prev * prev_scale (first level only, PREV).
#pragma once

#include <type_traits>

#include "mpk.hpp"

namespace sstep {

template <int L, int POS, int W>
struct Mpk3Tile {
    static constexpr int IX = 64 - 2 * L;   // exact interior along x
    static constexpr int PY = W * POS;      // rows of the tile, halo included
    static constexpr int IY = PY - 2 * L;   // exact interior along y
    static constexpr int THREADS = 64 * W;
};

// Value of the same register in lane l - 1 / lane l + 1 (whole-wave DPP shift;
// lanes 0 / 63, which have no source, receive 0 -- they are halo lanes, whose
// value is never needed).
template <int CTRL, typename T>
__device__ __forceinline__ T mpk3_lane_shift(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
        const unsigned slo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, true);
        const unsigned shi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, true);
        return __builtin_bit_cast(T, ((unsigned long long)shi << 32) | slo);
    } else {
        const unsigned u = __builtin_bit_cast(unsigned, v);
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(u, u, CTRL, 0xf, 0xf, true));
    }
}
template <typename T>
__device__ __forceinline__ T mpk3_lane_below(T v) { return mpk3_lane_shift<0x138>(v); }
template <typename T>
__device__ __forceinline__ T mpk3_lane_above(T v) { return mpk3_lane_shift<0x130>(v); }

// PREV: the first level reads y_{-1} (three-term recurrence continued from an
// earlier pass).  UNI: every level has the same alpha.  BETA / GAM: some level
// has a beta / gamma term (without them the terms are not compiled in: the
// monomial basis has neither, the Newton basis only beta).
template <typename T, int L, int POS, int W, bool PREV, bool UNI, bool BETA, bool GAM>
__global__ __launch_bounds__(64 * W) void k_mpk3d(
    StencilView A, T* __restrict__ out0, long long ldo, const T* __restrict__ in,
    const double* __restrict__ in_scale, const T* __restrict__ prev,
    const double* __restrict__ prev_scale, MpkLevels lv, int ntx, int nty, int zchunk,
    const int* __restrict__ skip) {
    if (skip && *skip) return;
    using G = Mpk3Tile<L, POS, W>;
    constexpr int IX = G::IX, IY = G::IY, PY = G::PY;
    // first and last row of every wave, [buffer][wave + 1][first, last][lane];
    // slots 0 and W + 1 stay zero (what they feed is halo only)
    __shared__ T xch[2][W + 2][2][64];

    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const long long splane = (long long)nx * ny;
    const unsigned pbytes = (unsigned)(splane * (long long)sizeof(T));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % ntx;
    const int ty = (b / ntx) % nty;
    const int zc = b / (ntx * nty);
    const int z0 = zc * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int zs = z0 - L;
    const int nsteps = (z1 - z0) + 2 * L;

    for (int i = threadIdx.x; i < 2 * 2 * 64; i += 64 * W) {
        const int bb = i / 128, e = (i / 64) & 1, l = i & 63;
        xch[bb][0][e][l] = T(0);
        xch[bb][W + 1][e][l] = T(0);
    }

    // per row: inside the grid, byte offset within a plane of the input and
    // of the output (kMpkOff: no access; only the exact interior is stored)
    const int gx = tx * IX - L + lane;
    const bool inx = gx >= 0 && gx < nx;
    const bool intx = lane >= L && lane < 64 - L;
    bool inxy[POS];
    unsigned oin[POS], oout[POS];
    T arow[UNI ? POS : 1];
#pragma unroll
    for (int r = 0; r < POS; ++r) {
        const int row = w * POS + r;
        const int gy = ty * IY - L + row;
        inxy[r] = inx && gy >= 0 && gy < ny;
        const bool interior = intx && row >= L && row < PY - L;
        const unsigned pt = (unsigned)gx + (unsigned)nx * (unsigned)gy;
        oin[r] = inxy[r] ? pt * (unsigned)sizeof(T) : kMpkOff;
        oout[r] = (inxy[r] && interior) ? oin[r] : kMpkOff;
        if constexpr (UNI) arow[r] = inxy[r] ? (T)lv.alpha[0] : T(0);
    }

    const T c0 = (T)A.c[0], c1 = (T)A.c[1], c2 = (T)A.c[2], c3 = (T)A.c[3], c4 = (T)A.c[4],
            c5 = (T)A.c[5], c6 = (T)A.c[6];
    const T sin0 = in_scale ? (T)*in_scale : T(1);
    const T sprev = prev_scale ? (T)*prev_scale : T(1);
    const __amdgpu_buffer_rsrc_t none = mpk_rsrc(in, 0u);
    auto plane_of = [&](const T* base, int z) {
        const bool ok = z >= 0 && z < nz;
        return mpk_rsrc(base + splane * (ok ? z : 0), ok ? pbytes : 0u);
    };

    // ring[j][slot][row]: three planes of level j (levels 0..L-1; level L is
    // only stored).  At step t, plane k of the ring (0: z - 1, 1: z, 2: z + 1
    // around the plane level j + 1 computes) sits in slot (t + k) mod 3.
    T ring[L][3][POS];
#pragma unroll
    for (int j = 0; j < L; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int r = 0; r < POS; ++r) ring[j][k][r] = T(0);

    T pre[POS];
    T ppre[PREV ? POS : 1], pv1[PREV ? POS : 1];
    // plane zs + tn enters level 0 in slot Q = (tn + 2) mod 3, then the loads
    // of step tn + 1 are issued
    auto advance = [&](auto Q, int tn) {
        constexpr int q = decltype(Q)::value;
#pragma unroll
        for (int r = 0; r < POS; ++r) {
            T y0 = pre[r] * sin0;
            // keep the product here: sunk to its use, the loaded value would
            // stay live across the next loads
            asm volatile("" : "+v"(y0));
            ring[0][q][r] = y0;
            if constexpr (PREV) {
                T ym = ppre[r] * sprev;
                asm volatile("" : "+v"(ym));
                pv1[r] = ym;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        const bool more = tn + 1 < nsteps;
        const __amdgpu_buffer_rsrc_t ri = more ? plane_of(in, zs + tn + 1) : none;
#pragma unroll
        for (int r = 0; r < POS; ++r) pre[r] = mpk_ld<T>(ri, oin[r]);
        if constexpr (PREV) {
            const __amdgpu_buffer_rsrc_t rp = more ? plane_of(prev, zs + tn) : none;
#pragma unroll
            for (int r = 0; r < POS; ++r) ppre[r] = mpk_ld<T>(rp, oin[r]);
        }
    };

    int nbar = 0;  // barriers passed: the exchange buffers alternate per barrier
    auto step = [&](auto RHO, int t) {
        constexpr int rho = decltype(RHO)::value;
        constexpr int P0 = rho % 3, P1 = (rho + 1) % 3, P2 = (rho + 2) % 3;
#pragma unroll
        for (int j = 1; j <= L; ++j) {
            const int zj = zs + t - j;  // plane level j computes at this step
            if (zj < z0 - (L - j) || zj > z1 - 1 + (L - j)) continue;  // not needed
            if (zj < 0 || zj >= nz) {  // outside the grid: zero
                if (j < L) {
#pragma unroll
                    for (int r = 0; r < POS; ++r) ring[j < L ? j : 0][P2][r] = T(0);
                }
                continue;
            }
            const int bf = (nbar++) & 1;
            xch[bf][w + 1][0][lane] = ring[j - 1][P1][0];
            xch[bf][w + 1][1][lane] = ring[j - 1][P1][POS - 1];
            __syncthreads();
            const T up = xch[bf][w][1][lane];      // the row before the wave's first
            const T dn = xch[bf][w + 2][0][lane];  // the row after the wave's last
            T val[POS];
#pragma unroll
            for (int r = 0; r < POS; ++r) {
                const T ctr = ring[j - 1][P1][r];
                const T ym = r == 0 ? up : ring[j - 1][P1][r > 0 ? r - 1 : 0];
                const T yp = r == POS - 1 ? dn : ring[j - 1][P1][r < POS - 1 ? r + 1 : 0];
                // neighbour order -x, +x, -y, +y, -z, +z, then the centre
                T acc = T(0);
                acc += c1 * mpk3_lane_below(ctr);
                acc += c2 * mpk3_lane_above(ctr);
                acc += c3 * ym;
                acc += c4 * yp;
                acc += c5 * ring[j - 1][P0][r];
                acc += c6 * ring[j - 1][P2][r];
                acc += c0 * ctr;
                T v;
                if constexpr (UNI) v = arow[r] * acc;
                else v = (T)lv.alpha[j - 1] * acc;
                if constexpr (BETA) v += (T)lv.beta[j - 1] * ctr;
                if constexpr (GAM) {
                    if (j >= 2) v += (T)lv.gam[j - 1] * ring[j >= 2 ? j - 2 : 0][P0][r];
                    else if constexpr (PREV) v += (T)lv.gam[j - 1] * pv1[r];
                }
                if constexpr (UNI) val[r] = v;
                else val[r] = inxy[r] ? v : T(0);
            }
            if (j < L) {
#pragma unroll
                for (int r = 0; r < POS; ++r) ring[j < L ? j : 0][P2][r] = val[r];
            }
            const bool own = zj >= z0 && zj < z1;
            const __amdgpu_buffer_rsrc_t ro = mpk_rsrc(
                out0 + (long long)(j - 1) * ldo + splane * (own ? zj : 0), own ? pbytes : 0u);
#pragma unroll
            for (int r = 0; r < POS; ++r) mpk_st<T>(val[r], ro, oout[r]);
        }
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    {
        const __amdgpu_buffer_rsrc_t ri = plane_of(in, zs);
#pragma unroll
        for (int r = 0; r < POS; ++r) pre[r] = mpk_ld<T>(ri, oin[r]);
        if constexpr (PREV) {
            const __amdgpu_buffer_rsrc_t rp = plane_of(prev, zs - 1);
#pragma unroll
            for (int r = 0; r < POS; ++r) ppre[r] = mpk_ld<T>(rp, oin[r]);
        }
    }
    __syncthreads();  // zeroed exchange slots visible to every wave
    advance(I2{}, 0);
    int t = 0;
    for (; t + 3 <= nsteps; t += 3) {
        step(I0{}, t);
        advance(I0{}, t + 1);
        step(I1{}, t + 1);
        advance(I1{}, t + 2);
        step(I2{}, t + 2);
        advance(I2{}, t + 3);
    }
    if (t < nsteps) {
        step(I0{}, t);
        advance(I0{}, t + 1);
        if (t + 1 < nsteps) {
            step(I1{}, t + 1);
            advance(I1{}, t + 2);
        }
    }
}

}  // namespace sstep
