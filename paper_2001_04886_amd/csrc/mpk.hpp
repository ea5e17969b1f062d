// mpk.hpp -- fused matrix-powers kernel: L levels of a 5-/7-point stencil in
// one pass over memory (the s directions of Sec. 3-4 from one vector).
//
// Each workgroup owns a tile of the grid "plane" (x-y in 3-D, x in 2-D): an
// exact interior of IX x IY points extended by a halo of L points on every
// side.  It marches along the slowest axis (z in 3-D, y in 2-D) over a chunk
// of planes extended by L planes on each side.  At step t the input plane t
// enters level 0; level j is then computed on plane t - j from level j-1.
// Every thread keeps, for each level, the three most recent planes of its own
// columns in registers (the neighbours along the march axis); the in-plane
// neighbours of level j-1 are exchanged through one plane of LDS.  Level j is
// exact on the tile shrunk by j, so after L levels the interior is exact; only
// interior points of the chunk's own planes are written.  HBM traffic per
// launch: the input read once (halos come from L2) and L output columns
// written.
//
// Level recurrence (per level j = 1..L, coefficients from the host):
//   y_j = alpha_j * A y_{j-1} + beta_j * y_{j-1} + gam_j * y_{j-2}
// with y_0 = in * in_scale and y_{-1} = prev * prev_scale (first level only).
//
// Memory operations carry no branches: every load and store is a raw buffer
// access whose out-of-range lanes read 0 and write nothing, and a plane
// outside the march range gets a resource of size 0.  With no branch around
// them the compiler can count the operations in flight exactly, so the next
// step's input plane, loaded one step ahead, and this step's stores stay in
// flight while the levels run (a branch makes it wait for all of them).
#pragma once

#include "kernels.hpp"

namespace sstep {

constexpr int kMpkMaxL = 8;

struct MpkLevels {
    double alpha[kMpkMaxL], beta[kMpkMaxL], gam[kMpkMaxL];
};

// Tile geometry.  The exact interior is 32 x 32 points in 3-D and a 256-point
// row segment in 2-D, so interiors tile power-of-two grids with no ragged
// tile and every stored row starts on a 256-byte boundary.  POS slots per
// thread; slots past the tile are idle.  PAD guard cells on each side of the
// LDS plane keep neighbour reads of edge slots inside the array (their
// values only reach halo points, which are never stored).
template <int DIM, int L>
struct MpkTile {
    static constexpr int IX = DIM == 3 ? 32 : 256, IY = DIM == 3 ? 32 : 1;
    static constexpr int PX = IX + 2 * L, PY = DIM == 3 ? IY + 2 * L : 1;
    static constexpr int NPOS = PX * PY;
    static constexpr int POS = DIM == 3 ? (L == 1 ? 2 : 3) : 1;
    static constexpr int THREADS = ((NPOS + POS - 1) / POS + 63) / 64 * 64;
    static constexpr int PAD = DIM == 3 ? PX : 1;
};

// Byte offset given to lanes that must not touch memory: beyond every plane
// (the host keeps plane sizes below 2^31 bytes).
constexpr unsigned kMpkOff = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mpk_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ T mpk_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Stores are nontemporal (cache policy bit nt): the output columns are not
// re-read by this launch, and streaming them past the caches raises the write
// bandwidth of the read-1 / write-L mix.
template <typename T>
__device__ __forceinline__ void mpk_st(T v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    constexpr int kNt = 2;
    if constexpr (sizeof(T) == 8) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, kNt);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, kNt);
    }
}

// VC: variable coefficients (A.coef, FP64 [7][N]); otherwise A.c.
template <typename T, int DIM, int L, bool VC>
__global__ __launch_bounds__((MpkTile<DIM, L>::THREADS)) void k_mpk_fused(
    StencilView A, T* __restrict__ out0, long long ldo, const T* __restrict__ in,
    const double* __restrict__ in_scale, const T* __restrict__ prev,
    const double* __restrict__ prev_scale, MpkLevels lv, int ntx, int nty, int zchunk,
    const int* __restrict__ skip) {
    if (skip && *skip) return;
    using G = MpkTile<DIM, L>;
    constexpr int PX = G::PX, IX = G::IX, IY = G::IY, NT = G::THREADS, POS = G::POS;
    constexpr int PAD = G::PAD, NSL = NT * POS + 2 * PAD;
    constexpr int NQ = 2 * DIM + 1;
    // two plane buffers used alternately by consecutive levels (also across
    // steps), so one barrier per level suffices
    __shared__ T plane[2][NSL];

    const int nx = A.nx, ny = A.ny;
    const int nmarch = (DIM == 3) ? A.nz : ny;
    const long long smarch = (DIM == 3) ? (long long)nx * ny : nx;
    const unsigned pbytes = (unsigned)(smarch * (long long)sizeof(T));
    const unsigned cbytes = (unsigned)(smarch * 8);

    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % ntx;
    const int ty = (b / ntx) % nty;
    const int zc = b / (ntx * nty);
    const int z0 = zc * zchunk;
    const int z1 = min(nmarch, z0 + zchunk);
    const int zs = z0 - L;
    const int nsteps = (z1 - z0) + 2 * L;

    // per slot: LDS index and the byte offsets of its point within a plane of
    // the input, the coefficient fields and the output (kMpkOff: no access)
    int ls[POS];
    bool inxy[POS];
    unsigned oin[POS], oout[POS], ocf[POS];
#pragma unroll
    for (int e = 0; e < POS; ++e) {
        const int slot = threadIdx.x + NT * e;
        const int px = slot % PX, py = slot / PX;
        const int gx = tx * IX - L + px;
        const int gy = (DIM == 3) ? ty * IY - L + py : 0;
        inxy[e] = slot < G::NPOS && gx >= 0 && gx < nx && (DIM == 2 || (gy >= 0 && gy < ny));
        const bool interior =
            px >= L && px < PX - L && (DIM == 2 || (py >= L && py < G::PY - L));
        const unsigned pt = (unsigned)gx + (unsigned)nx * (unsigned)gy;
        ls[e] = PAD + slot;
        oin[e] = inxy[e] ? pt * (unsigned)sizeof(T) : kMpkOff;
        oout[e] = (inxy[e] && interior) ? oin[e] : kMpkOff;
        ocf[e] = inxy[e] ? pt * 8u : kMpkOff;
    }

    T c[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) c[q] = (T)A.c[q];
    const T sin0 = in_scale ? (T)*in_scale : T(1);
    const T sprev = prev_scale ? (T)*prev_scale : T(1);
    const bool use_prev = prev != nullptr && lv.gam[0] != 0.0;
    const __amdgpu_buffer_rsrc_t none = mpk_rsrc(in, 0u);
    // resource of plane z of a T vector (empty outside the grid)
    auto plane_of = [&](const T* base, int z) {
        const bool ok = z >= 0 && z < nmarch;
        return mpk_rsrc(base + smarch * (ok ? z : 0), ok ? pbytes : 0u);
    };

    // levels 0..L-1, planes (z-1, z, z+1) of this thread's slots; level L is
    // only stored
    T ring[L][3][POS];
#pragma unroll
    for (int j = 0; j < L; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int e = 0; e < POS; ++e) ring[j][k][e] = T(0);

    // Step t's input plane enters ring[0] at the end of step t - 1, which then
    // issues the coefficient loads of step t and the input load of step t + 1
    // (loaded a step ahead).  With the loop rotated this way every path into
    // the loop head ends with the same loads in flight, so each wait counts
    // only what it needs (this step's stores stay in flight).
    T pre[POS], ppre[POS], pv1[POS];
    T cf[VC ? L : 1][VC ? NQ : 1][POS];
    auto advance = [&](int tn) {  // enter plane zs + tn; issue loads for steps tn, tn + 1
#pragma unroll
        for (int e = 0; e < POS; ++e) {
            T y0 = pre[e] * sin0;
            T ym = ppre[e] * sprev;  // y_{-1} on the plane level 1 computes at step tn
            // keep the products here: sunk to their first use, the loaded
            // values would stay live across the next loads, which then need
            // other registers and copies that wait for them
            asm volatile("" : "+v"(y0), "+v"(ym));
            ring[0][0][e] = ring[0][1][e];
            ring[0][1][e] = ring[0][2][e];
            ring[0][2][e] = y0;
            pv1[e] = ym;
        }
        if constexpr (VC) {
#pragma unroll
            for (int j = 1; j <= L; ++j) {
                const int zj = zs + tn - j;
                const bool ok = zj >= 0 && zj < nmarch;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const __amdgpu_buffer_rsrc_t rc =
                        mpk_rsrc(A.coef + q * A.N + smarch * (ok ? zj : 0), ok ? cbytes : 0u);
#pragma unroll
                    for (int e = 0; e < POS; ++e) cf[j - 1][q][e] = (T)mpk_ld<double>(rc, ocf[e]);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        const bool more = tn + 1 < nsteps;
        const __amdgpu_buffer_rsrc_t ri = more ? plane_of(in, zs + tn + 1) : none;
        const __amdgpu_buffer_rsrc_t rp = (more && use_prev) ? plane_of(prev, zs + tn) : none;
#pragma unroll
        for (int e = 0; e < POS; ++e) {
            pre[e] = mpk_ld<T>(ri, oin[e]);
            ppre[e] = mpk_ld<T>(rp, oin[e]);
        }
    };
    {
        const __amdgpu_buffer_rsrc_t ri = plane_of(in, zs);
        const __amdgpu_buffer_rsrc_t rp = use_prev ? plane_of(prev, zs - 1) : none;
#pragma unroll
        for (int e = 0; e < POS; ++e) {
            pre[e] = mpk_ld<T>(ri, oin[e]);
            ppre[e] = mpk_ld<T>(rp, oin[e]);
        }
    }
    advance(0);
    for (int t = 0; t < nsteps; ++t) {
#pragma unroll
        for (int j = 1; j <= L; ++j) {
            const int zj = zs + t - j;  // plane computed by level j at this step
            const bool zj_ok = zj >= 0 && zj < nmarch;
            T* buf = plane[(t * L + j) & 1];  // alternates across steps too
#pragma unroll
            for (int e = 0; e < POS; ++e) buf[ls[e]] = ring[j - 1][1][e];
            __syncthreads();
            T val[POS];
#pragma unroll
            for (int e = 0; e < POS; ++e) {
                T cc[7];
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    if constexpr (VC) cc[q] = q < NQ ? cf[j - 1][q < NQ ? q : 0][e] : T(0);
                    else cc[q] = c[q];
                }
                const int p = ls[e];
                const T ctr = ring[j - 1][1][e];
                // points outside the grid hold 0 at every level, so the
                // boundary terms vanish without tests
                T acc = T(0);
                acc += cc[1] * buf[p - 1];
                acc += cc[2] * buf[p + 1];
                if constexpr (DIM == 3) {
                    acc += cc[3] * buf[p - PX];
                    acc += cc[4] * buf[p + PX];
                    acc += cc[5] * ring[j - 1][0][e];
                    acc += cc[6] * ring[j - 1][2][e];
                } else {
                    acc += cc[3] * ring[j - 1][0][e];
                    acc += cc[4] * ring[j - 1][2][e];
                }
                acc += cc[0] * ctr;
                T v = (T)lv.alpha[j - 1] * acc;
                if (lv.beta[j - 1] != 0.0) v += (T)lv.beta[j - 1] * ctr;
                if (lv.gam[j - 1] != 0.0)
                    v += (T)lv.gam[j - 1] * (j == 1 ? pv1[e] : ring[j >= 2 ? j - 2 : 0][0][e]);
                val[e] = (inxy[e] && zj_ok) ? v : T(0);
            }
#pragma unroll
            for (int e = 0; e < POS; ++e) {
                if (j < L) {  // level j's ring (level L is only stored)
                    ring[j < L ? j : 0][0][e] = ring[j < L ? j : 0][1][e];
                    ring[j < L ? j : 0][1][e] = ring[j < L ? j : 0][2][e];
                    ring[j < L ? j : 0][2][e] = val[e];
                }
            }
            const bool own = zj >= z0 && zj < z1;
            const __amdgpu_buffer_rsrc_t ro =
                mpk_rsrc(out0 + (long long)(j - 1) * ldo + smarch * (own ? zj : 0),
                         own ? pbytes : 0u);
#pragma unroll
            for (int e = 0; e < POS; ++e) mpk_st<T>(val[e], ro, oout[e]);
        }
        advance(t + 1);  // also after the last step (empty loads): no branch
    }
}

}  // namespace sstep
