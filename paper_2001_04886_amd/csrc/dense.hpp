// dense.hpp -- small FP64 dense kernels run on the device by one thread
// (the s x s "Scalar1 / Scalar2" work of Sec. 3-4: decompose the Gram matrix
// of a block and solve with it).
#pragma once

#include <hip/hip_runtime.h>

namespace sstep {

constexpr int kMaxS = 16;

// Factor of a symmetric positive semi-definite s x s Gram matrix W:
// S = diag(W_ii)^(-1/2), U upper triangular with U^T U = S W S on the leading
// rank x rank part.  The factorisation stops at the first pivot (of the
// unit-diagonal matrix S W S) not above rank_tol: the columns from there on
// are numerically dependent on the earlier ones.
struct GramFactor {
    double U[kMaxS * kMaxS];  // column-major, leading dimension kMaxS
    double sc[kMaxS];
    int n;
    int rank;
};

__device__ inline void gram_factor(const double* W, int ldw, int n, double rank_tol,
                                   GramFactor* F) {
    F->n = n;
    F->rank = n;
    for (int i = 0; i < n; ++i) {
        const double d = W[i + i * ldw];
        F->sc[i] = d > 0.0 ? rsqrt(d) : 0.0;
    }
    for (int jc = 0; jc < n; ++jc) {
        if (F->sc[jc] == 0.0) { F->rank = jc; return; }
        double diag = W[jc + jc * ldw] * F->sc[jc] * F->sc[jc];
        for (int ir = 0; ir < jc; ++ir) {
            double v = W[ir + jc * ldw] * F->sc[ir] * F->sc[jc];
            for (int k = 0; k < ir; ++k) v -= F->U[k + ir * kMaxS] * F->U[k + jc * kMaxS];
            v /= F->U[ir + ir * kMaxS];
            F->U[ir + jc * kMaxS] = v;
            diag -= v * v;
        }
        if (!(diag > rank_tol)) { F->rank = jc; return; }
        F->U[jc + jc * kMaxS] = sqrt(diag);
        for (int ir = jc + 1; ir < n; ++ir) F->U[ir + jc * kMaxS] = 0.0;
    }
}

// gram_factor for a workgroup of one wave, in LDS: W (symmetric, ld kMaxS,
// overwritten) and F are shared.  The elimination runs column by column of U
// with the trailing updates spread over the lanes; every entry sees the same
// floating-point operations in the same order as in gram_factor (scaling,
// then the subtractions U_ki U_kj for k = 0, 1, ..., then the division or the
// square root), so F is identical on its leading rank x rank part and on
// column `rank` above the diagonal.  All lanes must call it.
__device__ inline void gram_factor_wave(double* W, int n, double rank_tol, GramFactor* F) {
    const int lane = threadIdx.x;
    if (lane == 0) {
        F->n = n;
        F->rank = n;
    }
    for (int i = lane; i < n; i += 64) {
        const double d = W[i + i * kMaxS];
        F->sc[i] = d > 0.0 ? rsqrt(d) : 0.0;
    }
    __syncthreads();
    // scaled upper triangle
    for (int idx = lane; idx < n * n; idx += 64) {
        const int i = idx % n, j = idx / n;
        if (i <= j) W[i + j * kMaxS] = W[i + j * kMaxS] * F->sc[i] * F->sc[j];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // pivot k (uniform decision)
        if (F->sc[k] == 0.0 || !(W[k + k * kMaxS] > rank_tol)) {
            __syncthreads();
            if (lane == 0) F->rank = k;
            return;
        }
        const double piv = sqrt(W[k + k * kMaxS]);
        for (int j = k + 1 + lane; j < n; j += 64) F->U[k + j * kMaxS] = W[k + j * kMaxS] / piv;
        for (int i = k + 1 + lane; i < n; i += 64) F->U[i + k * kMaxS] = 0.0;
        if (lane == 0) F->U[k + k * kMaxS] = piv;
        __syncthreads();
        // trailing update of the upper triangle: entries (i, j), k < i <= j
        const int m = n - 1 - k;
        for (int idx = lane; idx < m * m; idx += 64) {
            const int i = k + 1 + idx % m, j = k + 1 + idx / m;
            if (i <= j) {
                double v = W[i + j * kMaxS];
                v -= F->U[k + i * kMaxS] * F->U[k + j * kMaxS];
                W[i + j * kMaxS] = v;
            }
        }
        __syncthreads();
    }
}

// z = W^{-1} b on the leading rank x rank part; z[rank..n) = 0.  b, z may alias.
__device__ inline void gram_solve(const GramFactor& F, const double* b, double* z) {
    double u[kMaxS];
    const int q = F.rank;
    for (int i = 0; i < q; ++i) {  // U^T u = S b
        double v = b[i] * F.sc[i];
        for (int k = 0; k < i; ++k) v -= F.U[k + i * kMaxS] * u[k];
        u[i] = v / F.U[i + i * kMaxS];
    }
    for (int i = q - 1; i >= 0; --i) {  // U w = u
        double v = u[i];
        for (int k = i + 1; k < q; ++k) v -= F.U[i + k * kMaxS] * u[k];
        u[i] = v / F.U[i + i * kMaxS];
    }
    for (int i = 0; i < q; ++i) z[i] = u[i] * F.sc[i];
    for (int i = q; i < F.n; ++i) z[i] = 0.0;
}

// Same solve restricted to the leading m x m part (m <= rank).
__device__ inline void gram_solve_leading(const GramFactor& F, int m, const double* b, double* z) {
    double u[kMaxS];
    for (int i = 0; i < m; ++i) {
        double v = b[i] * F.sc[i];
        for (int k = 0; k < i; ++k) v -= F.U[k + i * kMaxS] * u[k];
        u[i] = v / F.U[i + i * kMaxS];
    }
    for (int i = m - 1; i >= 0; --i) {
        double v = u[i];
        for (int k = i + 1; k < m; ++k) v -= F.U[i + k * kMaxS] * u[k];
        u[i] = v / F.U[i + i * kMaxS];
    }
    for (int i = 0; i < m; ++i) z[i] = u[i] * F.sc[i];
}

// Entry (a, b) of the upper Cholesky factor L of W itself (L^T L = W):
// L = U S^{-1}.
__device__ inline double gram_L(const GramFactor& F, int a, int b) {
    return F.U[a + b * kMaxS] / F.sc[b];
}

}  // namespace sstep
