/* cnn_oracle.c -- plain FP64 CPU reference of the convolution layers used by
 * the learned initial-guess network (x0 = CNN(log k, f)).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): nothing in the GPU
 * library links or calls this file.
 *
 * The paper's s-step GMRES (Alg 4.2) accepts any starting vector x0; the
 * network that proposes one is an extension beyond the paper, so these
 * routines follow the textbook definitions of a dilated 3x3 convolution
 * (cross-correlation, zero padding equal to the dilation, output the size of
 * the input) and of its two adjoints.  Layout NCHW, row index i (y), column
 * index j (x), tap (ty, tx) in {0,1,2}^2 reads the input at
 * (i + (ty-1) d, j + (tx-1) d).  Every sum runs in index order, one term at a
 * time, with no blocking.
 */
#include <stddef.h>

static double at(const double* x, int H, int W, int i, int j) {
    if (i < 0 || i >= H || j < 0 || j >= W) return 0.0;
    return x[(size_t)i * W + j];
}

/* y[b][co] = bias[co] + sum_ci sum_tap w[co][ci][tap] x[b][ci](shifted) */
void cnn_conv_fwd(const double* x, int B, int Cin, int H, int W, const double* w,
                  const double* bias, int Cout, int d, double* y) {
    const size_t hw = (size_t)H * W;
    for (int b = 0; b < B; ++b)
        for (int co = 0; co < Cout; ++co)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j) {
                    double acc = bias ? bias[co] : 0.0;
                    for (int ci = 0; ci < Cin; ++ci) {
                        const double* xp = x + ((size_t)b * Cin + ci) * hw;
                        for (int ty = 0; ty < 3; ++ty)
                            for (int tx = 0; tx < 3; ++tx)
                                acc += w[(((size_t)co * Cin + ci) * 3 + ty) * 3 + tx] *
                                       at(xp, H, W, i + (ty - 1) * d, j + (tx - 1) * d);
                    }
                    y[((size_t)b * Cout + co) * hw + (size_t)i * W + j] = acc;
                }
}

/* Adjoint of cnn_conv_fwd in x (bias-free part):
 * dx[b][ci](i,j) = sum_co sum_tap w[co][ci][tap] dy[b][co](i - (ty-1)d, j - (tx-1)d) */
void cnn_conv_bwd_data(const double* dy, int B, int Cout, int H, int W, const double* w,
                       int Cin, int d, double* dx) {
    const size_t hw = (size_t)H * W;
    for (int b = 0; b < B; ++b)
        for (int ci = 0; ci < Cin; ++ci)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j) {
                    double acc = 0.0;
                    for (int co = 0; co < Cout; ++co) {
                        const double* gp = dy + ((size_t)b * Cout + co) * hw;
                        for (int ty = 0; ty < 3; ++ty)
                            for (int tx = 0; tx < 3; ++tx)
                                acc += w[(((size_t)co * Cin + ci) * 3 + ty) * 3 + tx] *
                                       at(gp, H, W, i - (ty - 1) * d, j - (tx - 1) * d);
                    }
                    dx[((size_t)b * Cin + ci) * hw + (size_t)i * W + j] = acc;
                }
}

/* Gradient of <dy, cnn_conv_fwd(x)> in w and bias:
 * dw[co][ci][tap] = sum_b sum_(i,j) dy[b][co](i,j) x[b][ci](i + (ty-1)d, j + (tx-1)d)
 * db[co]          = sum_b sum_(i,j) dy[b][co](i,j) */
void cnn_conv_bwd_weight(const double* x, const double* dy, int B, int Cin, int Cout, int H,
                         int W, int d, double* dw, double* db) {
    const size_t hw = (size_t)H * W;
    for (int co = 0; co < Cout; ++co) {
        for (int ci = 0; ci < Cin; ++ci)
            for (int ty = 0; ty < 3; ++ty)
                for (int tx = 0; tx < 3; ++tx) {
                    double acc = 0.0;
                    for (int b = 0; b < B; ++b) {
                        const double* gp = dy + ((size_t)b * Cout + co) * hw;
                        const double* xp = x + ((size_t)b * Cin + ci) * hw;
                        for (int i = 0; i < H; ++i)
                            for (int j = 0; j < W; ++j)
                                acc += gp[(size_t)i * W + j] *
                                       at(xp, H, W, i + (ty - 1) * d, j + (tx - 1) * d);
                    }
                    dw[(((size_t)co * Cin + ci) * 3 + ty) * 3 + tx] = acc;
                }
        if (db) {
            double acc = 0.0;
            for (int b = 0; b < B; ++b) {
                const double* gp = dy + ((size_t)b * Cout + co) * hw;
                for (size_t p = 0; p < hw; ++p) acc += gp[p];
            }
            db[co] = acc;
        }
    }
}
