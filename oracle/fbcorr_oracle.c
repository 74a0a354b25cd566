/*
 * Plain FP64 CPU oracle for the multi-channel 2-D filter-bank correlation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the library never does.  It
 * shares no code, header or constant with the GPU path.
 *
 * The operation is the "3D filter-bank convolution" of the Computational
 * Visual Neuroscience application (Sec. 6.2; table "Performance of RTCG
 * auto-tuning on 3D filter-bank convolutions"): a bank of N filters, each
 * fh x fw x D and spanning the full depth of an H x W x D input (the
 * table's shape strings pair a 256x256x8 input with a 64x9x9x8 bank), is slid
 * over the two spatial axes; each filter position yields one output value per
 * filter.  The paper gives no formula.  Readings (listed in the design notes):
 * correlation without flipping the filter, "valid" output extent
 * Ho = H - fh + 1, Wo = W - fw + 1, stride one, no padding; C-order layouts
 * x[b][H][W][D], w[N][fh][fw][D], y[b][Ho][Wo][N].
 *
 *   forward:   y[b,i,j,n] = sum_{u<fh} sum_{v<fw} sum_{d<D} x[b,i+u,j+v,d] * w[n,u,v,d]
 *
 * The paper has no backward pass.  The gradients are the adjoint of the
 * forward map for the loss L = sum g * y, written here in scatter form:
 *
 *   for every (b,i,j,n,u,v,d):
 *       dx[b,i+u,j+v,d] += g[b,i,j,n] * w[n,u,v,d]
 *       dw[n,u,v,d]     += g[b,i,j,n] * x[b,i+u,j+v,d]
 *
 * Every sum runs sequentially in double precision in the loop order written;
 * OpenMP only splits independent outputs between threads, never a sum.
 */
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

void fbo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int fbo_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Forward correlation.  Threads take whole output rows (b, i). */
void fbo_forward(const double* x, const double* w, double* y,
                 i64 B, i64 H, i64 W, i64 D, i64 N, i64 fh, i64 fw)
{
    const i64 Ho = H - fh + 1, Wo = W - fw + 1;
    if (Ho <= 0 || Wo <= 0) return;
    i64 row;
#pragma omp parallel for schedule(dynamic, 1)
    for (row = 0; row < B * Ho; ++row) {
        const i64 b = row / Ho, i = row % Ho;
        for (i64 j = 0; j < Wo; ++j) {
            for (i64 n = 0; n < N; ++n) {
                double acc = 0.0;
                for (i64 u = 0; u < fh; ++u)
                    for (i64 v = 0; v < fw; ++v)
                        for (i64 d = 0; d < D; ++d)
                            acc += x[((b * H + i + u) * W + j + v) * D + d]
                                 * w[((n * fh + u) * fw + v) * D + d];
                y[((b * Ho + i) * Wo + j) * N + n] = acc;
            }
        }
    }
}

/* Input gradient, scatter form.  A thread owns one (b, d) plane of dx, so no
 * two threads ever add into the same element. */
void fbo_backward_x(const double* w, const double* g, double* dx,
                    i64 B, i64 H, i64 W, i64 D, i64 N, i64 fh, i64 fw)
{
    const i64 Ho = H - fh + 1, Wo = W - fw + 1;
    memset(dx, 0, sizeof(double) * (size_t)(B * H * W * D));
    if (Ho <= 0 || Wo <= 0) return;
    i64 plane;
#pragma omp parallel for schedule(dynamic, 1)
    for (plane = 0; plane < B * D; ++plane) {
        const i64 b = plane / D, d = plane % D;
        for (i64 i = 0; i < Ho; ++i)
            for (i64 j = 0; j < Wo; ++j)
                for (i64 n = 0; n < N; ++n) {
                    const double gv = g[((b * Ho + i) * Wo + j) * N + n];
                    for (i64 u = 0; u < fh; ++u)
                        for (i64 v = 0; v < fw; ++v)
                            dx[((b * H + i + u) * W + j + v) * D + d] +=
                                gv * w[((n * fh + u) * fw + v) * D + d];
                }
    }
}

/* Filter gradient, scatter form.  A thread owns one filter n of dw. */
void fbo_backward_w(const double* x, const double* g, double* dw,
                    i64 B, i64 H, i64 W, i64 D, i64 N, i64 fh, i64 fw)
{
    const i64 Ho = H - fh + 1, Wo = W - fw + 1;
    memset(dw, 0, sizeof(double) * (size_t)(N * fh * fw * D));
    if (Ho <= 0 || Wo <= 0) return;
    i64 n;
#pragma omp parallel for schedule(dynamic, 1)
    for (n = 0; n < N; ++n)
        for (i64 b = 0; b < B; ++b)
            for (i64 i = 0; i < Ho; ++i)
                for (i64 j = 0; j < Wo; ++j) {
                    const double gv = g[((b * Ho + i) * Wo + j) * N + n];
                    for (i64 u = 0; u < fh; ++u)
                        for (i64 v = 0; v < fw; ++v)
                            for (i64 d = 0; d < D; ++d)
                                dw[((n * fh + u) * fw + v) * D + d] +=
                                    gv * x[((b * H + i + u) * W + j + v) * D + d];
                }
}
