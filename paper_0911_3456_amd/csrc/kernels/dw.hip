// Filter gradient, split-K over output pixels, on the matrix cores (fp32).
//
//   dw[n,u,v,d] = sum_b sum_{i<HO, j<WO} dy[b,i,j,n] * x[b,i+u,j+v,d]
//
// GEMM view: rows = filters n, columns = taps q = (u, v, d), contraction over
// output pixels (b, i, j).  Pixels are cut into chunks of RH x RW output
// positions; workgroup g takes chunks g, g + P, g + 2P, ... (P = gridDim.x)
// and writes its partial sums to part[g][n][q] (the caller's workspace).  A
// separate kernel adds the P partials in a fixed order, so the result does
// not depend on scheduling.  Per chunk, dy[chunk][n] and the matching input
// tile with its (FH-1, FW-1) halo are staged in LDS; the B fragment of a lane
// for column q is the input value at its pixel offset by (u, v), channel d.
//
// Compile-time constants:
//   problem  BATCH FH FW D N H W HO WO
//   tiling   RH RW (pixel chunk)  MT NT (32x32 tiles per wave)  WM WN
//            (waves along rows/cols)  GPAD XPAD (LDS padding)
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#ifdef FB_INJECT_ERROR
#error "injected code-generation failure (test hook)"
#endif
// Specialisation constants arrive as FB_<name> (see the host generator).
#define BATCH FB_BATCH
#define FH FB_FH
#define FW FB_FW
#define D FB_D
#define N FB_N
#define H FB_H
#define W FB_W
#define HO FB_HO
#define WO FB_WO
#define RH FB_RH
#define RW FB_RW
#define MT FB_MT
#define NT FB_NT
#define WM FB_WM
#define WN FB_WN
#define GPAD FB_GPAD
#define XPAD FB_XPAD

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define NWAVES (WM * WN)
#define NTHREADS (NWAVES * 64)
#define QTOT (FH * FW * D)
#define RB (WM * MT * 32)         // filter rows per workgroup
#define CBK (WN * NT * 32)        // tap columns per workgroup
#define PC (RH * RW)              // pixels per chunk
#define XR (RH + FH - 1)
#define XC (RW + FW - 1)
#define XRS (XC * D + XPAD)       // input tile row stride
#define GST (RB + GPAD)           // dy tile pixel stride
#define NCH_I ((HO + RH - 1) / RH)
#define NCH_J ((WO + RW - 1) / RW)
#define NCHUNKS (BATCH * NCH_I * NCH_J)

static_assert(PC % 2 == 0, "pixel chunk must be even");

extern "C" __global__ void __launch_bounds__(NTHREADS)
fbcorr_dw_partial(const float* __restrict__ x, const float* __restrict__ dy,
                  float* __restrict__ part)
{
    __shared__ __attribute__((aligned(16))) float gl[PC * GST];
    __shared__ __attribute__((aligned(16))) float xl[XR * XRS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int l32 = lane & 31, h = lane >> 5;
    const int P = gridDim.x;
    const int g = blockIdx.x;
    const int ncb = (QTOT + CBK - 1) / CBK;
    const int cb = blockIdx.y % ncb;
    const int rbk = blockIdx.y / ncb;
    const int n0 = rbk * RB, q0 = cb * CBK;

    // Per lane and column tile: the LDS offset of tap q = (u, v, d) relative
    // to the pixel's own position, or -1 past the last tap.
    int qoff[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int q = q0 + (wn * NT + nt) * 32 + l32;
        if (q < QTOT) {
            const int u = q / (FW * D), rem = q % (FW * D);
            qoff[nt] = u * XRS + rem;      // rem = v*D + d
        } else {
            qoff[nt] = 0;                  // any in-bounds value; never stored
        }
    }

    f32x16 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mt][nt][r] = 0.f;

    for (int ch = g; ch < NCHUNKS; ch += P) {
        const int b = ch / (NCH_I * NCH_J);
        const int ci = (ch / NCH_J) % NCH_I, cj = ch % NCH_J;
        const int i0 = ci * RH, j0 = cj * RW;
        __syncthreads();
        // dy chunk, [pixel][filter row in block]; zero outside.
        for (int e = tid; e < PC * RB; e += NTHREADS) {
            const int p = e / RB, n = e % RB;
            const int i = i0 + p / RW, j = j0 + p % RW;
            float v = 0.f;
            if (i < HO && j < WO && n0 + n < N)
                v = dy[(((long)b * HO + i) * WO + j) * N + n0 + n];
            gl[p * GST + n] = v;
        }
        // input tile with halo, [row][col][d]; zero outside.
        for (int e = tid; e < XR * XC * D; e += NTHREADS) {
            const int r = e / (XC * D), rem = e % (XC * D);
            const int ii = i0 + r, jj = j0 + rem / D;
            float v = 0.f;
            if (ii < H && jj < W) v = x[(((long)b * H + ii) * W + jj) * D + rem % D];
            xl[r * XRS + rem] = v;
        }
        __syncthreads();

        // Lane half h walks pixels [h*PC/2, (h+1)*PC/2) of the chunk.
#pragma unroll 4
        for (int t = 0; t < PC / 2; ++t) {
            const int p = h * (PC / 2) + t;
            const int pi = p / RW, pj = p % RW;
            float a[MT], bb[NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[mt] = gl[p * GST + (wm * MT + mt) * 32 + l32];
            const int xo = pi * XRS + pj * D;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bb[nt] = xl[xo + qoff[nt]];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mt], bb[nt], acc[mt][nt], 0, 0, 0);
        }
    }

    // Partial sums: part[g][n][q].
    float* out = part + (long)g * N * QTOT;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int q = q0 + (wn * NT + nt) * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int n = n0 + (wm * MT + mt) * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                if (n < N && q < QTOT) out[(long)n * QTOT + q] = acc[mt][nt][r];
            }
        }
}
