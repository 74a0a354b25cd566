// Direct filter-bank correlation on the vector ALUs (fp32).
//
//   y[b,i,j,n] = sum_{u<FH, v<FW, d<D} x[b,i+u,j+v,d] * w[n,u,v,d]
//
// One workgroup computes an output tile of TH x TW pixels for NB filters.
// The input tile with its (FH-1, FW-1) halo is staged once in LDS; the
// filter slice for one filter row u is staged per step (FSRC = 0), or, with
// FSRC = 1, every wave's threads share one filter group and read their
// weights with scalar loads from a tap-major copy of the filters (w then
// points at that copy, wt[((u*FW + v)*D + d)*NPAD + n]): no LDS for the
// weights and no barrier per filter row; the weights reach the FMAs as
// scalar operands.  Each thread
// accumulates P horizontally adjacent pixels x Q filters in registers; for a
// fixed (u, d) its P+FW-1 inputs are read once and reused across the FW taps
// (the sliding window), and the Q weights of a tap are one broadcast read
// shared by every lane of the same filter group.  With DS > 1 the D channels
// are split across DS neighbouring lanes and the partial sums are combined
// with cross-lane shuffles at the end (a fixed butterfly order).
//
// Compile-time constants (Sec. 4.2 "hardcoding", Sec. 5.3 keyword
// substitution; the knobs are the Sec. 6.2 tuning dimensions: unroll depth,
// block dimensions, thread work size, shared-memory padding):
//   problem  BATCH FH FW D N H W HO WO
//   tiling   TH TW (output tile)  P Q (pixels x filters per thread)
//            NB (filters per workgroup)  DS (channel split across lanes)
//            LAYOUT (0: tile [row][col][d], 1: tile [d][row][col])
//            XPAD WPAD (LDS padding)  UD (unroll of the channel loop)
//            XCDMAP (XCD-aware workgroup order)
//            FSRC (filter source: 0 LDS slice, 1 scalar loads; NPAD = filter
//            count of the tap-major copy)
//            SB (1: the input tile and each filter slice are staged with
//            every load of a batch issued before the first store)
//   EPILOGUE(v, c)  optional elementwise function of an output value v and
//            its filter c, applied before the store (a fused nonlinearity)
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
#define TH FB_TH
#define TW FB_TW
#define P FB_P
#define Q FB_Q
#define NB FB_NB
#define DS FB_DS
#define LAYOUT FB_LAYOUT
#define XPAD FB_XPAD
#define WPAD FB_WPAD
#define UD FB_UD
#define XCDMAP FB_XCDMAP
#ifdef FB_FSRC
#define FSRC FB_FSRC
#else
#define FSRC 0
#endif
#ifdef FB_SB
#define SB FB_SB              // 1: staging loads issued in batches (see below)
#else
#define SB 0
#endif

typedef float f32x4 __attribute__((ext_vector_type(4)));

#define NPG (TH * (TW / P))       // pixel groups per workgroup
#define NFG (NB / Q)              // filter groups per workgroup
#define NTHREADS (NPG * NFG * DS)
#define TRR (TH + FH - 1)         // tile rows
#define TCC (TW + FW - 1)         // tile columns
#if LAYOUT == 0
#define XRS (TCC * D + XPAD)
#define TILE_ELEMS (TRR * XRS)
#define TIDX(d, r, c) ((r) * XRS + (c) * D + (d))
#else
#define XRS (TCC + XPAD)
#define TILE_ELEMS (D * TRR * XRS)
#define TIDX(d, r, c) (((d) * TRR + (r)) * XRS + (c))
#endif
#define NBS (NB + WPAD)
#define WSL_ELEMS (FW * D * NBS)
#define WIT ((NB * FW * D + NTHREADS - 1) / NTHREADS)   // filter-slice values per thread

static_assert(TW % P == 0, "P must divide TW");
static_assert(NB % Q == 0, "Q must divide NB");
static_assert(Q % 4 == 0, "Q must be a multiple of 4");
static_assert(D % DS == 0, "DS must divide D");
static_assert(NBS % 4 == 0, "filter rows must stay 16-byte aligned");
#if FSRC
static_assert(DS == 1 && NPG % 64 == 0, "scalar weights need one filter group per wave");
#define NPAD FB_NPAD
#endif

extern "C" __global__ void __launch_bounds__(NTHREADS)
fbcorr_direct(const float* __restrict__ x, const float* __restrict__ w, float* __restrict__ y)
{
    __shared__ __attribute__((aligned(16))) float tile[TILE_ELEMS];
#if !FSRC
    __shared__ __attribute__((aligned(16))) float wsl[WSL_ELEMS];
#endif

    const int tid = threadIdx.x;
    const int ds = tid % DS;
    const int pg = (tid / DS) % NPG;
    const int fg = tid / (DS * NPG);
    const int ti = pg / (TW / P);
    const int tj = (pg % (TW / P)) * P;

    const int ntx = (WO + TW - 1) / TW;
    const int nty = (HO + TH - 1) / TH;
    const int nnb = (N + NB - 1) / NB;
    const int total = ntx * nty * nnb * BATCH;
    int lin = blockIdx.x;
#if XCDMAP
    {
        const int q = total / 8, r = total % 8, xc = lin % 8;
        lin = xc * q + (xc < r ? xc : r) + lin / 8;
    }
#endif
    const int tx = lin % ntx;
    const int ty = (lin / ntx) % nty;
    const int nb = (lin / (ntx * nty)) % nnb;
    const int b = lin / (ntx * nty * nnb);
    const int oi0 = ty * TH, oj0 = tx * TW, n0 = nb * NB;

    // Stage the input tile; outside the image stays zero (only reachable by
    // outputs that are not stored).
    const long xb = (long)b * H * W * D;
#if D % 4 == 0 && SB
    // In batches of XB 16-byte loads per thread, every load of a batch
    // issued before the first store (one memory latency per batch).
    {
        constexpr int XIT = (TRR * TCC * D + NTHREADS * 4 - 1) / (NTHREADS * 4);
        constexpr int XB = XIT < 6 ? XIT : 6;
#pragma unroll 1
        for (int i0 = 0; i0 < XIT; i0 += XB) {
            f32x4 v[XB];
#pragma unroll
            for (int i = 0; i < XB; ++i) {
                const int e = (tid + (i0 + i) * NTHREADS) * 4;
                const int r = e / (TCC * D), rem = e % (TCC * D);
                const int c = rem / D, d = rem % D;
                const int ii = oi0 + r, jj = oj0 + c;
                v[i] = (f32x4){0.f, 0.f, 0.f, 0.f};
                if (e < TRR * TCC * D && ii < H && jj < W) v[i] = *(const f32x4*)(x + xb + ((long)ii * W + jj) * D + d);
            }
#pragma unroll
            for (int i = 0; i < XB; ++i) {
                const int e = (tid + (i0 + i) * NTHREADS) * 4;
                const int r = e / (TCC * D), rem = e % (TCC * D);
                const int c = rem / D, d = rem % D;
                if (e < TRR * TCC * D) {
                    tile[TIDX(d, r, c)] = v[i][0];
                    tile[TIDX(d + 1, r, c)] = v[i][1];
                    tile[TIDX(d + 2, r, c)] = v[i][2];
                    tile[TIDX(d + 3, r, c)] = v[i][3];
                }
            }
        }
    }
#elif D % 4 == 0
    for (int e = tid * 4; e < TRR * TCC * D; e += NTHREADS * 4) {
        const int r = e / (TCC * D), rem = e % (TCC * D);
        const int c = rem / D, d = rem % D;
        const int ii = oi0 + r, jj = oj0 + c;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (ii < H && jj < W) v = *(const f32x4*)(x + xb + ((long)ii * W + jj) * D + d);
        tile[TIDX(d, r, c)] = v[0];
        tile[TIDX(d + 1, r, c)] = v[1];
        tile[TIDX(d + 2, r, c)] = v[2];
        tile[TIDX(d + 3, r, c)] = v[3];
    }
#else
    for (int e = tid; e < TRR * TCC * D; e += NTHREADS) {
        const int r = e / (TCC * D), rem = e % (TCC * D);
        const int c = rem / D, d = rem % D;
        const int ii = oi0 + r, jj = oj0 + c;
        float v = 0.f;
        if (ii < H && jj < W) v = x[xb + ((long)ii * W + jj) * D + d];
        tile[TIDX(d, r, c)] = v;
    }
#endif

    float acc[P][Q];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[p][q] = 0.f;

#if FSRC
    __syncthreads();
    // The wave's filter group, made explicitly uniform so that its weight
    // addresses are scalar.
    const int fgu = __builtin_amdgcn_readfirstlane(fg);
#endif
#pragma unroll 1
    for (int u = 0; u < FH; ++u) {
#if !FSRC
        __syncthreads();
        // Filter slice for row u, stored [v][d][filter] so that the Q weights
        // of one tap are contiguous; every load issued before the first store.
#if SB && WIT <= 32
        {
            float wv[WIT];
#pragma unroll
            for (int k = 0; k < WIT; ++k) {
                const int e = tid + k * NTHREADS;
                const int f = e / (FW * D), vd = e % (FW * D);
                const int n = n0 + f;
                wv[k] = (e < NB * FW * D && n < N) ? w[((long)n * FH + u) * FW * D + vd] : 0.f;
            }
#pragma unroll
            for (int k = 0; k < WIT; ++k) {
                const int e = tid + k * NTHREADS;
                const int f = e / (FW * D), vd = e % (FW * D);
                if (e < NB * FW * D) wsl[vd * NBS + f] = wv[k];
            }
        }
#else
        for (int e = tid; e < NB * FW * D; e += NTHREADS) {
            const int f = e / (FW * D), vd = e % (FW * D);
            const int n = n0 + f;
            wsl[vd * NBS + f] = (n < N) ? w[((long)n * FH + u) * FW * D + vd] : 0.f;
        }
#endif
        __syncthreads();
#endif

#pragma unroll UD
        for (int dd = 0; dd < D / DS; ++dd) {
            const int d = dd * DS + ds;
            float xr[P + FW - 1];
#pragma unroll
            for (int e = 0; e < P + FW - 1; ++e) xr[e] = tile[TIDX(d, ti + u, tj + e)];
#pragma unroll
            for (int v = 0; v < FW; ++v) {
#if FSRC
                const float* wp = w + ((long)(u * FW + v) * D + d) * NPAD + n0 + fgu * Q;
#else
                const float* wp = wsl + (v * D + d) * NBS + fg * Q;
#endif
#pragma unroll
                for (int q4 = 0; q4 < Q; q4 += 4) {
                    const f32x4 wv = *(const f32x4*)(wp + q4);
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        acc[p][q4 + 0] = __builtin_fmaf(xr[p + v], wv[0], acc[p][q4 + 0]);
                        acc[p][q4 + 1] = __builtin_fmaf(xr[p + v], wv[1], acc[p][q4 + 1]);
                        acc[p][q4 + 2] = __builtin_fmaf(xr[p + v], wv[2], acc[p][q4 + 2]);
                        acc[p][q4 + 3] = __builtin_fmaf(xr[p + v], wv[3], acc[p][q4 + 3]);
                    }
                }
            }
        }
    }

#if DS > 1
    // Channel reduction across the DS lanes of one pixel group (butterfly).
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            float a = acc[p][q];
#pragma unroll
            for (int off = 1; off < DS; off <<= 1) a += __shfl_xor(a, off, 64);
            acc[p][q] = a;
        }
#endif

    const int oi = oi0 + ti;
    if (oi < HO) {
        const long yb = ((long)b * HO + oi) * WO;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int oj = oj0 + tj + p;
            if (oj < WO) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int n = n0 + fg * Q + q;
                    if ((q % DS) == ds && n < N) {
#ifdef FB_EPILOGUE
                        y[(yb + oj) * N + n] = FB_EPILOGUE(acc[p][q], n);   // fused elementwise epilogue
#else
                        y[(yb + oj) * N + n] = acc[p][q];
#endif
                    }
                }
            }
        }
    }
}
