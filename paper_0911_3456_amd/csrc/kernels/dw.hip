// Filter gradient, split-K over output pixels, on the matrix cores (fp32).
//
//   dw[n,u,v,d] = sum_b sum_{i<HO, j<WO} dy[b,i,j,n] * x[b,i+u,j+v,d]
//
// GEMM view: rows = filters n, columns = taps q = (u, v, d), contraction over
// output pixels (b, i, j).  The 32x32 output tiles of the (n, q) plane are
// numbered row-fastest; workgroup row blockIdx.y owns TPB consecutive tiles
// and its NW waves take them round-robin (so no wave computes whole padding
// tiles).  Pixels are cut into chunks of RH x RW output positions; workgroup
// column g takes chunks g, g + NP, g + 2NP, ... and writes its partial sums to
// part[g][n][q] (the caller's workspace); a separate kernel adds the NP
// partials in a fixed order, so the result does not depend on scheduling.
// Per chunk, dy[chunk][all n] and the matching input tile with its
// (FH-1, FW-1) halo are staged in LDS; with PF the next chunk is fetched into
// registers while the current one is consumed (pre-fetching and software
// pipelining); with PF = 2 the LDS copy is double-buffered as well, so the
// next chunk is written to LDS while other waves still compute and each
// chunk costs one barrier.  The B fragment of a lane for tap column q is the input value
// at its pixel offset by (u, v), channel d.
//
//
// Balanced mode (BAL).  Dealing TPB tiles round-robin gives some waves one
// tile more than others, and since every chunk ends at a barrier the chunk
// takes as long as the busiest SIMD.  With BAL the workgroup's tiles are dealt
// in R = NTW / NW full rounds only; the RM = NTW % NW tiles left over are cut
// by pixel pairs instead: their RM * PC/2 (tile, step) units are split into
// NW contiguous ranges, one per wave, so every wave issues the same number of
// products per chunk.  A range touches at most two of those tiles (two extra
// accumulator slots); at the end the slots of each left-over tile are added
// in LDS in wave order (a fixed order, so results do not depend on timing).
//
// Compile-time constants (FB_<name>):
//   problem  BATCH FH FW D N H W HO WO
//   tiling   RH RW (pixel chunk)  NW (waves)  TPB (tiles per workgroup)
//            NP (partials = workgroup columns)  GPAD XPAD (LDS padding)
//            PF (0: none, 1: register prefetch of the next chunk,
//                2: register prefetch + double-buffered LDS)
//            BAL (0: round-robin tiles, 1: balanced split of the left-over
//                 tiles, see above)
//            UNR (unrolling of the per-chunk step loop: 0 = complete, which
//                 turns every LDS address into an immediate offset; k = by k)
//            SKIPE (1: a wave whose last round-robin slot is empty skips its
//                 products instead of computing a discarded tile)
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
#define NW FB_NW
#define TPB FB_TPB
#define NP FB_NP
#define GPAD FB_GPAD
#define XPAD FB_XPAD
#define PF FB_PF
#ifdef FB_BAL
#define BAL FB_BAL
#else
#define BAL 0
#endif
#ifdef FB_UNR
#define UNR FB_UNR
#else
#define UNR 4
#endif
#ifdef FB_SKIPE
#define SKIPE FB_SKIPE
#else
#define SKIPE 0
#endif

template <int V> struct IConst { static constexpr int value = V; };

typedef float f32x16 __attribute__((ext_vector_type(16)));

#define NTHREADS (NW * 64)
#define QTOT (FH * FW * D)
#define NROWT ((N + 31) / 32)
#define NCOLT ((QTOT + 31) / 32)
#define TILES (NROWT * NCOLT)
#define TPW ((TPB + NW - 1) / NW)        // tiles per wave (at most)
#define NPAD (NROWT * 32)
#define GST (NPAD + GPAD)                // dy tile pixel stride
#define PC (RH * RW)                     // pixels per chunk
#define XR (RH + FH - 1)
#define XC (RW + FW - 1)
#define XRS (XC * D + XPAD)              // input tile row stride
#define NCH_I ((HO + RH - 1) / RH)
#define NCH_J ((WO + RW - 1) / RW)
#define NCHUNKS (BATCH * NCH_I * NCH_J)
#define GITEMS (PC * NPAD)
#define XITEMS (XR * XC * D)
#define GPER ((GITEMS + NTHREADS - 1) / NTHREADS)
#define XPER ((XITEMS + NTHREADS - 1) / NTHREADS)

// A wave's tiles are NW apart in the row-fastest numbering, so they all lie
// in one filter-row tile when NW is a multiple of the row-tile count; the A
// fragment is then read once per step.  (If a wave's first tile is past the
// end, so are all its others.)
#define SAMEROW (NW % NROWT == 0)

static_assert(PC % 2 == 0, "pixel chunk must be even");

#define NBUF (PF == 2 ? 2 : 1)
#define HS (PC / 2)                      // MFMA steps per chunk (two pixels each)
#if BAL
#define RFULL (TPB / NW)                 // full rounds of tiles
#define NSLOT (RFULL + 2)                // + two slots for left-over tiles
#else
#define RFULL TPW
#define NSLOT TPW
#endif
#define STAGE_FLOATS (NBUF * (PC * GST + XR * XRS))
#define RED_FLOATS (BAL ? NW * 2 * 16 * 64 : 0)
#define LDS_FLOATS (STAGE_FLOATS > RED_FLOATS ? STAGE_FLOATS : RED_FLOATS)

extern "C" __global__ void __launch_bounds__(NTHREADS)
fbcorr_dw_partial(const float* __restrict__ x, const float* __restrict__ dy,
                  float* __restrict__ part)
{
    // Staging buffers (dy chunk, input tile; two of each with PF = 2); with
    // BAL the same memory holds the left-over slots for the final sum.
    __shared__ __attribute__((aligned(16))) float lds_raw[LDS_FLOATS];
    float* const gl_base = lds_raw;
    float* const xl_base = lds_raw + NBUF * PC * GST;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l32 = lane & 31, h = lane >> 5;
    const int g = blockIdx.x;

    // Slot k < RFULL holds tile wave + k*NW of the workgroup.  With BAL,
    // slots RFULL and RFULL + 1 hold left-over tiles r0 and r0 + 1 for the
    // steps [slo[j], shi[j]) of every chunk.
    int lt_of[NSLOT];
#if BAL
    const int ntw = (TILES - (int)blockIdx.y * TPB) < TPB ? TILES - (int)blockIdx.y * TPB : TPB;
    const int rfull = ntw / NW, rm = ntw % NW;
    const int units = rm * HS;
    const int lo = wave * units / NW, hi = (wave + 1) * units / NW;
    const int r0 = lo / HS;
    int slo[2], shi[2];
    slo[0] = lo - r0 * HS;
    shi[0] = hi - r0 * HS < HS ? hi - r0 * HS : HS;
    slo[1] = 0;
    shi[1] = hi - (r0 + 1) * HS > 0 ? hi - (r0 + 1) * HS : 0;
#pragma unroll
    for (int k = 0; k < RFULL; ++k) lt_of[k] = k < rfull ? wave + k * NW : TPB;
    lt_of[RFULL] = slo[0] < shi[0] ? rfull * NW + r0 : TPB;
    lt_of[RFULL + 1] = slo[1] < shi[1] ? rfull * NW + r0 + 1 : TPB;
#else
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) lt_of[k] = wave + k * NW;
#endif

    // Per slot: row offset into the dy tile and LDS offset of tap q relative
    // to the pixel's own position (0 for padding columns and empty slots: an
    // in-bounds read whose result is never stored).
    int arow[NSLOT], qoff[NSLOT], tq[NSLOT], tn[NSLOT];
    bool tval[NSLOT];
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) {
        const int lt = lt_of[k];
        const int t = blockIdx.y * TPB + lt;
        tval[k] = lt < TPB && t < TILES;
        const int rt = tval[k] ? t % NROWT : 0, ct = tval[k] ? t / NROWT : 0;
        arow[k] = rt * 32 + l32;
        tn[k] = rt * 32;
        const int q = ct * 32 + l32;
        tq[k] = q;
        if (q < QTOT) {
            const int u = q / (FW * D), rem = q % (FW * D);
            qoff[k] = u * XRS + rem;      // rem = v*D + d
        } else {
            qoff[k] = 0;
        }
    }

#if SKIPE && !BAL && RFULL > 1
    const bool last_ok = __builtin_amdgcn_readfirstlane(tval[RFULL - 1] ? 1 : 0) != 0;
#endif
    f32x16 acc[NSLOT];
#pragma unroll
    for (int k = 0; k < NSLOT; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;

    // Chunk staging: global -> registers (fetch) and registers -> LDS (store).
    float greg[GPER], xreg[XPER];
    auto fetch = [&](int ch) {
        const int b = ch / (NCH_I * NCH_J);
        const int i0 = ((ch / NCH_J) % NCH_I) * RH, j0 = (ch % NCH_J) * RW;
#pragma unroll
        for (int r = 0; r < GPER; ++r) {
            const int e = tid + r * NTHREADS;
            float v = 0.f;
            if (e < GITEMS) {
                const int p = e / NPAD, n = e % NPAD;
                const int i = i0 + p / RW, j = j0 + p % RW;
                if (i < HO && j < WO && n < N) v = dy[(((long)b * HO + i) * WO + j) * N + n];
            }
            greg[r] = v;
        }
#pragma unroll
        for (int r = 0; r < XPER; ++r) {
            const int e = tid + r * NTHREADS;
            float v = 0.f;
            if (e < XITEMS) {
                const int rr = e / (XC * D), rem = e % (XC * D);
                const int ii = i0 + rr, jj = j0 + rem / D;
                if (ii < H && jj < W) v = x[(((long)b * H + ii) * W + jj) * D + rem % D];
            }
            xreg[r] = v;
        }
    };
    auto store = [&](int b) {
        float* gl = gl_base + b * (PC * GST);
        float* xl = xl_base + b * (XR * XRS);
#pragma unroll
        for (int r = 0; r < GPER; ++r) {
            const int e = tid + r * NTHREADS;
            if (e < GITEMS) gl[(e / NPAD) * GST + e % NPAD] = greg[r];
        }
#pragma unroll
        for (int r = 0; r < XPER; ++r) {
            const int e = tid + r * NTHREADS;
            if (e < XITEMS) xl[(e / (XC * D)) * XRS + e % (XC * D)] = xreg[r];
        }
    };

    // The products of one staged chunk (LDS buffer b).
    auto compute = [&](int b) {
        // Lane half h walks pixels [h*HS, (h+1)*HS) of the chunk.  When the
        // chunk has an even number of rows a half starts on a row boundary:
        // the step's LDS offsets are then a per-lane base plus a constant of
        // the (unrolled) step, which the reads take as immediate offsets.
#if (HS % RW) == 0
        const float* gl = gl_base + b * (PC * GST) + h * (HS * GST);
        const float* xl = xl_base + b * (XR * XRS) + h * ((HS / RW) * XRS);
#define STEP_PIXEL(t) (t)
#else
        const float* gl = gl_base + b * (PC * GST);
        const float* xl = xl_base + b * (XR * XRS);
#define STEP_PIXEL(t) (h * HS + (t))
#endif
#if RFULL > 0
        // The step loop over the first NS slots (NS a compile-time count).
        auto steps = [&](auto ns) {
            constexpr int NS = decltype(ns)::value;
#if UNR == 0
#pragma unroll
#else
#pragma unroll UNR
#endif
            for (int t = 0; t < HS; ++t) {
                const int p = STEP_PIXEL(t);
                const int xo = (p / RW) * XRS + (p % RW) * D;
#if SAMEROW
                const float a0 = gl[p * GST + arow[0]];
#endif
#pragma unroll
                for (int k = 0; k < NS; ++k) {
#if SAMEROW
                    const float a = a0;
#else
                    const float a = gl[p * GST + arow[k]];
#endif
                    const float bb = xl[xo + qoff[k]];
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc[k], 0, 0, 0);
                }
            }
        };
#if SKIPE && !BAL && RFULL > 1
        // a wave whose last slot holds no tile skips its products
        if (last_ok) steps(IConst<RFULL>{});
        else steps(IConst<RFULL - 1>{});
#else
        steps(IConst<RFULL>{});
#endif
#endif
#if BAL
        // This wave's share of the left-over tiles.
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = RFULL + j;
#pragma unroll 4
            for (int t = slo[j]; t < shi[j]; ++t) {
                const int p = STEP_PIXEL(t);
                const int xo = (p / RW) * XRS + (p % RW) * D;
                const float a = gl[p * GST + arow[k]];
                const float bb = xl[xo + qoff[k]];
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc[k], 0, 0, 0);
            }
        }
#endif
#undef STEP_PIXEL
    };

#if PF == 2
    // Double-buffered: chunk ch is in LDS buffer b, chunk ch + NP in
    // registers; after computing ch the registers go to the other buffer and
    // ch + 2NP is fetched.  One barrier per chunk.
    if (g < NCHUNKS) {
        fetch(g);
        store(0);
        if (g + NP < NCHUNKS) fetch(g + NP);
    }
    __syncthreads();
    int buf = 0;
#pragma unroll 1
    for (int ch = g; ch < NCHUNKS; ch += NP) {
        compute(buf);
        if (ch + NP < NCHUNKS) {
            store(buf ^ 1);
            if (ch + 2 * NP < NCHUNKS) fetch(ch + 2 * NP);
        }
        __syncthreads();
        buf ^= 1;
    }
#else
    if (g < NCHUNKS) fetch(g);
#pragma unroll 1
    for (int ch = g; ch < NCHUNKS; ch += NP) {
        __syncthreads();               // everyone is done with the previous chunk
        store(0);
        __syncthreads();
#if PF
        if (ch + NP < NCHUNKS) fetch(ch + NP);    // in flight during the compute
#endif
        compute(0);
#if !PF
        if (ch + NP < NCHUNKS) fetch(ch + NP);
#endif
    }
#endif

    // Partial sums: part[g][n][q] (zeros from workgroups without chunks).
    float* out = part + (long)g * N * QTOT;
#pragma unroll
    for (int k = 0; k < RFULL; ++k) {
        if (!tval[k]) continue;
        const int q = tq[k];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = tn[k] + 8 * (r >> 2) + 4 * h + (r & 3);
            if (n < N && q < QTOT) out[(long)n * QTOT + q] = acc[k][r];
        }
    }
#if BAL
    // Left-over tiles: every wave parks its two slots in LDS (the staging
    // buffers are free once all waves are past their last chunk), then wave
    // w < RM adds the slots holding left-over tile w in wave order.
    __syncthreads();
    float* red = lds_raw;
#pragma unroll
    for (int j = 0; j < 2; ++j)
        if (tval[RFULL + j])
#pragma unroll
            for (int r = 0; r < 16; ++r) red[((wave * 2 + j) * 16 + r) * 64 + lane] = acc[RFULL + j][r];
    __syncthreads();
    if (wave < rm) {
        f32x16 s;
#pragma unroll
        for (int r = 0; r < 16; ++r) s[r] = 0.f;
#pragma unroll 1
        for (int w2 = 0; w2 < NW; ++w2) {
            const int lo2 = w2 * units / NW, hi2 = (w2 + 1) * units / NW;
            if (lo2 == hi2) continue;
            const int r02 = lo2 / HS;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // slot j of wave w2 covers tile r02 + j if its step range is non-empty
                const int jlo = j == 0 ? lo2 - r02 * HS : 0;
                const int jhi = j == 0 ? (hi2 - r02 * HS < HS ? hi2 - r02 * HS : HS)
                                       : (hi2 - (r02 + 1) * HS > 0 ? hi2 - (r02 + 1) * HS : 0);
                if (r02 + j != wave || jlo >= jhi) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) s[r] += red[((w2 * 2 + j) * 16 + r) * 64 + lane];
            }
        }
        const int t = blockIdx.y * TPB + rfull * NW + wave;
        const int rt = t % NROWT, ct = t / NROWT;
        const int q = ct * 32 + l32;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = rt * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            if (n < N && q < QTOT) out[(long)n * QTOT + q] = s[r];
        }
    }
#endif
}
