// Implicit-GEMM valid correlation on the CDNA matrix cores (MFMA).
//
//   O[b,i,j,c] = sum_{u<FH, v<FW, k<CIN} Ipad[b, i+u, j+v, k] * Wt[c, u, v, k]
//
// where Ipad is the input I[b][HI][WI][CIN] with PADH/PADW rows/columns of
// virtual zeros on every side.  With I = x, Wt = w and no padding this is the
// forward filter-bank correlation of Sec. 6.2; with I = dy, Wt = w flipped in
// (u, v) and transposed n <-> d, and padding (FH-1, FW-1), it is the input
// gradient.  The GEMM view: rows = output pixels, columns = output channels,
// contraction over (u, v, k).  A (the im2col matrix) is never materialised:
// for a fixed filter row u the (v, k) pairs of one output pixel are one
// contiguous run of FW*KC values in the LDS input tile, so each lane reads its
// A fragment straight from the staged tile.
//
// Column-shift packing: when COUT is smaller than the 32 MFMA columns, a column
// is a pair (c, s), s < S, computing output column S*m + s for base pixel m.
// The contraction then runs over FW+S-1 taps per filter row, and
// B[(u, v', k), (c, s)] = Wt[c, u, v'-s, k] (zero outside 0 <= v'-s < FW).
//
// Everything below is a compile-time constant substituted at plan time
// (Sec. 4.2, "hardcoding"; Sec. 5.3, keyword substitution):
//   problem  BATCH FH FW CIN COUT HI WI HO WO PADH PADW
//   tiling   KC (channels per K chunk)  S (column shift)  MT NT (32x32 tiles
//            per wave along rows/cols)  WM WN (waves along rows/cols)
//            USTAGE (filter rows staged per LDS fill)  XPAD WPAD (LDS row
//            padding, elements)  XCDMAP (XCD-aware workgroup order)
//   type     DT: 0 = fp32 operands (v_mfma 32x32x2 f32), 1 = bf16, 2 = fp16
//            (32x32x16 with 8 operands per lane; Wt is then pre-scaled and
//            pre-rounded 16-bit, and UNSCALE[c] multiplies each output)
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
#define CIN FB_CIN
#define COUT FB_COUT
#define HI FB_HI
#define WI FB_WI
#define HO FB_HO
#define WO FB_WO
#define PADH FB_PADH
#define PADW FB_PADW
#define KC FB_KC
#define S FB_S
#define MT FB_MT
#define NT FB_NT
#define WM FB_WM
#define WN FB_WN
#define DT FB_DT
#define XPAD FB_XPAD
#define WPAD FB_WPAD
#define USTAGE FB_USTAGE
#define XCDMAP FB_XCDMAP

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

#define NWAVES (WM * WN)
#define NTHREADS (NWAVES * 64)
#define TH (WM * MT)              // output rows per workgroup
#define TWO (32 * S)              // output columns per workgroup
#define NCOL (WN * NT * 32)       // MFMA columns per workgroup
#define CB (NCOL / S)             // output channels per workgroup
#define TR (TH + FH - 1)          // input tile rows
#define KRRAW ((FW + S - 1) * KC) // contraction run per filter row and chunk
#if DT == 0
#define RUNIT 8
#else
#define RUNIT 16
#endif
#define KR (((KRRAW + RUNIT - 1) / RUNIT) * RUNIT)
#define HALF (KR / 2)
#define ROWE (31 * S * KC + KR)   // tile row elements any lane may read
#define ROWS (ROWE + XPAD)        // tile row stride
#define WRS (KR + WPAD)           // filter-slice row stride
#define TILE_ELEMS (TR * ROWS)
#define WSL_ELEMS (USTAGE * NCOL * WRS)
#define NCHUNK ((CIN + KC - 1) / KC)

#if DT == 0
typedef float elem_t;
#else
typedef unsigned short elem_t;    // raw 16-bit patterns
#endif

// A-read vector width (elements) from the lane-to-lane stride S*KC.
#if DT == 0
#define AV (((S * KC) % 4 == 0) ? 4 : (((S * KC) % 2 == 0) ? 2 : 1))
#else
#define AV (((S * KC) % 8 == 0) ? 8 : (((S * KC) % 4 == 0) ? 4 : (((S * KC) % 2 == 0) ? 2 : 1)))
#endif

static_assert(NCOL % S == 0, "columns must split evenly into shifts");
static_assert(ROWS % AV == 0, "tile rows must keep the A reads aligned");
static_assert(WRS % 8 == 0 || (DT == 0 && WRS % 4 == 0), "filter rows must stay 16-byte aligned");

__device__ __forceinline__ elem_t to_elem(float v) {
#if DT == 0
    return v;
#elif DT == 1
    __bf16 h = (__bf16)v;                 // round to nearest even
    return __builtin_bit_cast(unsigned short, h);
#else
    _Float16 h = (_Float16)v;             // round to nearest even
    return __builtin_bit_cast(unsigned short, h);
#endif
}

// The symbol name is chosen by the generator (forward and input-gradient
// instances get distinct names, so profiles tell them apart).
#ifndef FB_KNAME
#define FB_KNAME fbcorr_igemm
#endif
extern "C" __global__ void __launch_bounds__(NTHREADS)
FB_KNAME(const float* __restrict__ I, const elem_t* __restrict__ Wt,
             const float* __restrict__ UNSCALE, float* __restrict__ O)
{
    __shared__ __attribute__((aligned(16))) elem_t tile[TILE_ELEMS];
    __shared__ __attribute__((aligned(16))) elem_t wsl[WSL_ELEMS];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM;
    const int wn = wave / WM;
    const int l32 = lane & 31;
    const int h = lane >> 5;

    // Workgroup -> tile.  With XCDMAP the dispatcher's round-robin over the
    // eight XCDs is undone so that each XCD works on a contiguous range of
    // tiles (shared halos and filter slices stay in that XCD's L2).
    const int ntx = (WO + TWO - 1) / TWO;
    const int nty = (HO + TH - 1) / TH;
    const int ncb = (COUT + CB - 1) / CB;
    const int total = ntx * nty * ncb * BATCH;   // == gridDim.x
    int lin = blockIdx.x;
#if XCDMAP
    {
        const int q = total / 8, r = total % 8, x = lin % 8;
        lin = x * q + (x < r ? x : r) + lin / 8;
    }
#endif
    const int tx = lin % ntx;
    const int ty = (lin / ntx) % nty;
    const int cblk = (lin / (ntx * nty)) % ncb;
    const int b = lin / (ntx * nty * ncb);
    const int oi0 = ty * TH;
    const int oj0 = tx * TWO;
    const int c0 = cblk * CB;

    f32x16 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mt][nt][r] = 0.0f;

    const long ibase = (long)b * HI * WI * CIN;

    for (int kci = 0; kci < NCHUNK; ++kci) {
        const int kc0 = kci * KC;
        for (int u0 = 0; u0 < FH; u0 += USTAGE) {
            __syncthreads();
            if (u0 == 0) {
                // Stage the input tile (all rows, this channel chunk), with
                // virtual zero padding and zero fill past the data.
#if (KC % 4 == 0) && (CIN % 4 == 0)
                for (int e = tid * 4; e < TR * ROWE; e += NTHREADS * 4) {
                    const int r = e / ROWE, q = e % ROWE;
                    const int tc = q / KC, k = q % KC;
                    const int ii = oi0 + r - PADH, jj = oj0 + tc - PADW, ch = kc0 + k;
                    f32x4 v = {0.f, 0.f, 0.f, 0.f};
                    if (ii >= 0 && ii < HI && jj >= 0 && jj < WI && ch < CIN)
                        v = *(const f32x4*)(I + ibase + ((long)ii * WI + jj) * CIN + ch);
                    elem_t* dst = tile + r * ROWS + q;
                    dst[0] = to_elem(v[0]); dst[1] = to_elem(v[1]);
                    dst[2] = to_elem(v[2]); dst[3] = to_elem(v[3]);
                }
#else
                for (int e = tid; e < TR * ROWE; e += NTHREADS) {
                    const int r = e / ROWE, q = e % ROWE;
                    const int tc = q / KC, k = q % KC;
                    const int ii = oi0 + r - PADH, jj = oj0 + tc - PADW, ch = kc0 + k;
                    float v = 0.f;
                    if (ii >= 0 && ii < HI && jj >= 0 && jj < WI && ch < CIN)
                        v = I[ibase + ((long)ii * WI + jj) * CIN + ch];
                    tile[r * ROWS + q] = to_elem(v);
                }
#endif
            }
            // Stage filter rows u0 .. u0+USTAGE-1 as B slices [col][kr].
            for (int e = tid; e < USTAGE * NCOL * KR; e += NTHREADS) {
                const int uu = e / (NCOL * KR);
                const int rem = e % (NCOL * KR);
                const int col = rem / KR, kr = rem % KR;
                const int s = col / CB, c = col % CB;
                const int vp = kr / KC, k = kr % KC;
                const int v = vp - s, u = u0 + uu, cc = c0 + c, ch = kc0 + k;
                elem_t val = 0;
                if (u < FH && kr < KRRAW && v >= 0 && v < FW && cc < COUT && ch < CIN)
                    val = Wt[(((long)cc * FH + u) * FW + v) * CIN + ch];
                wsl[(uu * NCOL + col) * WRS + kr] = val;
            }
            __syncthreads();

#pragma unroll 1
            for (int uu = 0; uu < USTAGE; ++uu) {
                const int u = u0 + uu;
                if (u >= FH) break;
                const elem_t* arow[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    arow[mt] = tile + (wm * MT + mt + u) * ROWS + S * l32 * KC + h * HALF;
                const elem_t* brow[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    brow[nt] = wsl + (uu * NCOL + (wn * NT + nt) * 32 + l32) * WRS + h * HALF;
#if DT == 0
#pragma unroll
                for (int t = 0; t < HALF; t += 4) {
                    f32x4 av[MT], bv[NT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
#if AV == 4
                        av[mt] = *(const f32x4*)(arow[mt] + t);
#elif AV == 2
                        const float2 p0 = *(const float2*)(arow[mt] + t);
                        const float2 p1 = *(const float2*)(arow[mt] + t + 2);
                        av[mt][0] = p0.x; av[mt][1] = p0.y; av[mt][2] = p1.x; av[mt][3] = p1.y;
#else
                        av[mt][0] = arow[mt][t]; av[mt][1] = arow[mt][t + 1];
                        av[mt][2] = arow[mt][t + 2]; av[mt][3] = arow[mt][t + 3];
#endif
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) bv[nt] = *(const f32x4*)(brow[nt] + t);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt)
                                acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                    av[mt][q], bv[nt][q], acc[mt][nt], 0, 0, 0);
                }
#else
#pragma unroll
                for (int t = 0; t < HALF; t += 8) {
                    u16x8 av[MT], bv[NT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
#if AV == 8
                        av[mt] = *(const u16x8*)(arow[mt] + t);
#elif AV == 4
                        const u16x4 p0 = *(const u16x4*)(arow[mt] + t);
                        const u16x4 p1 = *(const u16x4*)(arow[mt] + t + 4);
#pragma unroll
                        for (int q = 0; q < 4; ++q) { av[mt][q] = p0[q]; av[mt][q + 4] = p1[q]; }
#else
#pragma unroll
                        for (int q = 0; q < 8; ++q) av[mt][q] = arow[mt][t + q];
#endif
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) bv[nt] = *(const u16x8*)(brow[nt] + t);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
#if DT == 1
                            acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, av[mt]), __builtin_bit_cast(bf16x8, bv[nt]),
                                acc[mt][nt], 0, 0, 0);
#else
                            acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(f16x8, av[mt]), __builtin_bit_cast(f16x8, bv[nt]),
                                acc[mt][nt], 0, 0, 0);
#endif
                        }
                }
#endif
            }
        }
    }

    // Epilogue.  32x32 accumulator layout: lane l, register r holds
    // row 8*(r/4) + 4*(l/32) + r%4 (base pixel) and column l%32.
    const long obase = (long)b * HO * WO * COUT;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int col = (wn * NT + nt) * 32 + l32;
        const int s = col / CB, cc = c0 + col % CB;
#if DT != 0
        const float us = (cc < COUT) ? UNSCALE[cc] : 0.f;
#endif
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int oi = oi0 + wm * MT + mt;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = 8 * (r >> 2) + 4 * h + (r & 3);
                const int oj = oj0 + S * m + s;
                if (oi < HO && oj < WO && cc < COUT) {
#if DT == 0
                    O[obase + ((long)oi * WO + oj) * COUT + cc] = acc[mt][nt][r];
#else
                    O[obase + ((long)oi * WO + oj) * COUT + cc] = acc[mt][nt][r] * us;
#endif
                }
            }
        }
    }
}
