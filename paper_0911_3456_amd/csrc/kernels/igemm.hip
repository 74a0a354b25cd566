// Implicit-GEMM valid correlation on the CDNA matrix cores (MFMA).
//
//   O[b,i,j,c] = sum_{u<FH, v<FW, k<CIN} Ipad[b, i+u, j+v, k] * Wt[c, u, v, k]
//
// where Ipad is the input I[b][HI][WI][CIN] with PADH/PADW rows/columns of
// virtual zeros on every side.  With I = x, Wt = w and no padding this is the
// forward filter-bank correlation of Sec. 6.2; with I = dy, Wt = w flipped in
// (u, v) and transposed n <-> d, and padding (FH-1, FW-1), it is the input
// gradient.  GEMM view: rows = output pixels, columns = output channels,
// contraction over (u, v, k).  A (the im2col matrix) is never materialised:
// for a fixed filter row u the (v, k) pairs of one output pixel are one
// contiguous run of FW*KC values in the LDS input tile, so each lane reads
// its A fragment straight from the staged tile.
//
// Tiles.  A 32-row MFMA tile is 32 "base pixels" laid out as MR rows x MC
// columns (MC = 32/MR).  Column-shift packing: when COUT is smaller than the
// 32 MFMA columns, a column is a pair (c, s), s < S, computing output column
// S*tj + s for base pixel column tj; the contraction then runs over FW+S-1
// taps per filter row with B[(u, v', k), (c, s)] = Wt[c, u, v'-s, k] (zero
// outside 0 <= v'-s < FW).  A wave holds MT x NT tiles; WM x WN waves cover
// the workgroup's output tile; KS groups of such waves split the contraction
// (each group owns its own LDS buffers and a contiguous range of (channel
// chunk, filter-row stage) units) and add their accumulators in a fixed
// order at the end.  Filter slices are double-buffered in LDS and the next
// slice is fetched into registers while the current one is consumed
// (pre-fetching and software pipelining, Sec. 6.2).
//
// Compile-time constants (Sec. 4.2 "hardcoding", Sec. 5.3 keyword
// substitution), passed as FB_<name>:
//   problem  BATCH FH FW CIN COUT HI WI HO WO PADH PADW
//   tiling   KC (channels per chunk)  S (column shift)  MR (tile rows)
//            MT NT (tiles per wave)  WM WN (waves)  KS (contraction split)
//            USTAGE (filter rows per stage)  XPAD WPAD (LDS row padding)
//            XCDMAP (XCD-aware workgroup order)
//   type     DT: 0 = fp32 operands (v_mfma 32x32x2 f32), 1 = bf16, 2 = fp16
//            (32x32x16 with 8 operands per lane; Wt is then pre-scaled and
//            pre-rounded 16-bit and UNSCALE[c] multiplies each output)
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
#define MR FB_MR
#define MT FB_MT
#define NT FB_NT
#define WM FB_WM
#define WN FB_WN
#define KS FB_KS
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

#define MC (32 / MR)              // base-pixel columns of one MFMA tile
#define GWAVES (WM * WN)          // waves per contraction group
#define NTHREADS (GWAVES * KS * 64)
#define GTHREADS (GWAVES * 64)
#define TH (WM * MT * MR)         // output rows per workgroup
#define TWO (S * MC)              // output columns per workgroup
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
#define ROWE ((MC - 1) * S * KC + KR)   // tile row elements any lane may read
#define ROWS (ROWE + XPAD)              // tile row stride
#define WRS (KR + WPAD)                 // filter-slice row stride
#define TILE_ELEMS (((TR * ROWS) + 7) / 8 * 8)
#define WSL_ELEMS (USTAGE * NCOL * WRS)
#define NCHUNK ((CIN + KC - 1) / KC)
#define NUS ((FH + USTAGE - 1) / USTAGE)      // filter-row stages per chunk
#define NUNITS (NCHUNK * NUS)                 // contraction units
#define UPG ((NUNITS + KS - 1) / KS)          // units per group
#define GROUP_ELEMS (((TILE_ELEMS + 2 * WSL_ELEMS) + 7) / 8 * 8)
// filter-slice staging: groups of 4 consecutive kr (same tap, 4 channels)
#define WVEC ((KC % 4 == 0 && CIN % 4 == 0) ? 4 : 1)
#define WITEMS (USTAGE * NCOL * (KR / WVEC))
#define WPER ((WITEMS + GTHREADS - 1) / GTHREADS)

#if DT == 0
typedef float elem_t;
#define ESZ 4
#else
typedef unsigned short elem_t;    // raw 16-bit patterns
#define ESZ 2
#endif
// the split-K reduction reuses the LDS of groups 1..KS-1 (fp32 accumulators)
#define RED_FLOATS ((KS - 1) * GWAVES * MT * NT * 16 * 64)
#define LDS_ELEMS_LOOP (KS * GROUP_ELEMS)
#define LDS_BYTES_LOOP (LDS_ELEMS_LOOP * ESZ)
#define LDS_BYTES ((LDS_BYTES_LOOP > RED_FLOATS * 4) ? LDS_BYTES_LOOP : RED_FLOATS * 4)

// A-read vector width (elements) from the lane-to-lane stride S*KC.
#if DT == 0
#define AV (((S * KC) % 4 == 0) ? 4 : (((S * KC) % 2 == 0) ? 2 : 1))
#else
#define AV (((S * KC) % 8 == 0) ? 8 : (((S * KC) % 4 == 0) ? 4 : (((S * KC) % 2 == 0) ? 2 : 1)))
#endif

static_assert(32 % MR == 0, "MR must divide 32");
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

#if DT == 0
typedef f32x4 wvec_t;                     // 4 fp32 filter values
#else
typedef u16x4 wvec_t;                     // 4 16-bit filter values
#endif

// One staged filter slice item: 4 (or 1) consecutive kr of one column.
__device__ __forceinline__ void w_item(int e, int kc0, int u0, int c0, int& dst, bool& ok, long& src) {
    const int per_col = KR / WVEC;
    const int uu = e / (NCOL * per_col);
    const int rem = e % (NCOL * per_col);
    const int col = rem / per_col;
    const int kr = (rem % per_col) * WVEC;
    const int s = col / CB, c = col % CB;
    const int vp = kr / KC, k = kr % KC;
    const int v = vp - s, u = u0 + uu, cc = c0 + c, ch = kc0 + k;
    ok = (u < FH && kr < KRRAW && v >= 0 && v < FW && cc < COUT && ch < CIN);
    src = ((((long)cc * FH + u) * FW + v) * CIN + ch);
    dst = (uu * NCOL + col) * WRS + kr;
}

// The (chunk, stage) of unit q.
__device__ __forceinline__ void unit_of(int q, int& kci, int& us) {
    kci = q / NUS;
    us = q % NUS;
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
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[LDS_BYTES];
    elem_t* const lds = (elem_t*)lds_raw;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int kg = wave / GWAVES;             // contraction group
    const int gw = wave % GWAVES;             // wave within the group
    const int gtid = tid % GTHREADS;          // thread within the group
    const int wm = gw % WM;
    const int wn = gw / WM;
    const int l32 = lane & 31;
    const int h = lane >> 5;
    const int ti = l32 / MC, tj = l32 % MC;   // this lane's base pixel in a tile

    elem_t* const tile = lds + kg * GROUP_ELEMS;
    elem_t* const wsl0 = tile + TILE_ELEMS;

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
    const long ibase = (long)b * HI * WI * CIN;

    f32x16 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mt][nt][r] = 0.0f;

    // Stage the group's input tile for a channel chunk (virtual zero padding,
    // zero fill past the data).
    auto load_tile = [&](int kc0) {
#if (KC % 4 == 0) && (CIN % 4 == 0)
        for (int e = gtid * 4; e < TR * ROWE; e += GTHREADS * 4) {
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
        for (int e = gtid; e < TR * ROWE; e += GTHREADS) {
            const int r = e / ROWE, q = e % ROWE;
            const int tc = q / KC, k = q % KC;
            const int ii = oi0 + r - PADH, jj = oj0 + tc - PADW, ch = kc0 + k;
            float v = 0.f;
            if (ii >= 0 && ii < HI && jj >= 0 && jj < WI && ch < CIN)
                v = I[ibase + ((long)ii * WI + jj) * CIN + ch];
            tile[r * ROWS + q] = to_elem(v);
        }
#endif
    };

    // Filter-slice prefetch registers.
    wvec_t wreg[WPER];
    auto fetch_w = [&](int q) {
        int kci, us;
        unit_of(q, kci, us);
#pragma unroll
        for (int i = 0; i < WPER; ++i) {
            const int e = gtid + i * GTHREADS;
            wvec_t v = {};
            if (e < WITEMS) {
                int dst; bool ok; long src;
                w_item(e, kci * KC, us * USTAGE, c0, dst, ok, src);
                if (ok) {
#if WVEC == 4
                    v = *(const wvec_t*)(Wt + src);
#else
                    v[0] = Wt[src];
#endif
                }
            }
            wreg[i] = v;
        }
    };
    auto store_w = [&](int q, elem_t* wsl) {
        int kci, us;
        unit_of(q, kci, us);
#pragma unroll
        for (int i = 0; i < WPER; ++i) {
            const int e = gtid + i * GTHREADS;
            if (e < WITEMS) {
                int dst; bool ok; long src;
                w_item(e, kci * KC, us * USTAGE, c0, dst, ok, src);
#if WVEC == 4
                *(wvec_t*)(wsl + dst) = wreg[i];
#else
                wsl[dst] = wreg[i][0];
#endif
            }
        }
    };

    // Units [q0, q1) of this group, processed in lock-step rounds with the
    // other groups (every group runs UPG rounds; units past the end idle).
    const int q0 = kg * UPG;
    const int q1 = (q0 + UPG < NUNITS) ? q0 + UPG : NUNITS;
    int cur_chunk = -1;
    if (q0 < q1) {
        fetch_w(q0);
        store_w(q0, wsl0);
        int kci, us;
        unit_of(q0, kci, us);
        load_tile(kci * KC);
        cur_chunk = kci;
    }
    __syncthreads();

#pragma unroll 1
    for (int rnd = 0; rnd < UPG; ++rnd) {
        const int q = q0 + rnd;
        const bool active = q < q1;
        const bool more = q + 1 < q1;
        if (more) fetch_w(q + 1);
        elem_t* const wsl = wsl0 + (rnd & 1) * WSL_ELEMS;
        if (active) {
            int kci, us;
            unit_of(q, kci, us);
#pragma unroll 1
            for (int uu = 0; uu < USTAGE; ++uu) {
                const int u = us * USTAGE + uu;
                if (u >= FH) break;
                const elem_t* arow[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    arow[mt] = tile + ((wm * MT + mt) * MR + ti + u) * ROWS + S * tj * KC + h * HALF;
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
                    for (int qq = 0; qq < 4; ++qq)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt)
                                acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                    av[mt][qq], bv[nt][qq], acc[mt][nt], 0, 0, 0);
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
                        for (int qq = 0; qq < 4; ++qq) { av[mt][qq] = p0[qq]; av[mt][qq + 4] = p1[qq]; }
#else
#pragma unroll
                        for (int qq = 0; qq < 8; ++qq) av[mt][qq] = arow[mt][t + qq];
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
        if (rnd + 1 < UPG) {
            // The other filter buffer was last read in the previous round,
            // which ended with a barrier: fill it now.
            if (more) store_w(q + 1, wsl0 + ((rnd + 1) & 1) * WSL_ELEMS);
            // A new channel chunk needs a new input tile: wait until every
            // wave is done with the current one first.
            int nk = -1, nus = 0;
            if (more) unit_of(q + 1, nk, nus);
            const bool new_tile = more && nk != cur_chunk;
            if (__syncthreads_or(new_tile)) {
                if (new_tile) {
                    load_tile(nk * KC);
                    cur_chunk = nk;
                }
                __syncthreads();
            }
        }
    }

    const long obase = (long)b * HO * WO * COUT;
#if KS > 1
    // Fixed-order reduction of the KS groups' accumulators through LDS.
    __syncthreads();
    float* const red = (float*)lds_raw;
    if (kg > 0) {
        float* dst = red + (((kg - 1) * GWAVES + gw) * MT * NT * 16) * 64 + lane;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) dst[((mt * NT + nt) * 16 + r) * 64] = acc[mt][nt][r];
    }
    __syncthreads();
    if (kg == 0) {
#pragma unroll 1
        for (int g = 1; g < KS; ++g) {
            const float* src = red + (((g - 1) * GWAVES + gw) * MT * NT * 16) * 64 + lane;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[mt][nt][r] += src[((mt * NT + nt) * 16 + r) * 64];
        }
    }
    if (kg != 0) return;
#endif

    // Epilogue.  32x32 accumulator layout: lane l, register r holds
    // row 8*(r/4) + 4*(l/32) + r%4 (base pixel) and column l%32.
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int col = (wn * NT + nt) * 32 + l32;
        const int s = col / CB, cc = c0 + col % CB;
#if DT != 0
        const float us = (cc < COUT) ? UNSCALE[cc] : 0.f;
#endif
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = 8 * (r >> 2) + 4 * h + (r & 3);
                const int oi = oi0 + (wm * MT + mt) * MR + m / MC;
                const int oj = oj0 + S * (m % MC) + s;
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
