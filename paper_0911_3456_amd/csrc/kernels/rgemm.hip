// Implicit-GEMM valid correlation on the matrix cores with the filter
// operand streamed straight into registers.
//
//   O[b,i,j,c] = sum_{u<FH, v<FW, k<CIN} Ipad[b, i+u, j+v, k] * Wt[c, u, v, k]
//
// (Ipad: the input I[b][HI][WI][CIN] with PADH/PADW rows/columns of virtual
// zeros on every side.)  Same GEMM view as the LDS-staged kernel: rows =
// output pixels, columns = output channels (filters), contraction over
// (u, v, k).  What differs is where the operands come from.
//
// * The filter bank is first rewritten by fbcorr_pack_frag (below) in the
//   exact order in which the matrix-core instructions consume it: for an
//   MF-filter column tile j, a channel chunk, a filter row u and a step t,
//   the 64 lanes' 16-byte fragments are one contiguous kilobyte.  Each wave
//   loads its own column tiles' fragments from L2 with one 16-byte load per
//   lane per tile and step, PF steps ahead, into a ring of registers.  The
//   filters never pass through LDS, so there is no per-filter-row staging
//   and no barrier inside a channel chunk: a chunk is one uninterrupted run
//   of FH * NSTEP steps of products.
// * The input tile of a channel chunk (with its FH-1 / FW-1 halo) is staged
//   once in LDS as 16-byte cells of PE consecutive channels, NPL = KC/PE
//   planes of cells.  The 16 lanes that read together take 16 consecutive
//   pixel columns of one plane: 256 contiguous bytes.  (gfx950 also pairs
//   lanes l and l+16 of each half-wave: their two 256-byte runs cost no
//   extra cycle only when they start at the same offset modulo 256 bytes,
//   i.e. when the row stride TCP is a multiple of 16 cells for MC = 16;
//   XPADC sets the stride.)
//
// Contraction order.  Within a filter row u and chunk, the run of (v, k)
// pairs (tap-major, FW*KC values, zero-padded to NSTEP*E) is cut into steps
// of E = NKG*PE values, NKG = 64/MF lane groups; lane group g of an
// instruction takes values [E*t + g*PE, E*t + g*PE + PE) of step t.  Run
// position e lies in cell plane (e % KC)/PE, tap e / KC.  For 16-bit
// operands one step is one v_mfma_f32_{32x32x16,16x16x32} (8 values per
// lane); for fp32 it is four v_mfma_f32_{32x32x2,16x16x4}_f32 (value q of the
// lane's cell in product q).  A and B use the same order, so every padding
// value multiplies a zero weight.
//
// Column shift S (narrow outputs).  A workgroup's NCOLW = WN*NT*MF matrix
// columns are S shifts x CB = NCOLW/S output channels: column (s, c)
// computes output column S*j + s of base pixel column j, with filter
// B[(u, v', k), (s, c)] = Wt[c, u, v'-s, k] (zero outside 0 <= v'-s < FW)
// over NTAPF = FW+S-1 taps per filter row; the pack writes each shifted
// copy, and a lane's A run starts at pixel column S*j.
//
// Compile-time constants (FB_<name>):
//   problem  BATCH FH FW CIN COUT HI WI HO WO PADH PADW
//   DT       0 fp32 operands, 1 bf16, 2 fp16 (B pre-scaled and rounded by
//            the pack; UNSCALE[c] multiplies each output)
//   XMOFF    fp16 only: UNSCALE[XMOFF .. XMOFF+255] hold partial maxima of |x|
//            (fbcorr_absmax); when the input reaches 2^15 it is scaled by
//            2^-k while staged (max |x| * 2^-k < 2^15, inside the fp16
//            range) and the outputs by 2^k -- both exact powers of two
//   tiling   MF (32 or 16: MFMA tile), KC (channels per chunk: PE times a
//            power of two), S (column shift, above), MR (rows of an
//            MF-pixel tile), MT NT (tiles per
//            wave), WM WN (waves), PF (filter-fragment ring depth in steps),
//            XPADC (LDS row padding in cells), WPE (waves per SIMD the
//            register budget is sized for), UNR (1: unroll the step loop
//            completely), XCDMAP (XCD-aware workgroup order), NTS (1:
//            non-temporal output stores), STE (1: tiles of whole column
//            blocks store through LDS as 16-byte vectors, pixels past the
//            image edge skipped)
//   naming   KNAME   EPILOGUE(v, c) as in the LDS-staged kernel
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#ifdef FB_INJECT_ERROR
#error "injected code-generation failure (test hook)"
#endif

typedef float rg_f32x4 __attribute__((ext_vector_type(4)));
typedef float rg_f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int rg_u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 rg_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 rg_f16x8 __attribute__((ext_vector_type(8)));

#define FH FB_FH
#define FW FB_FW
#define CIN FB_CIN
#define COUT FB_COUT
#define DT FB_DT
#define KC FB_KC
#ifdef FB_MF
#define MF FB_MF
#else
#define MF 32
#endif

#if DT == 0
#define PE 4                      // channels per 16-byte cell
#else
#define PE 8
#endif
#ifdef FB_S
#define S FB_S
#else
#define S 1
#endif
#define NKG (64 / MF)             // lane groups of one instruction
#define E (NKG * PE)              // contraction values per step
#define NPL (KC / PE)             // cell planes per channel chunk
#define NTAPF (FW + S - 1)        // taps of one filter row with the column shifts
#define NSTEP ((NTAPF * KC + E - 1) / E)   // steps per filter row and chunk
#define NTAPS ((NSTEP * E) / KC)        // taps covered, padding included
#define NCHUNK ((CIN + KC - 1) / KC)
#define KSTEPS (FH * NSTEP)             // steps per chunk
#ifdef FB_PF
#define KSTEPS2 (KSTEPS + FB_PF)        // packed steps per chunk: PF zero steps after the real ones
#endif

static_assert(MF == 32 || MF == 16, "MFMA tiles are 32x32 or 16x16");
static_assert(KC % PE == 0 && ((KC / PE) & (KC / PE - 1)) == 0, "KC must be PE times a power of two");

// Cell offset (plane * plane_cells + tap) of run position e.
#define RUN_PLANE(e) (((e) % KC) / PE)
#define RUN_TAP(e) ((e) / KC)

// ------------------------------------------------------------------ pack
#ifdef FB_PACK_FRAG
// One workgroup per column pc of the packed bank: whole column blocks of
// the correlation kernel, NCOLW columns each, column (s, c) of a block
// holding filter c shifted by s taps (columns of filters at or past COUT
// are zero).  Layout: 16-byte cell ((j*NCHUNK + chunk)*KSTEPS2 + u*NSTEP +
// t)*64 + lane for column tile j = pc / MF, lane = MF*g + pc%MF.  16-bit
// operands: e_c = floor(log2 max|w[c]|), values scaled by 2^-e_c (exact)
// and rounded to nearest even, unscale[pc] = 2^e_c (an all-zero filter gets
// e_c = 0).  FB_FLIP: the
// filters are those of the input-gradient correlation, read from the
// forward bank w[CIN][FH][FW][COUT] flipped in (u, v) with the channel axes
// exchanged.
extern "C" __global__ void __launch_bounds__(256)
fbcorr_pack_frag(const float* __restrict__ w, rg_u32x4* __restrict__ bp, float* __restrict__ unscale)
{
    // items: (chunk, filter row, tap slot, plane), plane fastest; a thread
    // takes items tid, tid + 256, ...  When they fit (HELD), every item's
    // values are loaded once, all loads in flight together, and kept for
    // both the maximum and the packing; otherwise they are read twice.
    constexpr int ITEMS = NCHUNK * FH * NTAPS * NPL;
    constexpr int PER = (ITEMS + 255) / 256;
    constexpr bool HELD = PER * PE <= 64;
    const int pc = blockIdx.x;
    const int j = pc / MF, col = pc % MF;
#ifdef FB_NCOLW
    // column (s, c) of its block
    const int sh = (pc % FB_NCOLW) / (FB_NCOLW / S);
    const int c = (pc / FB_NCOLW) * (FB_NCOLW / S) + (pc % FB_NCOLW) % (FB_NCOLW / S);
#else
    const int sh = 0, c = pc;
#endif
    const bool real = c < COUT;
    auto load_item = [&](int e, float* vals) {
        const int p = e % NPL;
        int r = e / NPL;
        const int vv = r % NTAPS;
        r /= NTAPS;
        const int u = r % FH, kci = r / FH;
        const int ch0 = kci * KC + p * PE;
        const int vf = vv - sh;                   // filter tap of this (shifted) column
        const bool ok = e < ITEMS && real && vf >= 0 && vf < FW;
#if !defined(FB_FLIP) && CIN % PE == 0
        // PE consecutive channels of one tap: contiguous in w[c][u][v][:]
        if (ok && ch0 < CIN) {
            const float* src = w + (((long)c * FH + u) * FW + vf) * CIN + ch0;
#pragma unroll
            for (int q = 0; q < PE; q += 4) {
                const rg_f32x4 x4 = *(const rg_f32x4*)(src + q);
                vals[q] = x4[0]; vals[q + 1] = x4[1]; vals[q + 2] = x4[2]; vals[q + 3] = x4[3];
            }
        } else {
#pragma unroll
            for (int i = 0; i < PE; ++i) vals[i] = 0.f;
        }
#else
#pragma unroll
        for (int i = 0; i < PE; ++i) {
            const int ch = ch0 + i;
#ifdef FB_FLIP
            vals[i] = (ok && ch < CIN) ? w[(((long)ch * FH + (FH - 1 - u)) * FW + (FW - 1 - vf)) * COUT + c] : 0.f;
#else
            vals[i] = (ok && ch < CIN) ? w[(((long)c * FH + u) * FW + vf) * CIN + ch] : 0.f;
#endif
        }
#endif
    };
    auto store_item = [&](int e, const float* vals, float sc) {
        if (e >= ITEMS) return;
        const int p = e % NPL;
        int r = e / NPL;
        const int vv = r % NTAPS;
        r /= NTAPS;
        const int u = r % FH, kci = r / FH;
        const int el = vv * KC + p * PE;          // position in the row's run
        const int t = el / E, g = (el % E) / PE;
        rg_u32x4 cell;
#if DT == 0
        (void)sc;
        cell = __builtin_bit_cast(rg_u32x4, (rg_f32x4){vals[0], vals[1], vals[2], vals[3]});
#else
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float lo_v = vals[2 * i] * sc, hi_v = vals[2 * i + 1] * sc;   // exact: power of two
#if DT == 1
            const unsigned lo = __builtin_bit_cast(unsigned short, (__bf16)lo_v);
            const unsigned hi = __builtin_bit_cast(unsigned short, (__bf16)hi_v);
#else
            const unsigned lo = __builtin_bit_cast(unsigned short, (_Float16)lo_v);
            const unsigned hi = __builtin_bit_cast(unsigned short, (_Float16)hi_v);
#endif
            cell[i] = lo | (hi << 16);
        }
#endif
        bp[(((long)j * NCHUNK + kci) * KSTEPS2 + u * NSTEP + t) * 64 + g * MF + col] = cell;
    };

    float held[HELD ? PER : 1][PE];
    float m = 0.f;
    if (HELD) {
#pragma unroll
        for (int i = 0; i < (HELD ? PER : 1); ++i) load_item(threadIdx.x + i * 256, held[i]);
#pragma unroll
        for (int i = 0; i < (HELD ? PER : 1); ++i)
#pragma unroll
            for (int q = 0; q < PE; ++q) m = fmaxf(m, fabsf(held[i][q]));
    } else {
        for (int e = threadIdx.x; e < ITEMS; e += 256) {
            float vals[PE];
            load_item(e, vals);
#pragma unroll
            for (int q = 0; q < PE; ++q) m = fmaxf(m, fabsf(vals[q]));
        }
    }
    float sc = 1.0f;
#if DT != 0
    // e_c = floor(log2 max|w[c]|) over the filter's values (the padding
    // zeros change nothing)
    __shared__ float red[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int ex = 0;
    if (m > 0.f) {
        (void)frexpf(m, &ex);     // m = f * 2^ex, f in [0.5, 1)
        ex -= 1;                  // floor(log2 m)
    }
    sc = ldexpf(1.0f, -ex);
    if (threadIdx.x == 0) unscale[pc] = real ? ldexpf(1.0f, ex) : 0.f;
#else
    (void)unscale;
    (void)m;
#endif
    if (HELD) {
#pragma unroll
        for (int i = 0; i < (HELD ? PER : 1); ++i) store_item(threadIdx.x + i * 256, held[i], sc);
    } else {
        for (int e = threadIdx.x; e < ITEMS; e += 256) {
            float vals[PE];
            load_item(e, vals);
            store_item(e, vals, sc);
        }
    }
    // the zero steps after each chunk (read by the ring's last refills)
    for (int e = threadIdx.x; e < NCHUNK * (KSTEPS2 - KSTEPS) * NKG; e += 256) {
        const int g = e % NKG, st = (e / NKG) % (KSTEPS2 - KSTEPS), kci = e / (NKG * (KSTEPS2 - KSTEPS));
        const rg_u32x4 z = {0u, 0u, 0u, 0u};
        bp[(((long)j * NCHUNK + kci) * KSTEPS2 + KSTEPS + st) * 64 + g * MF + col] = z;
    }
}
#endif  // FB_PACK_FRAG

// ---------------------------------------------------------------- correlation
#ifndef FB_PACK_FRAG
#define BATCH FB_BATCH
#define HI FB_HI
#define WI FB_WI
#define HO FB_HO
#define WO FB_WO
#define PADH FB_PADH
#define PADW FB_PADW
#define MR FB_MR
#define MT FB_MT
#define NT FB_NT
#define WM FB_WM
#define WN FB_WN
#define PF FB_PF
#define XPADC FB_XPADC
#ifdef FB_WPE
#define WPE FB_WPE
#else
#define WPE 2
#endif

#define NREG (MF * MF / 64)           // accumulator registers per tile
#define MC (MF / MR)                  // pixel columns of a tile
#define TH (WM * MT * MR)             // output rows per workgroup
#define TWO (S * MC)                  // output columns per workgroup
#define NCOLW (WN * NT * MF)          // matrix columns per workgroup
#define CB (NCOLW / S)                // filters per workgroup
#define TR (TH + FH - 1)              // tile rows
#define TC (S * (MC - 1) + NTAPS)     // tile columns any lane reads
#define TCP (TC + XPADC)              // tile row stride in cells
#define PLANE (TR * TCP)              // cells per plane
#define TILE_CELLS (NPL * PLANE)
#define NTHREADS (WM * WN * 64)
#if defined(FB_STE) && FB_STE
// Stores through LDS: per wave, one pixel tile's worth of its columns as
// rows of NT*MF floats (+8: the two lane groups' rows land on different
// banks), read back as 16-byte vectors
#define STE 1
#define SROW (NT * MF + 8)
#define SWAVE (MF * SROW)
#define STE_CELLS ((WM * WN * SWAVE + 3) / 4)
#define LDS_CELLS (TILE_CELLS > STE_CELLS ? TILE_CELLS : STE_CELLS)
#else
#define STE 0
#define LDS_CELLS TILE_CELLS
#endif
// tile cells staged per thread and batch (all of them when they are few)
#define SCELLS ((NPL * TR * TC + NTHREADS - 1) / NTHREADS)
#define SB (SCELLS < (DT == 0 ? 16 : 8) ? SCELLS : (DT == 0 ? 16 : 8))

static_assert(MF % MR == 0, "MR must divide MF");
static_assert(NCOLW % S == 0, "the columns must split evenly into shifts");
static_assert(!STE || S == 1, "stores through LDS need unshifted columns");
static_assert(PF >= 1, "ring depth");
static_assert(CIN % PE == 0 || KC == PE, "partial cells need KC == PE");

template <bool V> struct RgBool { static constexpr bool value = V; };

#if MF == 32
typedef rg_f32x16 rg_acc;
#else
typedef rg_f32x4 rg_acc;
#endif

// fp16 input scale exponent k >= 0 from the 256 partial maxima of |x| (four
// per lane of the wave, combined by shuffles; the same in every lane).
__device__ __forceinline__ int rg_input_scale_exp(const float* __restrict__ UNSCALE) {
#if DT == 2 && defined(FB_XMOFF)
    const float* pm = UNSCALE + FB_XMOFF + 4 * (threadIdx.x & 63);
    float m = fmaxf(fmaxf(pm[0], pm[1]), fmaxf(pm[2], pm[3]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    int e = 0;
    if (m >= 32768.f) (void)frexpf(m, &e);    // m < 2^e
    return e > 15 ? e - 15 : 0;
#else
    (void)UNSCALE;
    return 0;
#endif
}

// One 16-byte cell of PE values (scaled by xs, exact) in the operand type.
__device__ __forceinline__ rg_u32x4 rg_cell(const float* v, const float xs) {
    rg_u32x4 c;
#if DT == 0
    (void)xs;
    c = __builtin_bit_cast(rg_u32x4, (rg_f32x4){v[0], v[1], v[2], v[3]});
#else
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#if DT == 1
        (void)xs;
        const unsigned lo = __builtin_bit_cast(unsigned short, (__bf16)v[2 * i]);      // nearest even
        const unsigned hi = __builtin_bit_cast(unsigned short, (__bf16)v[2 * i + 1]);
#else
        const unsigned lo = __builtin_bit_cast(unsigned short, (_Float16)(v[2 * i] * xs));
        const unsigned hi = __builtin_bit_cast(unsigned short, (_Float16)(v[2 * i + 1] * xs));
#endif
        c[i] = lo | (hi << 16);
    }
#endif
    return c;
}

// acc += A * B for one step of one (pixel tile, column tile) pair.
__device__ __forceinline__ void rg_mma(rg_acc& acc, const rg_u32x4 a, const rg_u32x4 b) {
#if DT == 0
    const rg_f32x4 af = __builtin_bit_cast(rg_f32x4, a);
    const rg_f32x4 bf = __builtin_bit_cast(rg_f32x4, b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#if MF == 32
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af[q], bf[q], acc, 0, 0, 0);
#else
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q], bf[q], acc, 0, 0, 0);
#endif
    }
#elif DT == 1 && MF == 32
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(rg_bf16x8, a), __builtin_bit_cast(rg_bf16x8, b),
                                                  acc, 0, 0, 0);
#elif DT == 1
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(rg_bf16x8, a), __builtin_bit_cast(rg_bf16x8, b),
                                                  acc, 0, 0, 0);
#elif MF == 32
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(rg_f16x8, a), __builtin_bit_cast(rg_f16x8, b),
                                                 acc, 0, 0, 0);
#else
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(rg_f16x8, a), __builtin_bit_cast(rg_f16x8, b),
                                                 acc, 0, 0, 0);
#endif
}

extern "C" __global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
FB_KNAME(const float* __restrict__ I, const rg_u32x4* __restrict__ Bp, const float* __restrict__ UNSCALE,
         float* __restrict__ O)
{
    __shared__ rg_u32x4 tile[LDS_CELLS];

    // Workgroup -> (image, column block, tile row, tile column); with XCDMAP
    // each XCD gets a contiguous range (shared halos stay in its L2).
    const int ntx = (WO + TWO - 1) / TWO;
    const int nty = (HO + TH - 1) / TH;
    const int ncb = (COUT + CB - 1) / CB;
    const int total = ntx * nty * ncb * BATCH;
    int lin = blockIdx.x;
#if FB_XCDMAP
    {
        const int q = total / 8, r = total % 8, x = lin % 8;
        lin = x * q + (x < r ? x : r) + lin / 8;
    }
#endif
    const int tx = lin % ntx;
    const int ty = (lin / ntx) % nty;
    const int cblk = (lin / (ntx * nty)) % ncb;
    const int b = lin / (ntx * nty * ncb);
    const int oi0 = ty * TH, oj0 = tx * TWO, c0 = cblk * CB;
    const float* Ib = I + (long)b * HI * WI * CIN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int lr = lane % MF, g = lane / MF;       // tile row (pixel) / lane group
    const int ti = lr / MC, tj = lr % MC;
    // this lane's first cell (step 0, filter row 0, pixel tile 0)
    const int lb = RUN_PLANE(g * PE) * PLANE + (wm * MT * MR + ti) * TCP + S * tj + RUN_TAP(g * PE);
    // this wave's first column tile of the packed bank; column tiles are
    // NCHUNK*KSTEPS2 kilobyte blocks apart (the bank has whole column
    // blocks, so every tile a wave names exists)
    const int j0 = cblk * (NCOLW / MF) + wn * NT;
    const rg_u32x4* bw = Bp + (long)j0 * NCHUNK * KSTEPS2 * 64 + lane;

    rg_acc acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < NREG; ++r) acc[mt][nt][r] = 0.f;

    // fp16: per-tensor input scale 2^-kx (1 unless the input reaches 2^15)
#if DT == 2
    const int kx = rg_input_scale_exp(UNSCALE);
    const float xs = ldexpf(1.f, -kx), ys = ldexpf(1.f, kx);
#else
    const float xs = 1.f, ys = 1.f;
#endif
    (void)ys;

#pragma unroll 1
    for (int kci = 0; kci < NCHUNK; ++kci) {
        const rg_u32x4* bc = bw + (long)kci * KSTEPS2 * 64;
        rg_u32x4 bq[PF][NT];
        // the first PF steps' fragments are in flight while the tile is staged
#pragma unroll
        for (int r = 0; r < PF; ++r)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                bq[r][nt] = bc[((long)nt * NCHUNK * KSTEPS2 + r) * 64];
        if (kci > 0) __syncthreads();        // every wave is done with the previous chunk
        // Stage the chunk's input tile: cell (plane p, row r, column cc) =
        // channels kci*KC + p*PE .. +PE-1 of input pixel (oi0+r-PADH,
        // oj0+cc-PADW); zero outside the image and past CIN.  In batches of
        // SB cells per thread, every load of a batch issued before the
        // first conversion (one memory latency per batch, not per cell).
#pragma unroll 1
        for (int e0 = 0; e0 < NPL * TR * TC; e0 += SB * NTHREADS) {
            float v[SB][PE];
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int e = e0 + i * NTHREADS + tid;
                const int p = e % NPL;
                const int rc = e / NPL;
                const int cc = rc % TC, r = rc / TC;
                const int ii = oi0 + r - PADH, jj = oj0 + cc - PADW;
                const int ch = kci * KC + p * PE;
                const bool in = e < NPL * TR * TC && ii >= 0 && ii < HI && jj >= 0 && jj < WI;
                const float* src = Ib + ((long)ii * WI + jj) * CIN + ch;
#if CIN % PE == 0
                if (in && ch < CIN) {
#pragma unroll
                    for (int q = 0; q < PE; q += 4) {
                        const rg_f32x4 x4 = *(const rg_f32x4*)(src + q);
                        v[i][q] = x4[0]; v[i][q + 1] = x4[1]; v[i][q + 2] = x4[2]; v[i][q + 3] = x4[3];
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < PE; ++q) v[i][q] = 0.f;
                }
#else
#pragma unroll
                for (int q = 0; q < PE; ++q) v[i][q] = (in && ch + q < CIN) ? src[q] : 0.f;
#endif
            }
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int e = e0 + i * NTHREADS + tid;
                const int p = e % NPL;
                const int rc = e / NPL;
                const int cc = rc % TC, r = rc / TC;
                if (e < NPL * TR * TC) tile[(p * TR + r) * TCP + cc] = rg_cell(v[i], xs);
            }
        }
        __syncthreads();

        // cell offset of step s relative to the lane's first cell
        auto step_off = [](int s) -> int {
            const int u = s / NSTEP, t = s % NSTEP;
            return RUN_PLANE(E * t) * PLANE + RUN_TAP(E * t) + u * TCP;
        };
        // A fragments one step ahead of the products that use them
        rg_u32x4 a[2][MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[0][mt] = tile[lb + mt * MR * TCP];

        // One step: read the next step's A fragments, the products of this
        // one, then refill this ring slot with the fragments PF steps ahead
        // (the packed bank has PF zero steps after each chunk, so the refill
        // needs no bounds test; nor does the A read, whose step is clamped).
        auto step = [&](const int s, const int r, const int ab) {
            const int sn = s + 1 < KSTEPS ? s + 1 : KSTEPS - 1;
            const int so = step_off(sn);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[ab ^ 1][mt] = tile[lb + so + mt * MR * TCP];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) rg_mma(acc[mt][nt], a[ab][mt], bq[r][nt]);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bq[r][nt] = bc[((long)nt * NCHUNK * KSTEPS2 + s + PF) * 64];
            // Keep this order (LDS reads, products, refill loads) and keep
            // each step's instructions within the step: left free, the
            // scheduler sinks the refills next to their use, which leaves
            // the ring one step deep.
            __builtin_amdgcn_sched_group_barrier(0x100, MT, 0);        // LDS reads
            __builtin_amdgcn_sched_group_barrier(0x008, MT * NT * (DT == 0 ? 4 : 1), 0);   // products
            __builtin_amdgcn_sched_group_barrier(0x020, NT, 0);        // global loads
            __builtin_amdgcn_sched_barrier(0);
        };
        // whole groups of 2*PF steps (ring slot and A buffer repeat with
        // that period), then the remainder, unrolled
        constexpr int G = 2 * PF;
#if defined(FB_UNR) && FB_UNR
#pragma unroll
#else
#pragma unroll 1
#endif
        for (int base = 0; base < KSTEPS / G * G; base += G) {
#pragma unroll
            for (int r2 = 0; r2 < G; ++r2) step(base + r2, r2 % PF, r2 & 1);
        }
#pragma unroll
        for (int r2 = 0; r2 < KSTEPS % G; ++r2) step(KSTEPS / G * G + r2, r2 % PF, r2 & 1);
    }

    // Epilogue.  Accumulator layouts: 32x32 -- lane l, register r holds tile
    // row 8*(r/4) + 4*(l/32) + r%4 and column l%32; 16x16 -- row 4*(l/16) + r
    // and column l%16.  Workgroups whose tile lies inside the output store
    // without per-element bounds tests.
    float* const Ob = O + (long)b * HO * WO * COUT;
    const bool interior = oi0 + TH <= HO && oj0 + TWO <= WO && c0 + CB <= COUT;
    auto store_all = [&](auto checked) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int col = (wn * NT + nt) * MF + lr;       // matrix column: (shift, filter)
            const int sh = col / CB, cc = c0 + col % CB;
#if DT != 0
            const float us = (!decltype(checked)::value || cc < COUT) ? UNSCALE[cblk * NCOLW + col] * ys : 0.f;   // exact: powers of two
#endif
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int r = 0; r < NREG; ++r) {
#if MF == 32
                    const int m = 8 * (r >> 2) + 4 * g + (r & 3);
#else
                    const int m = 4 * g + r;
#endif
                    const int oi = oi0 + (wm * MT + mt) * MR + m / MC;
                    const int oj = oj0 + S * (m % MC) + sh;
                    if (!decltype(checked)::value || (oi < HO && oj < WO && cc < COUT)) {
#if DT == 0
                        float val = acc[mt][nt][r];
#else
                        float val = acc[mt][nt][r] * us;
#endif
#ifdef FB_EPILOGUE
                        val = FB_EPILOGUE(val, cc);
#endif
                        // unsigned 32-bit offset from the image's base: a
                        // scalar base plus a vector offset per store
                        float* const dst = Ob + (unsigned)((oi * WO + oj) * COUT + cc);
#if defined(FB_NTS) && FB_NTS
                        // streaming store: the output is not read again here,
                        // and leaving L2 to the filter fragments and input
                        // tiles that every workgroup re-reads
                        __builtin_nontemporal_store(val, dst);
#else
                        *dst = val;
#endif
                    }
                }
            }
        }
    };
#if STE
    if (c0 + CB <= COUT) {
        // Stores through LDS: each pixel tile of the wave's columns goes to
        // the wave's own LDS rows (the input tile is dead once every wave is
        // past its last step) and back out as 16-byte vectors, so that one
        // store instruction writes whole runs of a pixel's channels.  Every
        // channel of the column block exists (COUT is a multiple of 4);
        // pixels past the image edge are skipped per vector.
        __syncthreads();
        float* const sbuf = (float*)tile + wave * SWAVE;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int col = (wn * NT + nt) * MF + lr;
#if DT != 0
                const float us = UNSCALE[cblk * NCOLW + col] * ys;      // exact: powers of two
#endif
#pragma unroll
                for (int r = 0; r < NREG; ++r) {
#if MF == 32
                    const int m = 8 * (r >> 2) + 4 * g + (r & 3);
#else
                    const int m = 4 * g + r;
#endif
#if DT == 0
                    float val = acc[mt][nt][r];
#else
                    float val = acc[mt][nt][r] * us;
#endif
#ifdef FB_EPILOGUE
                    val = FB_EPILOGUE(val, c0 + col);
#endif
                    sbuf[m * SROW + nt * MF + lr] = val;
                }
            }
            // MF rows of NT*MF/4 vectors, 64 per instruction
#pragma unroll
            for (int it = lane; it < MF * NT * MF / 4; it += 64) {
                const int m = it / (NT * MF / 4), c4 = it % (NT * MF / 4);
                const rg_f32x4 v = *(const rg_f32x4*)(sbuf + m * SROW + c4 * 4);
                const int oi = oi0 + (wm * MT + mt) * MR + m / MC;
                const int oj = oj0 + m % MC;
                rg_f32x4* const dst =
                    (rg_f32x4*)(Ob + (unsigned)((oi * WO + oj) * COUT + c0 + wn * NT * MF + c4 * 4));
                if (interior || (oi < HO && oj < WO)) {
#if defined(FB_NTS) && FB_NTS
                    __builtin_nontemporal_store(v, dst);
#else
                    *dst = v;
#endif
                }
            }
        }
    } else {
        store_all(RgBool<true>{});
    }
#else
    if (interior) store_all(RgBool<false>{});
    else store_all(RgBool<true>{});
#endif
}
#endif  // !FB_PACK_FRAG
