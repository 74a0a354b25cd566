// Exact brute-force nearest-neighbour search over 8-bit patches (Sec. 6.4:
// every target patch against every patch of a neighbour set, exact rather
// than approximate), on the int8 matrix cores of gfx950.
//
//   dist[t] = min_m sum_d (targets[t][d] - neighbors[m][d])^2,
//   idx[t]  = lowest m attaining it.
//
// Pixels are centred, c = p - 128 (a byte XOR 0x80 read as a signed byte),
// which leaves every difference unchanged.  With |t|^2 fixed per target the
// nearest neighbour maximises the exact integer score
//
//   S(t, m) = 2 t.n_m - |n_m|^2          (= |t|^2 - dist(t, m)).
//
// 2t does not fit in int8.  Two exact ways round it, chosen by SPLIT:
//
//  SPLIT = 0  the matrix cores run twice over the same operands from a start
//             value of -|n|^2, which gives S itself.
//  SPLIT = 1  one pass gives the half score s = t.n - floor(|n|^2 / 2), and
//             S = 2s - (|n|^2 odd).  Inside a set of neighbours whose |n|^2
//             have the same parity, s orders them as S does, and neighbours
//             of different parity never have equal S.  The neighbours are
//             partitioned, stably, into an even and an odd class, each padded
//             to whole 16-row tiles, and scanned in that order.
//
// fbnn_norms    |n_m|^2 of every row (4 lanes per row).  SPLIT = 0: the start
//               values -|n|^2 (a sentinel far below any real score for the
//               padding rows of the last tile).  SPLIT = 1: the norms and the
//               number of even norms in each 64-row block.
// fbnn_offsets  (SPLIT = 1) one workgroup: exclusive prefix sum of the block
//               counts (in place), the class sizes, and the padding entries.
// fbnn_scatter  (SPLIT = 1) perm[pos] = m and cneg[pos] = -floor(|n_m|^2/2)
//               at the row's place in its class (lane order inside a block,
//               blocks in order); the odd class starts on a new tile.
// fbnn_scan     one workgroup = a block of targets x a chunk of CH tiles.
//               Batches of BT tiles are staged once per workgroup in LDS
//               (double-buffered, centred on the way in) and shared by its
//               WV waves.  A v_mfma_i32_16x16x64_i8 product of a tile (rows
//               = neighbours) with 16 targets (columns), started from the
//               rows' score terms, gives the (half) score in int32 exactly.
//               Lane l holds target l%16 against rows 4(l/16)..+3 of a tile;
//               it keeps a running maximum over groups of TG tiles and the
//               first group reaching it (a later group replaces it only when
//               strictly greater).  Per scanned range (SPLIT = 1: the even
//               and the odd part of the chunk) the key is (S, then the lower
//               group start); the four lane groups are merged and the chunk's
//               key is written to part[chunk][t].
// fbnn_final    per target: the largest key over all chunks names the first
//               group of TG tiles holding a nearest neighbour (in scan order,
//               which is index order inside a class); its 16 TG rows are
//               re-measured from the bytes and the smallest (distance,
//               index) wins: the lowest-index nearest neighbour.
//
// Compile-time constants (FB_<name>):
//   problem  T (targets)  M (neighbours)  D (bytes per patch, D % 16 == 0)
//   method   SPLIT
//   scan     NT (16-target tiles per wave)  WV (waves per workgroup)
//            CH (tiles per chunk)  BT (tiles per LDS batch)
//            TG (tiles per tracking group, divides BT)  XCDMAP
//   final    FW (waves per workgroup, 1, 2, 4, 8 or 16)  TG  NCHK (chunks)
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#ifdef FB_INJECT_ERROR
#error "injected code-generation failure (test hook)"
#endif

#define T FB_T
#define M FB_M
#define D FB_D
#define SPLIT FB_SPLIT
#define MT ((M + 15) / 16)
#define NB ((M + 63) / 64)           // 64-row blocks
#define KB ((D + 63) / 64)
#if SPLIT
#define MTS (MT + 1)                 // tiles of the partitioned order (two padded classes)
#else
#define MTS MT
#endif

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Score term of padding rows: -2^28 keeps them below every real score, which
// lies in (-2^25, 2^25) for D <= 512 (half scores in (-2^24, 2^24)).
#define NN_PAD_TERM (-(1 << 28))

// Header words in the workspace (SPLIT = 1): [0] even rows, [1] first tile of
// the odd class.
#define HDR_EVEN 0
#define HDR_KODD 1

#ifdef FB_NN_NORMS
// NBW 64-row blocks per workgroup of 256 threads (4 threads per row, one
// block per pass); every row's loads are issued before any is used.
#define NBW 4
extern "C" __global__ void __launch_bounds__(256)
fbnn_norms(const unsigned char* __restrict__ nb, int* __restrict__ nn, int* __restrict__ cnt)
{
    __shared__ int wsum[NBW][4];
    const int q = threadIdx.x & 3;
    int s[NBW];
    long rows[NBW];
#pragma unroll
    for (int bb = 0; bb < NBW; ++bb) {
        const long row = ((long)blockIdx.x * NBW + bb) * 64 + (threadIdx.x >> 2);
        rows[bb] = row;
        int acc = 0;
        if (row < M) {
#pragma unroll
            for (int k = q * 16; k < D; k += 64) {
                const i32x4 v = *(const i32x4*)(nb + row * D + k);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const unsigned x = (unsigned)v[w];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int c = (int)((x >> (8 * j)) & 255u) - 128;
                        acc += c * c;
                    }
                }
            }
        }
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        s[bb] = acc;
    }
#pragma unroll
    for (int bb = 0; bb < NBW; ++bb) {
        const long row = rows[bb];
#if SPLIT
        if (q == 0 && row < M) nn[row] = s[bb];
        const unsigned long long even = __ballot(q == 0 && row < M && (s[bb] & 1) == 0);
        if ((threadIdx.x & 63) == 0) wsum[bb][threadIdx.x >> 6] = __popcll(even);
#else
        // nn is the start-value array here: -|n|^2, sentinel past the last row
        if (q == 0 && row < (long)MT * 16) nn[row] = row < M ? -s[bb] : NN_PAD_TERM;
#endif
    }
#if SPLIT
    __syncthreads();
    if (threadIdx.x < NBW) {
        const long blk = (long)blockIdx.x * NBW + threadIdx.x;
        if (blk < NB) cnt[blk] = wsum[threadIdx.x][0] + wsum[threadIdx.x][1] + wsum[threadIdx.x][2] + wsum[threadIdx.x][3];
    }
#else
    (void)cnt;
    (void)wsum;
#endif
}
#endif

#ifdef FB_NN_OFFSETS
// One workgroup of 1024 threads; cnt[] becomes the exclusive prefix sum.
// Each thread owns PER consecutive counts (16-byte loads and stores when PER
// is a multiple of four); the 1024 segment sums are scanned within each wave
// by shuffles, then across the 16 waves.
#define OPER ((NB + 1023) / 1024)
extern "C" __global__ void __launch_bounds__(1024)
fbnn_offsets(int* __restrict__ cnt, int* __restrict__ hdr, int* __restrict__ perm, int* __restrict__ cneg)
{
    __shared__ int wtot[16];
    __shared__ int tot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long b0 = (long)tid * OPER;
    int s = 0;
#if OPER > 32
    // long segments: summed here, read again below
    for (long b = b0; b < b0 + OPER && b < NB; ++b) s += cnt[b];
#else
    int vals[OPER];
#if OPER % 4 == 0
#pragma unroll
    for (int i = 0; i < OPER; i += 4) {
        i32x4 v = {0, 0, 0, 0};
        if (b0 + i + 3 < NB) {
            v = *(const i32x4*)(cnt + b0 + i);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = (b0 + i + j < NB) ? cnt[b0 + i + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) vals[i + j] = v[j];
    }
#else
#pragma unroll
    for (int i = 0; i < OPER; ++i) vals[i] = (b0 + i < NB) ? cnt[b0 + i] : 0;
#endif
#pragma unroll
    for (int i = 0; i < OPER; ++i) s += vals[i];
#endif
    // inclusive scan of the segment sums: within the wave, then the waves
    int inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(inc, off);
        if (lane >= off) inc += v;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int t = lane < 16 ? wtot[lane] : 0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int v = __shfl_up(t, off);
            if (lane >= off) t += v;
        }
        if (lane < 16) wtot[lane] = t;
        if (lane == 15) tot = t;
    }
    __syncthreads();
    int run = inc - s + (wave > 0 ? wtot[wave - 1] : 0);   // exclusive start of this segment
#if OPER > 32
    for (long b = b0; b < b0 + OPER && b < NB; ++b) {
        const int v = cnt[b];
        cnt[b] = run;
        run += v;
    }
#elif OPER % 4 == 0
#pragma unroll
    for (int i = 0; i < OPER; i += 4) {
        i32x4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) { v[j] = run; run += vals[i + j]; }
        if (b0 + i + 3 < NB) {
            *(i32x4*)(cnt + b0 + i) = v;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) if (b0 + i + j < NB) cnt[b0 + i + j] = v[j];
        }
    }
#else
#pragma unroll
    for (int i = 0; i < OPER; ++i) {
        if (b0 + i < NB) cnt[b0 + i] = run;
        run += vals[i];
    }
#endif
    const int me = tot, mo = M - me;
    const int kodd = (me + 15) / 16;
    if (tid == 0) {
        hdr[HDR_EVEN] = me;
        hdr[HDR_KODD] = kodd;
    }
    // padding of the even class's last tile and everything after the odd class
    for (int p = me + tid; p < kodd * 16; p += 1024) {
        perm[p] = -1;
        cneg[p] = NN_PAD_TERM;
    }
    for (long p = (long)kodd * 16 + mo + tid; p < (long)MTS * 16; p += 1024) {
        perm[p] = -1;
        cneg[p] = NN_PAD_TERM;
    }
}
#endif

#ifdef FB_NN_SCATTER
// One wave per 64-row block, one row per lane.
extern "C" __global__ void __launch_bounds__(64)
fbnn_scatter(const int* __restrict__ nn, const int* __restrict__ off, const int* __restrict__ hdr,
             int* __restrict__ perm, int* __restrict__ cneg)
{
    const int lane = threadIdx.x;
    const long b = blockIdx.x;
    const long row = b * 64 + lane;
    const bool valid = row < M;
    const int v = valid ? nn[row] : 0;
    const bool even = valid && (v & 1) == 0, odd = valid && (v & 1) != 0;
    const unsigned long long me = __ballot(even), mo = __ballot(odd);
    const unsigned long long below = (1ull << lane) - 1ull;
    const long e0 = off[b];
    const long o0 = b * 64 - e0;                    // odd rows in earlier blocks
    long pos = 0;
    if (even) pos = e0 + __popcll(me & below);
    if (odd) pos = (long)hdr[HDR_KODD] * 16 + o0 + __popcll(mo & below);
    if (valid) {
        perm[pos] = (int)row;
        cneg[pos] = -(v >> 1);
    }
}
#endif

#ifdef FB_NN_SCAN
#define NT FB_NT
#define WV FB_WV
#define CH FB_CH
#define BT FB_BT
#define TG FB_TG
#define XCDMAP FB_XCDMAP
#define NTH (WV * 64)
#define TPW (NT * 16)
#define TPG (WV * TPW)
#define TB ((T + TPG - 1) / TPG)
#define NCHK ((MTS + CH - 1) / CH)
#define RS (D + 16)                  // LDS row stride (bytes): 16 bytes of padding
#define SEGR (D / 16)                // 16-byte segments per row
#define NSEG (BT * 16 * SEGR)        // segments per batch
#define LPT ((NSEG + NTH - 1) / NTH) // segments loaded per thread
#define PASSES (SPLIT ? 1 : 2)

static_assert(BT % TG == 0, "tracking groups must tile the LDS batch");

// At least two waves per SIMD caps the kernel at 256 VGPRs, which lets the
// compiler keep the accumulators in ordinary VGPRs (no accumulator-register
// copies before the running maximum).
extern "C" __global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(2)))
fbnn_scan(const unsigned char* __restrict__ tg, const unsigned char* __restrict__ nb,
          const int* __restrict__ perm, const int* __restrict__ cneg, const int* __restrict__ hdr,
          unsigned long long* __restrict__ part)
{
    __shared__ __attribute__((aligned(16))) unsigned char arow[2][BT * 16 * RS];
    __shared__ __attribute__((aligned(16))) int cterm[2][BT * 16];

    int lin = blockIdx.x;
#if XCDMAP
    {   // undo the round-robin over the eight XCDs: the target blocks of one
        // chunk run on one XCD and share its L2 copy of the chunk
        const int total = TB * NCHK, q = total / 8, r = total % 8, x = lin % 8;
        lin = x * q + (x < r ? x : r) + lin / 8;
    }
#endif
    const int tb = lin % TB, chunk = lin / TB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;

    // Target fragments (B operand, column = target), resident for the chunk.
    i32x4 bf[NT][KB];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        int t = tb * TPG + wave * TPW + nt * 16 + col;
        t = t < T ? t : T - 1;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int k0 = kb * 64 + grp * 16;
            i32x4 v = {0, 0, 0, 0};
            if (k0 < D) v = *(const i32x4*)(tg + (long)t * D + k0) ^ (int)0x80808080u;
            bf[nt][kb] = v;
        }
    }

    unsigned long long best[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) best[nt] = 0ull;

    // Batch staging: rows of tiles [k, k + BT) (only tiles < kl are read),
    // global -> registers, then registers -> LDS buffer, centred.
    i32x4 sreg[LPT];
    int creg = 0;
    auto fetch = [&](int k, int kl) {
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int e = tid + i * NTH;
            i32x4 v = {0, 0, 0, 0};
            if (e < NSEG) {
                const int r = e / SEGR, q = e % SEGR;
                const int kt = k + r / 16;
                if (kt < kl) {
                    const long pos = (long)kt * 16 + r % 16;
#if SPLIT
                    const int pr = perm[pos];
                    const long row = pr < 0 ? 0 : pr;   // padding rows lose on their score term
#else
                    const long row = pos < M ? pos : M - 1;
#endif
                    v = *(const i32x4*)(nb + row * D + q * 16);
                }
            }
            sreg[i] = v;
        }
        if (tid < BT * 16 && k + tid / 16 < kl) creg = cneg[(long)k * 16 + tid];
    };
    auto store = [&](int b) {
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int e = tid + i * NTH;
            if (e < NSEG) {
                const int r = e / SEGR, q = e % SEGR;
                *(i32x4*)&arow[b][r * RS + q * 16] = sreg[i] ^ (int)0x80808080u;
            }
        }
        if (tid < BT * 16) cterm[b][tid] = creg;
    };

    // Scan tiles [k0, k1) (cls: parity class for SPLIT = 1, else 0).
    auto scan_range = [&](int k0, int k1, int cls) {
        if (k0 >= k1) return;
        int mx[NT], st[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            mx[nt] = -2147483647 - 1;
            st[nt] = k0;
        }
        fetch(k0, k1);
        store(0);
        __syncthreads();
        int buf = 0;
#pragma unroll 1
        for (int kb0 = k0; kb0 < k1; kb0 += BT) {
            const bool more = kb0 + BT < k1;
            if (more) fetch(kb0 + BT, k1);
#pragma unroll
            for (int g = 0; g < BT; g += TG) {
                if (kb0 + g < k1) {
                    int gm[NT];              // max(running maximum, this group)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) gm[nt] = mx[nt];
#pragma unroll
                    for (int j = 0; j < TG; ++j) {
                        const int tl = g + j;
                        if (kb0 + tl < k1) {
                            i32x4 af[KB];
#pragma unroll
                            for (int kb = 0; kb < KB; ++kb) {
                                const int k0b = kb * 64 + grp * 16;
                                i32x4 v = {0, 0, 0, 0};
                                if (k0b < D) v = *(const i32x4*)&arow[buf][(tl * 16 + col) * RS + k0b];
                                af[kb] = v;
                            }
                            const i32x4 ci = *(const i32x4*)&cterm[buf][tl * 16 + grp * 4];
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt) {
                                i32x4 acc = ci;
#pragma unroll
                                for (int pass = 0; pass < PASSES; ++pass)
#pragma unroll
                                    for (int kb = 0; kb < KB; ++kb)
                                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[kb], bf[nt][kb], acc, 0, 0, 0);
                                gm[nt] = max(max(gm[nt], acc[0]), acc[1]);
                                gm[nt] = max(max(gm[nt], acc[2]), acc[3]);
                            }
                        }
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        st[nt] = gm[nt] != mx[nt] ? kb0 + g : st[nt];
                        mx[nt] = gm[nt];
                    }
                }
            }
            if (more) store(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
        // Key = (exact score S mapped to unsigned order) : (~first row of the
        // group): the unsigned maximum takes the higher S, then the earlier
        // group.
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#if SPLIT
            const int S = 2 * mx[nt] - cls;
#else
            const int S = mx[nt];
#endif
            const unsigned hi = (unsigned)S ^ 0x80000000u;
            const unsigned lo = 0xFFFFFFFFu - (unsigned)st[nt] * 16u;
            const unsigned long long key = ((unsigned long long)hi << 32) | lo;
            best[nt] = key > best[nt] ? key : best[nt];
        }
    };

    const int k_begin = chunk * CH;
    const int k_end = (k_begin + CH < MTS) ? k_begin + CH : MTS;
#if SPLIT
    const int kodd = hdr[HDR_KODD];
    scan_range(k_begin, min(k_end, kodd), 0);
    scan_range(max(k_begin, kodd), k_end, 1);
#else
    (void)hdr;
    scan_range(k_begin, k_end, 0);
#endif

    // merge the four lane groups of each target and store the chunk's key
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        unsigned long long key = best[nt];
#pragma unroll
        for (int s = 16; s <= 32; s <<= 1) {
            const unsigned ohi = (unsigned)__shfl_xor((int)(unsigned)(key >> 32), s);
            const unsigned olo = (unsigned)__shfl_xor((int)(unsigned)key, s);
            const unsigned long long o = ((unsigned long long)ohi << 32) | olo;
            key = o > key ? o : key;
        }
        const int t = tb * TPG + wave * TPW + nt * 16 + col;
        if (grp == 0 && t < T) part[(long)chunk * T + t] = key;
    }
}
#endif

#ifdef FB_NN_FINAL
#define FW FB_FW
#define TG FB_TG
#define NCHK FB_NCHK
#define CAND (16 * TG)               // rows of one tracking group

__device__ __forceinline__ int sq_dist(const unsigned char* a, const unsigned char* b)
{
    int s = 0;
#pragma unroll 2
    for (int k = 0; k < D; k += 16) {
        const i32x4 va = *(const i32x4*)(a + k), vb = *(const i32x4*)(b + k);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const unsigned x = (unsigned)va[w], y = (unsigned)vb[w];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = (int)((x >> (8 * j)) & 255u) - (int)((y >> (8 * j)) & 255u);
                s += e * e;
            }
        }
    }
    return s;
}

// 16 targets per workgroup.  Thread (target tl = tid % 16, chunk lane
// cl = tid / 16) takes chunks cl, cl + CL, ... (16 consecutive targets of
// one chunk are one 128-byte row of part), the CL chunk lanes are merged
// in LDS, then the workgroup's threads re-measure the 16 x CAND candidates.
#define FT 16
#define CL (FW * 64 / FT)
extern "C" __global__ void __launch_bounds__(FW * 64)
fbnn_final(const unsigned char* __restrict__ tg, const unsigned char* __restrict__ nb,
           const int* __restrict__ perm, const unsigned long long* __restrict__ part,
           int* __restrict__ idx, int* __restrict__ dist)
{
    __shared__ unsigned long long red[CL][FT];
    __shared__ unsigned long long win[FT];
    __shared__ int g0s[FT];
    const int tid = threadIdx.x;
    const int tl = tid % FT, cl = tid / FT;
    const int t = blockIdx.x * FT + tl;
    unsigned long long key = 0;
    if (t < T) {
#pragma unroll 4
        for (int c = cl; c < NCHK; c += CL) {
            const unsigned long long v = part[(long)c * T + t];
            key = v > key ? v : key;
        }
    }
    red[cl][tl] = key;
    if (tid < FT) win[tid] = ~0ull;
    __syncthreads();
    for (int h = CL / 2; h > 0; h >>= 1) {          // CL is a power of two
        if (cl < h) {
            const unsigned long long o = red[cl + h][tl];
            if (o > red[cl][tl]) red[cl][tl] = o;
        }
        __syncthreads();
    }
    if (tid < FT) g0s[tid] = (int)((0xFFFFFFFFu - (unsigned)(red[0][tid] & 0xFFFFFFFFull)) >> 4);
    __syncthreads();
    for (int e = tid; e < FT * CAND; e += FW * 64) {
        const int el = e / CAND, j = e % CAND;
        const int tt = blockIdx.x * FT + el;
        const long pos = (long)g0s[el] * 16 + j;
        if (tt < T && pos < (long)MTS * 16) {
#if SPLIT
            const int orig = perm[pos];
#else
            const int orig = pos < M ? (int)pos : -1;
            (void)perm;
#endif
            if (orig >= 0) {
                const int d = sq_dist(tg + (long)tt * D, nb + (long)orig * D);
                atomicMin(&win[el], ((unsigned long long)(unsigned)d << 32) | (unsigned)orig);
            }
        }
    }
    __syncthreads();
    if (tid < FT && blockIdx.x * FT + tid < T) {
        idx[blockIdx.x * FT + tid] = (int)(unsigned)(win[tid] & 0xFFFFFFFFull);
        dist[blockIdx.x * FT + tid] = (int)(unsigned)(win[tid] >> 32);
    }
}
#endif
