// Small helper kernels of the filter-bank correlation library.
//
//   fbcorr_sum_partials  out[i] = sum_{p<NP} part[p*L + i]; slice k < RS adds
//                        p = k, k+RS, k+2RS, ... in increasing order, then the
//                        RS slice sums are added in increasing k (a fixed
//                        order, so the result is deterministic); four
//                        consecutive i per thread when L % 4 == 0, LANES
//                        threads per slice.
//   fbcorr_flip_filters  wf[d,u,v,n] = w[n, FH-1-u, FW-1-v, d]: the filters of
//                        the input-gradient correlation.
//   fbcorr_pack_lowp     per filter n: e_n = floor(log2 max|w[n]|),
//                        wq[n,k] = round_to_nearest_even(w[n,k] * 2^-e_n) as
//                        bf16 (LOWP=1) or fp16 (LOWP=2), unscale[n] = 2^e_n
//                        (an all-zero filter gets e_n = 0).
//   fbcorr_absmax        part[g] = max |x[i]| over workgroup g's share of the
//                        n input values (256 workgroups): the fp16 forward's
//                        per-tensor input scale is derived from these.
//   fbcorr_fill_int      integer-valued pattern in [-R, R] (tuner gate data).
//   fbcorr_transpose_filters  wt[((u*FW + v)*D + d)*NPAD + n] = w[n,u,v,d]
//                        (zero for N <= n < NPAD): the filters of one tap
//                        contiguous, for the direct kernel's scalar loads.
//
// Compile-time constants: L NP RS LANES (sum); N FH FW D (flip, pack,
// transpose); LOWP (pack); NPAD (transpose).
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

// Specialisation constants arrive as FB_<name> (see the host generator).
#ifdef FB_L
#define L FB_L
#endif
#ifdef FB_NP
#define NP FB_NP
#endif
#ifdef FB_RS
#define RS FB_RS
#endif
#ifdef FB_N
#define N FB_N
#endif
#ifdef FB_FH
#define FH FB_FH
#endif
#ifdef FB_FW
#define FW FB_FW
#endif
#ifdef FB_D
#define D FB_D
#endif
#ifdef FB_LOWP
#define LOWP FB_LOWP
#endif

#ifdef FB_SUM_PARTIALS
// Four consecutive outputs per thread when L allows 16-byte loads; a
// workgroup covers LANES x SV outputs with RS slices.
#define SV ((L % 4 == 0) ? 4 : 1)
#define LV (L / SV)
#ifdef FB_LANES
#define LANES FB_LANES
#else
#define LANES 64
#endif
typedef float f32x4s __attribute__((ext_vector_type(4)));
extern "C" __global__ void __launch_bounds__(LANES * RS)
fbcorr_sum_partials(const float* __restrict__ part, float* __restrict__ out)
{
    __shared__ float red[RS][LANES * SV];
    const int e = threadIdx.x % LANES, sl = threadIdx.x / LANES;
    const long i = (long)blockIdx.x * LANES + e;     // in units of SV floats
#if SV == 4
    f32x4s acc = {0.f, 0.f, 0.f, 0.f};
    if (i < LV) {
        for (int p = sl; p < NP; p += RS) acc += *(const f32x4s*)(part + (long)p * L + i * 4);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[sl][e * 4 + k] = acc[k];
    __syncthreads();
    if (sl == 0 && i < LV) {
        f32x4s t = {red[0][e * 4], red[0][e * 4 + 1], red[0][e * 4 + 2], red[0][e * 4 + 3]};
#pragma unroll
        for (int k = 1; k < RS; ++k) {
            t[0] += red[k][e * 4]; t[1] += red[k][e * 4 + 1];
            t[2] += red[k][e * 4 + 2]; t[3] += red[k][e * 4 + 3];
        }
        *(f32x4s*)(out + i * 4) = t;
    }
#else
    float acc = 0.f;
    if (i < LV) {
        for (int p = sl; p < NP; p += RS) acc += part[(long)p * L + i];
    }
    red[sl][e] = acc;
    __syncthreads();
    if (sl == 0 && i < LV) {
        float t = red[0][e];
#pragma unroll
        for (int k = 1; k < RS; ++k) t += red[k][e];
        out[i] = t;
    }
#endif
}
#endif

#ifdef FB_FLIP_FILTERS
extern "C" __global__ void __launch_bounds__(256)
fbcorr_flip_filters(const float* __restrict__ w, float* __restrict__ wf)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)N * FH * FW * D) return;
    // e indexes wf[d][u][v][n]
    const int n = e % N;
    const int v = (e / N) % FW;
    const int u = (e / ((long)N * FW)) % FH;
    const int d = e / ((long)N * FW * FH);
    wf[e] = w[(((long)n * FH + (FH - 1 - u)) * FW + (FW - 1 - v)) * D + d];
}
#endif

#ifdef FB_PACK_LOWP
extern "C" __global__ void __launch_bounds__(256)
fbcorr_pack_lowp(const float* __restrict__ w, unsigned short* __restrict__ wq,
                 float* __restrict__ unscale)
{
    // One filter per workgroup.  Small filters are read once into registers
    // (all loads in flight together), larger ones twice; the maximum is
    // reduced within each wave by shuffles, then across the four waves.
    constexpr int K = FH * FW * D;
    constexpr int PER = (K + 255) / 256;
    constexpr bool HELD = PER <= 32;
    __shared__ float red[4];
    const int n = blockIdx.x;
    const float* wn = w + (long)n * K;
    float vals[HELD ? PER : 1];
    float m = 0.f;
    if (HELD) {
#pragma unroll
        for (int i = 0; i < (HELD ? PER : 1); ++i) {
            const int k = threadIdx.x + i * 256;
            vals[i] = k < K ? wn[k] : 0.f;
            m = fmaxf(m, fabsf(vals[i]));
        }
    } else {
        for (int k = threadIdx.x; k < K; k += 256) m = fmaxf(m, fabsf(wn[k]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int ex = 0;
    if (m > 0.f) {
        (void)frexpf(m, &ex);   // m = f * 2^ex, f in [0.5, 1)
        ex -= 1;                // floor(log2 m)
    }
    const float sc = ldexpf(1.0f, -ex);
    auto put = [&](int k, float x) {
        const float v = x * sc;       // exact: power-of-two scale
#if LOWP == 1
        const __bf16 hv = (__bf16)v;
#else
        const _Float16 hv = (_Float16)v;
#endif
        wq[(long)n * K + k] = __builtin_bit_cast(unsigned short, hv);
    };
    if (HELD) {
#pragma unroll
        for (int i = 0; i < (HELD ? PER : 1); ++i) {
            const int k = threadIdx.x + i * 256;
            if (k < K) put(k, vals[i]);
        }
    } else {
        for (int k = threadIdx.x; k < K; k += 256) put(k, wn[k]);
    }
    if (threadIdx.x == 0) unscale[n] = ldexpf(1.0f, ex);
}
#endif

#ifdef FB_ABSMAX
typedef float f32x4a __attribute__((ext_vector_type(4)));
extern "C" __global__ void __launch_bounds__(256)
fbcorr_absmax(const float* __restrict__ x, long n, float* __restrict__ part)
{
    // 16-byte loads where the data allows, four in flight per thread, then
    // the scalar tail
    __shared__ float red[4];
    float m = 0.f;
    const long n4 = (((unsigned long)x & 15) == 0) ? n / 4 : 0;
    const long stride = (long)gridDim.x * 256;
    long i = (long)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        f32x4a v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = ((const f32x4a*)x)[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v[k][0]), fabsf(v[k][1])), fmaxf(fabsf(v[k][2]), fabsf(v[k][3]))));
    }
    for (; i < n4; i += stride) {
        const f32x4a v = ((const f32x4a*)x)[i];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
    }
    for (long i = n4 * 4 + (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        m = fmaxf(m, fabsf(x[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}
#endif

#ifdef FB_FILL_INT
// Integer-valued test pattern in [-R, R] for the tuner's exactness gate:
// out[i] = (h(i, seed) mod (2R+1)) - R with a 32-bit integer mixing hash.
extern "C" __global__ void __launch_bounds__(256)
fbcorr_fill_int(float* __restrict__ out, long n, unsigned seed, int R)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    unsigned hsh = (unsigned)i * 0x9E3779B1u ^ (unsigned)(i >> 32) ^ seed;
    hsh ^= hsh >> 15; hsh *= 0x85EBCA77u; hsh ^= hsh >> 13; hsh *= 0xC2B2AE3Du; hsh ^= hsh >> 16;
    out[i] = (float)((int)(hsh % (unsigned)(2 * R + 1)) - R);
}
#endif

#ifdef FB_TRANSPOSE_FILTERS
extern "C" __global__ void __launch_bounds__(256)
fbcorr_transpose_filters(const float* __restrict__ w, float* __restrict__ wt)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;    // over FH*FW*D*NPAD
    if (e >= (long)FH * FW * D * FB_NPAD) return;
    const int n = (int)(e % FB_NPAD);
    const long k = e / FB_NPAD;                              // (u*FW + v)*D + d
    wt[e] = n < N ? w[(long)n * FH * FW * D + k] : 0.f;
}
#endif
