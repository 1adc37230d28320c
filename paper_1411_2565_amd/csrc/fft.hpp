// fft.hpp -- hand-written power-of-two complex FFT for gfx950, FP32.
//
// The demagnetising field is a zero-padded linear convolution evaluated with
// the discrete convolution theorem (Zhu, arXiv:1411.2565, Sec. 3).  This file
// holds the 1D transform every pass uses: a Stockham autosort FFT (no bit
// reversal pass), radix 8 with a final radix-4/4 or radix-2 stage, on lines
// held in LDS by a whole workgroup.  Forward uses exp(-2 pi i jk/L); the
// inverse uses exp(+2 pi i jk/L) and is unnormalised.
//
// Twiddles come from one table of exp(-2 pi i t / MAXL), t < MAXL, rounded
// once from FP64 (init kernel), so every twiddle is within 0.5 ulp.
#pragma once
#include <hip/hip_runtime.h>

namespace mmk {

constexpr int MAXL = 1024;  // longest line along any padded axis

extern __device__ float2 g_tw[MAXL];

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward quarter turn) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a)
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// exp(-+2 pi i t / L), t in [0, L), L a power of two <= MAXL
template <bool INV>
__device__ __forceinline__ float2 twiddle(int t, int L)
{
    const float2 w = g_tw[t * (MAXL / L)];
    return INV ? make_float2(w.x, -w.y) : w;
}

// ---- small DFTs in registers ---------------------------------------------

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
    static __device__ __forceinline__ void run(float2 *) {}
};

template <bool INV>
struct Dft<2, INV> {
    static __device__ __forceinline__ void run(float2 *v)
    {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <bool INV>
struct Dft<4, INV> {
    static __device__ __forceinline__ void run(float2 *v)
    {
        const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const float2 t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <bool INV>
struct Dft<8, INV> {
    static __device__ __forceinline__ void run(float2 *v)
    {
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        const float h = 0.70710678118654752440f;
        // o[k] *= w8^k, w8 = exp(-+ i pi/4)
        o[1] = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                   : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        o[2] = mul_mi<INV>(o[2]);
        o[3] = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                   : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
};

// ---- one Stockham stage ----------------------------------------------------
// Sub-transforms of length Ns are complete on entry; the stage merges R of
// them into sub-transforms of length Ns*R.  j indexes the L/R butterflies.
template <int R, bool INV>
__device__ __forceinline__ void stockham_stage(const float2 *__restrict__ src,
                                               float2 *__restrict__ dst, int L, int Ns, int j)
{
    const int stride = L / R;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * stride];
    const int k = j & (Ns - 1);
    if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle<INV>(r * k, Ns * R));
    }
    Dft<R, INV>::run(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
}

// radix for the next stage when `rem` = L/Ns points remain to be merged:
// 8 while possible, ending in 8*4*4 / 8*4 / 4*4 / 4 / 2 shapes
__host__ __device__ constexpr int next_radix(int rem)
{
    return (rem == 16 || rem == 4) ? 4 : (rem == 2 ? 2 : 8);
}

template <int L, int Ns, bool INV>
struct Stages {
    static __device__ __forceinline__ void run(float2 *&src, float2 *&dst, int nlines, int ls)
    {
        if constexpr (Ns < L) {
            constexpr int R = next_radix(L / Ns);
            constexpr int B = L / R;  // butterflies per line
            __syncthreads();
            for (int idx = threadIdx.x; idx < nlines * B; idx += blockDim.x) {
                const int line = idx / B, j = idx - line * B;
                stockham_stage<R, INV>(src + line * ls, dst + line * ls, L, Ns, j);
            }
            float2 *t = src;
            src = dst;
            dst = t;
            Stages<L, Ns * R, INV>::run(src, dst, nlines, ls);
        }
    }
};

// FFT of `nlines` lines of length L stored in LDS at line stride `ls`,
// ping-ponging between buffers a and b.  All threads of the block must call
// it.  Returns the buffer holding the result (natural order), after a
// barrier.
template <int L, bool INV>
__device__ __forceinline__ float2 *lds_fft(float2 *a, float2 *b, int nlines, int ls)
{
    float2 *src = a, *dst = b;
    Stages<L, 1, INV>::run(src, dst, nlines, ls);
    __syncthreads();
    return src;
}

}  // namespace mmk
