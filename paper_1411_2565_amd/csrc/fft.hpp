// fft.hpp -- hand-written power-of-two complex FFT for gfx950, FP32.
//
// The demagnetising field is a zero-padded linear convolution evaluated with
// the discrete convolution theorem (Zhu, arXiv:1411.2565, Sec. 3).  This file
// holds the 1D transform every pass uses: a Stockham autosort FFT whose data
// stays in registers.  A line of length L is spread over L/E threads, E
// values each, thread t holding positions t + q*(L/E), q < E.  Every radix
// stage (radix 8, then 4 or 2 to finish) runs in registers; between stages
// the line is exchanged once through LDS.  The caller loads global memory
// straight into the first stage's inputs and stores the last stage's outputs
// straight to global memory; both are in natural order and coalesced.
//
// Forward uses exp(-2 pi i jk/L); the inverse exp(+2 pi i jk/L), unnormalised.
// Twiddles come from one table of exp(-2 pi i t / MAXL), t < MAXL, rounded
// once from FP64 (within 0.5 ulp); a radix-R butterfly loads w and w^2 and
// forms the other powers with at most three complex products (a few ulp).
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

// LDS index with one pad slot every 8 complex values (spreads the strided
// Stockham writes over the banks)
__device__ __forceinline__ int lpad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_line(int L) { return L + L / 8 + 1; }

__host__ __device__ constexpr int elems_per_thread(int L) { return L < 8 ? L : 8; }

// radix of the stage that merges sub-transforms of length Ns when rem = L/Ns
// points remain: as large as the per-thread element count allows
__host__ __device__ constexpr int stage_radix(int rem, int E) { return rem < E ? rem : E; }

// Twiddles one thread needs over all stages of a length-L FFT with E points
// per thread: w and w^2 (w alone for radix 2) of each of its butterflies in
// every stage after the first.  Loaded together, while the data loads are in
// flight, they keep table-load latency off the chain of exchanges between
// stages; one set serves the forward and the inverse transform (conjugated).
__host__ __device__ constexpr int tw_offset(int L, int E, int Ns_end)
{
    int n = 0;
    for (int Ns = 1; Ns < L && Ns < Ns_end;) {
        const int R = stage_radix(L / Ns, E);
        if (Ns > 1) n += (E / R) * (R > 2 ? 2 : 1);
        Ns *= R;
    }
    return n;
}

template <int L, int E>
struct TwSet {
    static constexpr int N = tw_offset(L, E, L);
    float2 w[N > 0 ? N : 1];
};

template <int L, int E, int Ns = 1>
__device__ __forceinline__ void load_twiddles(TwSet<L, E> &s, int t)
{
    if constexpr (Ns < L) {
        constexpr int R = stage_radix(L / Ns, E), NB = E / R, T = L / E, G = R > 2 ? 2 : 1;
        constexpr int off = tw_offset(L, E, Ns);
        if constexpr (Ns > 1) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int k = (t + i * T) & (Ns - 1);
                s.w[off + i * G] = twiddle<false>(k, Ns * R);
                if constexpr (R > 2) s.w[off + i * G + 1] = twiddle<false>(2 * k, Ns * R);
            }
        }
        load_twiddles<L, E, Ns * R>(s, t);
    }
}

// Orders one stage's LDS writes before the next stage's reads, and those
// reads before the writes after them.  WAVE: every line lies within one
// wavefront, whose LDS operations execute in issue order, so only the
// compiler has to be kept from moving them (a fence at wavefront scope);
// otherwise a block barrier.
template <bool WAVE>
__device__ __forceinline__ void exchange_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Stages of an FFT of length L over NC lines held by one thread group:
// v[c][q] = line c, position t + q*(L/E).  lds[c] is line c's exchange buffer
// (lds_line(L) complex); tw holds this thread's twiddles (load_twiddles).
// Every thread of the block (WAVE: of the line's wavefront) must take part,
// as the exchanges are ordered by block barriers (WAVE: wavefront fences).
template <int L, int E, int NC, int Ns, bool INV, bool WAVE>
__device__ __forceinline__ void fft_stages(float2 (&v)[NC][E], float2 *const (&lds)[NC], int t,
                                           const TwSet<L, E> &tw)
{
    if constexpr (Ns < L) {
        constexpr int R = stage_radix(L / Ns, E);
        constexpr int NB = E / R;      // butterflies per thread in this stage
        constexpr int T = L / E;       // threads per line
        constexpr bool last = (Ns * R == L);
        constexpr int off = tw_offset(L, E, Ns), G = R > 2 ? 2 : 1;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * T;
            const int k = j & (Ns - 1);
            // w^r from w, w^2 and at most three complex products
            float2 w[R];
            if constexpr (Ns > 1) {
                w[1] = INV ? cconj(tw.w[off + i * G]) : tw.w[off + i * G];
                if constexpr (R > 2) {
                    w[2] = INV ? cconj(tw.w[off + i * G + 1]) : tw.w[off + i * G + 1];
#pragma unroll
                    for (int r = 3; r < R; ++r) w[r] = cmul(w[r - 2], w[2]);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                float2 u[R];
#pragma unroll
                for (int r = 0; r < R; ++r) u[r] = v[c][i + r * NB];
                if constexpr (Ns > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) u[r] = cmul(u[r], w[r]);
                }
                Dft<R, INV>::run(u);
                if constexpr (last) {
#pragma unroll
                    for (int r = 0; r < R; ++r) v[c][i + r * NB] = u[r];
                } else {
                    const int base = (j - k) * R + k;
#pragma unroll
                    for (int r = 0; r < R; ++r) lds[c][lpad(base + r * Ns)] = u[r];
                }
            }
        }
        if constexpr (!last) {
            exchange_sync<WAVE>();
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int q = 0; q < E; ++q) v[c][q] = lds[c][lpad(t + q * T)];
            exchange_sync<WAVE>();
            fft_stages<L, E, NC, Ns * R, INV, WAVE>(v, lds, t, tw);
        }
    }
}

// In-register FFT of NC lines per thread group (see fft_stages) with
// twiddles from a set filled by load_twiddles<L, E>.  On entry and exit
// v[c][q] holds position t + q*(L/E) of line c, natural order.  WAVE: the
// caller lays each line's L/E threads out as consecutive lanes of one
// wavefront (thread = line * (L/E) + t, L/E <= 64), so the stages need no
// block barrier.
template <int L, bool INV, bool WAVE = false, int NC, int E>
__device__ __forceinline__ void reg_fft(float2 (&v)[NC][E], float2 *const (&lds)[NC], int t, const TwSet<L, E> &tw)
{
    static_assert(!WAVE || (L / E <= 64 && (64 % (L / E)) == 0), "a line must lie within one wavefront");
    static_assert(E >= 1 && E <= L && (L % E) == 0, "element count");
    // Wait for the whole set here, before the first stage.  Left to itself
    // the compiler waits for the last stage's twiddles only when it needs
    // them, which can fall after the caller's first output stores; one
    // counter tracks vector-memory loads and stores alike, so that wait would
    // also hold until those stores complete.
#pragma unroll
    for (int i = 0; i < TwSet<L, E>::N; ++i) asm volatile("" ::"v"(tw.w[i].x), "v"(tw.w[i].y));
    fft_stages<L, E, NC, 1, INV, WAVE>(v, lds, t, tw);
}

// The same, loading the twiddle set on entry (issued before the first stage
// waits for the data in v); for callers whose stores all follow the last
// stage, so no early wait is needed.
template <int L, bool INV, bool WAVE = false, int NC, int E>
__device__ __forceinline__ void reg_fft(float2 (&v)[NC][E], float2 *const (&lds)[NC], int t)
{
    static_assert(E >= 1 && E <= L && (L % E) == 0, "element count");
    static_assert(!WAVE || (L / E <= 64 && (64 % (L / E)) == 0), "a line must lie within one wavefront");
    TwSet<L, E> tw;
    load_twiddles<L, E>(tw, t);
    fft_stages<L, E, NC, 1, INV, WAVE>(v, lds, t, tw);
}

}  // namespace mmk
