// kernels.hip -- gfx950 kernels of the micromagnetic step.
//
// Paper: Zhu, "Grace" (arXiv:1411.2565).  Sec. 2: energy density eq. (1),
// effective field eq. (2), LLG eq. (3).  Sec. 3: demagnetising field as the
// zero-padded FFT convolution of M with the demag tensor, six-neighbour
// exchange, explicit Euler; all of it kept on the GPU between steps.
//
// Demag pipeline for one sample (SoA m[3][nz][ny][nx], FP32):
//   xfwd : M = Ms m, real FFT of length Px along x (nx non-zeros), half
//          spectrum kx in [0, Px/2] written transposed: S1[c][z][kx][y]
//   yfwd : FFT of length Py along y (ny non-zeros): S2[c][z][kx][ky]
//   zconv: per (kx, ky): FFT along z (nz non-zeros), H^ = K^ M^ with the real
//          symmetric 3x3 tensor spectrum, inverse FFT, keep nz: in place
//   yinv : inverse along y, keep ny: S1
//   xinv : inverse real FFT along x, keep nx: H_demag[3][nz][ny][nx]
// The tensor spectrum already holds the factor -1/(Px Py Pz), so the last
// inverse transform yields H_demag directly.
#include <hip/hip_ext.h>

#include <type_traits>

#include "fft.hpp"
#include "launch.hpp"

namespace mmk {

__device__ float2 g_tw[MAXL];

__global__ void k_init_tw()
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < MAXL) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)MAXL, &s, &c);
        g_tw[t] = make_float2((float)c, (float)s);
    }
}

// Scratch of the loss reduction for callers that cannot allocate
// (mm_reduce_loss_noalloc): FP64 partial sums, one per block of the
// reduction.  A __device__ array, so each GPU the library runs on holds its
// own copy, at its own address, until the process ends.  Host code never
// passes this name to a kernel: it uses the address init_tables looks up.
static __device__ __align__(256) double scratch[kScratchPartials];

// Per device, with that device current: the twiddle table, and the device
// address of `scratch` into *scratch_dev.
hipError_t init_tables(hipStream_t s, double **scratch_dev)
{
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    *scratch_dev = static_cast<double *>(p);
    hipLaunchKernelGGL(k_init_tw, dim3(MAXL / 256), dim3(256), 0, s);
    return hipGetLastError();
}

constexpr int kThreads = 256;

// Elements per thread in the z pass (4: fewer live registers, one more LDS
// exchange; measured faster than 8 on the 512x512x64 padded grid).
#ifndef MMK_ZC_E
#define MMK_ZC_E 4
#endif
// LDS budget (KB) of a z-pass block: sets its columns per block
#ifndef MMK_ZC_LDS_KB
#define MMK_ZC_LDS_KB 32
#endif
// Long z transforms: 8 points per thread from 256 points on, and from 128 on
// a larger LDS budget with at most 16 columns (16 adjacent ky = one
// 128-byte run per z row).  Measured on the 128^3 and 256^3 cubes: 2.6 ms
// -> 1.9 ms per step at 256^3 against 4 points and the 32 KB budget.
#ifndef MMK_ZC_E_LONG
#define MMK_ZC_E_LONG 8
#endif
#ifndef MMK_ZC_LDS_KB_LONG
#define MMK_ZC_LDS_KB_LONG 128
#endif
#ifndef MMK_ZC_CB_LONG
#define MMK_ZC_CB_LONG 16
#endif
// x passes and y-inverse: FFT stages ordered within each wavefront instead of
// by block barriers (every line of these passes lies within one wavefront)
#ifndef MMK_ZC_SEQ_MIN
#define MMK_ZC_SEQ_MIN 256
#endif
#ifndef MMK_ZC_SEQ_CB
#define MMK_ZC_SEQ_CB 8
#endif
#ifndef MMK_ZC_SEQ_WAVES
#define MMK_ZC_SEQ_WAVES 3
#endif
#if MMK_ZC_SEQ_WAVES > 0
#define MMK_ZC_SEQ_ATTR __attribute__((amdgpu_waves_per_eu(MMK_ZC_SEQ_WAVES)))
#else
#define MMK_ZC_SEQ_ATTR
#endif
#ifndef MMK_ZC_SEQ_THREADS
#define MMK_ZC_SEQ_THREADS 256
#endif
#ifndef MMK_WAVE_FFT
#define MMK_WAVE_FFT 1
#endif
// lines per thread group in the y passes
#ifndef MMK_Y_NC
#define MMK_Y_NC 1
#endif
// lines per block of the x passes (16: 128-byte runs in the transposed S1)
#ifndef MMK_X_LPB
#define MMK_X_LPB 16
#endif

__host__ __device__ constexpr int pow2floor(int v)
{
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
// With every axis padded to P >= 2n - 1, the non-zero inputs and the kept
// outputs of a line all lie in its first half, which is the first half of
// each thread's registers (q < E/2): loads and stores skip the other half,
// and the zeros are compile-time constants for the first radix stage.
__host__ __device__ constexpr int half_elems(int E) { return (E + 1) / 2; }

__host__ __device__ constexpr int nstages(int L, int E)
{
    int s = 0;
    for (int n = 1; n < L; n *= stage_radix(L / n, E)) ++s;
    return s;
}

// ---- launch shapes (shared by kernels and launchers) ----------------------
// Each pass has launch-shape variants V = 0 (the compile-time default), 1
// and 2, chosen per geometry by mm_autotune / mm_set_tuning (single-sample
// launches with L >= 64; batched launches and shorter lines use V = 0).
// The x and y variants only regroup lines, so their results are identical
// bit for bit; the z variants change the radix split (rounding only).
constexpr int kVariants = 3;
constexpr int kTuneMinL = 64;

// y passes: one line of L per T = L/E threads, 256 threads per block;
// V = 1 / 2: 2 / 4 lines per thread group (instead of MMK_Y_NC)
template <int L, int V = 0>
struct YShape {
    static constexpr int E = elems_per_thread(L), T = L / E;
    static constexpr int NC = V == 0 ? MMK_Y_NC : (V == 1 ? 2 : 4);  // lines per thread group
    static constexpr int G = kThreads / T;    // thread groups per block
    static constexpr int LPB = G * NC;        // lines per block
    static constexpr int LDS = LPB * lds_line(L);
};
// z pass: CB columns of the three components per block; V = 1: the other
// point count per thread (4 <-> 8), V = 2: half the columns.
// Transforms of MMK_ZC_SEQ_MIN points and more: V = 0 is the SEQ form
// (k_zconv_seq), where the three components of a column are transformed one
// after another through one exchange buffer per column, in blocks of
// MMK_ZC_SEQ_THREADS threads (CB = 8 columns of 256 points, 4 of 512; the
// G = 16/CB tiles of a 128-byte S2 row run as blocks 8 apart, on one XCD);
// V = 2 is then the concurrent form with the default columns (16 of 256
// points, 8 of 512 with two tiles per block).
template <int L, int V = 0>
struct ZShape {
    static constexpr bool LONG = L >= MMK_ZC_SEQ_MIN;
    static constexpr bool SEQ = LONG && V == 0;
    static constexpr int Ed = L >= 256 ? MMK_ZC_E_LONG : MMK_ZC_E;
    static constexpr int E0 = V == 1 ? (Ed == 4 ? 8 : 4) : Ed;
    static constexpr int E = L < E0 ? L : E0, T = L / E;
    static constexpr int KB = L >= 128 ? MMK_ZC_LDS_KB_LONG : MMK_ZC_LDS_KB;
    static constexpr int BUFS = SEQ ? 1 : 3;  // exchange buffers per column
    static constexpr int CBmax = cmax(1, (KB * 1024) / (BUFS * 8 * lds_line(L)));
    static constexpr int CB0 = cmin(cmin(cmax(1, 1024 / T), pow2floor(CBmax)), L >= 128 ? MMK_ZC_CB_LONG : 1024);
    static constexpr int CB = SEQ ? cmin(cmin(CB0, MMK_ZC_SEQ_CB), cmax(1, MMK_ZC_SEQ_THREADS / T))
                                  : ((V == 2 && !LONG) ? cmax(1, CB0 / 2) : CB0);
    // Long concurrent transforms whose LDS budget leaves fewer than 16
    // columns per pass: one block takes NSUB adjacent tiles of CB columns in
    // turn, so the 128-byte rows of S2 that the tiles share are read by one
    // block, back to back, instead of by blocks on different XCDs.  SEQ
    // blocks of fewer than 16 columns take one tile, and the G = 16/CB tiles
    // of a row run as blocks dispatched back to back on one XCD.
    static constexpr int NSUB = (!SEQ && L >= 128 && CB < 16) ? 16 / CB : 1;
    static constexpr int G = (SEQ && CB < 16) ? 16 / CB : 1;
    static constexpr int THREADS = T * CB;
    static constexpr int LDS = nstages(L, E) > 1 ? BUFS * CB * lds_line(L) : 1;
};
// x passes: LPB lines of L = Px/2 complex per block (16 for 128-byte runs
// in the transposed layout); V = 1 / 2: 8 / 32 lines
template <int L, int V = 0>
struct XShape {
    static constexpr int E = elems_per_thread(L), T = L / E;
    static constexpr int LPB0 = V == 0 ? MMK_X_LPB : (V == 1 ? 8 : 32);
    static constexpr int LPB = cmax(1, cmin(64, cmin(LPB0, 1024 / T)));
    static constexpr int THREADS = T * LPB;
    static constexpr int LDS = LPB * lds_line(L) + L + 1;  // + twiddles exp(-2 pi i k/Px), k <= L
};

// exp(-2 pi i k / (2L)) for k in [0, L] into LDS (first barrier of the caller
// makes it visible)
template <int L, int THREADS>
__device__ __forceinline__ void load_half_twiddles(float2 *tw)
{
    for (int k = threadIdx.x; k <= L; k += THREADS) tw[k] = twiddle<false>(k, 2 * L);
}

// ------------------------------------------------------------------------
// a1: x-forward real FFT.  A real line x[0..Px) (nx non-zeros) is packed as
// z[k] = x[2k] + i x[2k+1], k < L = Px/2, transformed with a length-L complex
// FFT, and unpacked with X[k] = E[k] + exp(-2 pi i k/Px) O[k],
// E[k] = (Z[k] + conj Z[L-k])/2, O[k] = (Z[k] - conj Z[L-k])/(2i).
// The half spectrum kx in [0, L] is written transposed, S1[c][z][kx][y].
// ------------------------------------------------------------------------
// Block (row, tile) of an x pass: row = 3 z + c, tile = y tile.  Rows are the
// fast index, so consecutive blocks (one per XCD in turn) are different rows
// and, with a multiple of 8 rows, all tiles of a row land on one XCD (rows
// first measured 2% faster on the x-forward of the 256x256x32 block).
// The descriptor is copied whole (one batch of scalar loads) before any of
// its fields decides anything.
template <typename D, bool TAB>
__device__ __forceinline__ D pass_desc(const PassArg<D, TAB> &A)
{
    D d;
    if constexpr (TAB)
        d = A.desc[blockIdx.y];
    else
        d = A.d;
    // every field in scalar registers here: the loads of the whole
    // descriptor issue together and complete at one wait, instead of one
    // wait per field as the code first needs it
    static_assert(sizeof(D) % 4 == 0, "descriptor of whole words");
    const uint32_t *w = reinterpret_cast<const uint32_t *>(&d);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(D) / 4); ++i) asm volatile("" ::"s"(w[i]));
    return d;
}
template <typename D, bool TAB>
__device__ __forceinline__ void x_block(const PassArg<D, TAB> &, const Geo &g, int &row, int &tile)
{
    if constexpr (TAB) {
        const int rows = 3 * g.nz;
        row = (int)(blockIdx.x % rows);
        tile = (int)(blockIdx.x / rows);
    } else {
        row = blockIdx.x;
        tile = blockIdx.y;
    }
}

template <int L, int V, bool TAB>
__global__ __launch_bounds__((XShape<L, V>::THREADS)) void k_xfwd(PassArg<XfwdDesc, TAB> A)
{
    using S = XShape<L, V>;
    constexpr int E = S::E, T = S::T, LPB = S::LPB, LD = lds_line(L);
    extern __shared__ float2 sm[];
    const XfwdDesc D = pass_desc(A);
    const Geo &g = D.g;
    int brow = 0, btile = 0;
    x_block(A, g, brow, btile);
    const float *__restrict__ m = D.m;
    const float *__restrict__ ms_map = D.ms_map;
    const float ms = D.ms;
    float2 *__restrict__ S1 = D.S1;
    const int c = brow % 3, z = brow / 3, y0 = btile * LPB;
    if (z >= g.nz || y0 >= g.ny) return;
    const int ll = threadIdx.x / T, t = threadIdx.x - ll * T;
    const int y = y0 + ll;
    const bool ok = y < g.ny;
    const long long cell0 = ((long long)z * g.ny + y) * g.nx;
    const float *row = m + (long long)c * g.N + cell0;
    // every load of the tile is issued before any arithmetic on it
    float2 a[E], sc[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        a[q] = make_float2(0.f, 0.f);
        sc[q] = make_float2(ms, ms);
    }
    if ((g.nx & 1) == 0) {
        // loads from clamped addresses need no branch; lanes past the row's
        // end or the last row take their zero afterwards
        const long long cellc = ((long long)z * g.ny + (ok ? y : g.ny - 1)) * g.nx;
        const float *rowc = m + (long long)c * g.N + cellc;
#pragma unroll
        for (int q = 0; q < half_elems(E); ++q) {
            const int x0 = 2 * (t + q * T);
            const float2 val = *reinterpret_cast<const float2 *>(rowc + min(x0, g.nx - 2));
            a[q] = (ok && x0 < g.nx) ? val : make_float2(0.f, 0.f);
        }
        if (ms_map) {
#pragma unroll
            for (int q = 0; q < half_elems(E); ++q) {
                const int x0 = 2 * (t + q * T);
                const float2 val = *reinterpret_cast<const float2 *>(ms_map + cellc + min(x0, g.nx - 2));
                sc[q] = (ok && x0 < g.nx) ? val : sc[q];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < half_elems(E); ++q) {
            const int x0 = 2 * (t + q * T);
            if (ok && x0 < g.nx) {
                a[q].x = row[x0];
                if (ms_map) sc[q].x = ms_map[cell0 + x0];
                if (x0 + 1 < g.nx) {
                    a[q].y = row[x0 + 1];
                    if (ms_map) sc[q].y = ms_map[cell0 + x0 + 1];
                }
            }
        }
    }
    TwSet<L, E> twl;
    load_twiddles<L, E>(twl, t);
    float2 v[1][E];
#pragma unroll
    for (int q = 0; q < E; ++q)  // the upper half stays a compile-time zero
        v[0][q] = q < half_elems(E) ? make_float2(a[q].x * sc[q].x, a[q].y * sc[q].y) : make_float2(0.f, 0.f);
    float2 *const tw = sm + LPB * LD;
    load_half_twiddles<L, S::THREADS>(tw);
    float2 *const lds[1] = {sm + ll * LD};
    reg_fft<L, false, MMK_WAVE_FFT && (T <= 64)>(v, lds, t, twl);
#pragma unroll
    for (int q = 0; q < E; ++q) sm[ll * LD + t + q * T] = v[0][q];
    __syncthreads();
    float2 *out = S1 + ((long long)(c * g.nz + z) * g.Hx) * g.ny + y0;
    const int nl = min(LPB, g.ny - y0);
    // compile-time trip count: every iteration's loads/stores issue together
    constexpr int NIT = ((L + 1) * LPB + S::THREADS - 1) / S::THREADS;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * S::THREADS;
        const int kx = idx / LPB, yl = idx - kx * LPB;
        if (idx >= (L + 1) * LPB || yl >= nl) continue;
        const float2 *Z = sm + yl * LD;
        const float2 zk = Z[kx & (L - 1)];
        const float2 zc = cconj(Z[(L - kx) & (L - 1)]);
        const float2 Ev = cscale(cadd(zk, zc), 0.5f);
        const float2 Od = mul_mi<false>(cscale(csub(zk, zc), 0.5f));
        out[(long long)kx * g.ny + yl] = cadd(Ev, cmul(tw[kx], Od));
    }
}

// S2 holds the y spectra as [c][kx][z][ky]: the z column of one (kx, ky)
// has stride Py (one ky line) and a component spans nz Py-lines per kx, so
// the z pass reads a compact address range per block.  S1 lines are
// ordered (c, z, kx); this is the S2 line of S1 line `line`.
__device__ __forceinline__ long long s2_line(long long line, const Geo &g)
{
    const long long kx = line % g.Hx, r = line / g.Hx;
    const long long z = r % g.nz, c = r / g.nz;
    return (c * g.Hx + kx) * g.nz + z;
}

// ------------------------------------------------------------------------
// a2 / a4: FFT along y of contiguous columns (length Py, ny non-zeros in /
// ny kept out), one column per T threads.
// ------------------------------------------------------------------------
template <int L, int V, bool TAB>
__global__ __launch_bounds__(kThreads) void k_yfwd(PassArg<YDesc, TAB> A)
{
    using S = YShape<L, V>;
    constexpr int E = S::E, T = S::T, NC = S::NC, LPB = S::LPB;
    extern __shared__ float2 sm[];
    const long long lb = blockIdx.x;
    const YDesc D = pass_desc(A);
    const Geo &g = D.g;
    const float2 *__restrict__ S1 = D.in;
    float2 *__restrict__ S2 = D.out;
    const long long nlines = 3LL * g.nz * g.Hx;
    if (lb * LPB >= nlines) return;
    const int gi = threadIdx.x / T, t = threadIdx.x - gi * T;
    float2 v[NC][E];
    float2 *lds[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const long long line = lb * LPB + gi * NC + c;
        const bool ok = line < nlines;
        const float2 *in = S1 + line * g.ny;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int y = t + q * T;
            v[c][q] = (q < half_elems(E) && ok && y < g.ny) ? in[y] : make_float2(0.f, 0.f);
        }
        lds[c] = sm + (gi * NC + c) * lds_line(L);
    }
    // block barriers kept here: measured 0.3-0.6 us faster than wavefront
    // ordering on the 512-point lines of the 512x512x64 padded grid
    reg_fft<L, false>(v, lds, t);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const long long line = lb * LPB + gi * NC + c;
        if (line < nlines) {
            float2 *out = S2 + s2_line(line, g) * L;
#pragma unroll
            for (int q = 0; q < E; ++q) out[t + q * T] = v[c][q];
        }
    }
}

template <int L, int V, bool TAB>
__global__ __launch_bounds__(kThreads) void k_yinv(PassArg<YDesc, TAB> A)
{
    using S = YShape<L, V>;
    constexpr int E = S::E, T = S::T, NC = S::NC, LPB = S::LPB;
    extern __shared__ float2 sm[];
    const long long lb = blockIdx.x;
    const YDesc D = pass_desc(A);
    const Geo &g = D.g;
    const float2 *__restrict__ S2 = D.in;
    float2 *__restrict__ S1 = D.out;
    const long long nlines = 3LL * g.nz * g.Hx;
    if (lb * LPB >= nlines) return;
    const int gi = threadIdx.x / T, t = threadIdx.x - gi * T;
    float2 v[NC][E];
    float2 *lds[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const long long line = lb * LPB + gi * NC + c;
        const bool ok = line < nlines;
        const float2 *in = S2 + s2_line(line, g) * L;
#pragma unroll
        for (int q = 0; q < E; ++q) v[c][q] = ok ? in[t + q * T] : make_float2(0.f, 0.f);
        lds[c] = sm + (gi * NC + c) * lds_line(L);
    }
    reg_fft<L, true, MMK_WAVE_FFT && (T <= 64)>(v, lds, t);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const long long line = lb * LPB + gi * NC + c;
        if (line < nlines) {
            float2 *out = S1 + line * g.ny;
#pragma unroll
            for (int q = 0; q < half_elems(E); ++q) {
                const int y = t + q * T;
                if (y < g.ny) out[y] = v[c][q];
            }
        }
    }
}

// ------------------------------------------------------------------------
// a3: z transform + tensor multiply + inverse z transform, per (kx, ky).
// K holds the octant kx in [0,Hx), ky in [0,Hy), kz in [0,Hz) as
// K[kx][ky][kz][comp], comp = xx, yy, zz, xy, xz, yz: a block's 16 columns
// read one contiguous chunk.  Components odd in y
// (xy, yz) change sign for ky > Py/2, components odd in z (xz, yz) for
// kz > Pz/2.  Compensated form: each of the six real dot products of three
// terms is accumulated error-free (fma products, two-sum) and rounded once.
// ------------------------------------------------------------------------
// Contraction is off in both helpers: an fma formed from a product and a
// later sum would make the two-sum act on unrounded products, and the
// correction term would then count each product's rounding twice.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
#pragma clang fp contract(off)
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ float dot3_comp(float k0, float x0, float k1, float x1, float k2, float x2)
{
#pragma clang fp contract(off)
    // Dot2 (Ogita, Rump, Oishi 2005): p + sum of all rounding errors
    float p = k0 * x0;
    float s = fmaf(k0, x0, -p);
    float h = k1 * x1;
    float r = fmaf(k1, x1, -h);
    float q, e;
    two_sum(p, h, q, e);
    s += r + e;
    p = q;
    h = k2 * x2;
    r = fmaf(k2, x2, -h);
    two_sum(p, h, q, e);
    s += r + e;
    return q + s;
}

// The plain form: two fmas and a product, rounded three times.
__device__ __forceinline__ float dot3_plain(float k0, float x0, float k1, float x1, float k2, float x2)
{
    return fmaf(k0, x0, fmaf(k1, x1, k2 * x2));
}

// Diagnostic of the multiply's two forms on n triples (k0, x0, k1, x1, k2,
// x2) at in[6 i]: out[2 i] the plain form, out[2 i + 1] the compensated one.
__global__ __launch_bounds__(kThreads) void k_diag_dot3(const float *__restrict__ in, float *__restrict__ out,
                                                        long long n)
{
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float *a = in + 6 * i;
    out[2 * i] = dot3_plain(a[0], a[1], a[2], a[3], a[4], a[5]);
    out[2 * i + 1] = dot3_comp(a[0], a[1], a[2], a[3], a[4], a[5]);
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// ky tiles are ordered so that a tile and its mirror tile (whose columns use
// the same octant rows of K) are 8 blocks apart, i.e. on the same XCD.
__device__ __forceinline__ int zc_tile(int slot, int ntiles)
{
    if ((ntiles & 15) != 0) return slot;
    const int grp = slot >> 4, r = slot & 15;
    const int lower = grp * 8 + (r & 7);
    return r < 8 ? lower : ntiles - 1 - lower;
}

// H(k) = K(k) M(k) at one frequency kz of a column: the octant entries
// K[kx][kyf][kzf] (6 floats: xx yy zz xy xz yz; zc_kload) with the signs of
// the mirrored axes (N_xy odd in ky, N_xz in kz, N_yz in both; zc_apply).
// ok = false (a column beyond Py) multiplies by zero.
__device__ __forceinline__ void zc_kload(float2 (&k)[3], const float *kcol, bool ok, int kz, int Pz)
{
    const int kzf = kz > Pz / 2 ? Pz - kz : kz;
    k[0] = k[1] = k[2] = make_float2(0.f, 0.f);
    if (ok) {
        const float2 *kp = reinterpret_cast<const float2 *>(kcol + kzf * 6);
        k[0] = kp[0];
        k[1] = kp[1];
        k[2] = kp[2];
    }
}

template <bool COMP>
__device__ __forceinline__ void zc_apply(float2 &mx, float2 &my, float2 &mz, const float2 (&k)[3], int kz, int Pz,
                                         float sy)
{
    const float sz = kz > Pz / 2 ? -1.f : 1.f;
    const float kxx = k[0].x, kyy = k[0].y, kzz = k[1].x;
    const float kxy = sy * k[1].y, kxz = sz * k[2].x, kyz = sy * sz * k[2].y;
    const float2 ax = mx, ay = my, az = mz;
    if (COMP) {
        mx = make_float2(dot3_comp(kxx, ax.x, kxy, ay.x, kxz, az.x), dot3_comp(kxx, ax.y, kxy, ay.y, kxz, az.y));
        my = make_float2(dot3_comp(kxy, ax.x, kyy, ay.x, kyz, az.x), dot3_comp(kxy, ax.y, kyy, ay.y, kyz, az.y));
        mz = make_float2(dot3_comp(kxz, ax.x, kyz, ay.x, kzz, az.x), dot3_comp(kxz, ax.y, kyz, ay.y, kzz, az.y));
    } else {
        mx = make_float2(dot3_plain(kxx, ax.x, kxy, ay.x, kxz, az.x), dot3_plain(kxx, ax.y, kxy, ay.y, kxz, az.y));
        my = make_float2(dot3_plain(kxy, ax.x, kyy, ay.x, kyz, az.x), dot3_plain(kxy, ax.y, kyy, ay.y, kyz, az.y));
        mz = make_float2(dot3_plain(kxz, ax.x, kyz, ay.x, kzz, az.x), dot3_plain(kxz, ax.y, kyz, ay.y, kzz, az.y));
    }
}

// Both steps at one point, for the long transforms (k_zconv_seq), whose
// register allocation is at its limit: written out in one piece, as the
// composition of the two helpers above allocated 2 VGPRs more and spilled
// them at 512 points.
template <bool COMP>
__device__ __forceinline__ void zc_point(float2 &mx, float2 &my, float2 &mz, const float *kcol, bool ok, int kz,
                                         int Pz, float sy)
{
    const bool fz = kz > Pz / 2;
    const int kzf = fz ? Pz - kz : kz;
    const float sz = fz ? -1.f : 1.f;
    float2 k01 = make_float2(0.f, 0.f), k23 = k01, k45 = k01;
    if (ok) {
        const float2 *kp = reinterpret_cast<const float2 *>(kcol + kzf * 6);
        k01 = kp[0];
        k23 = kp[1];
        k45 = kp[2];
    }
    const float kxx = k01.x, kyy = k01.y, kzz = k23.x;
    const float kxy = sy * k23.y, kxz = sz * k45.x, kyz = sy * sz * k45.y;
    const float2 ax = mx, ay = my, az = mz;
    if (COMP) {
        mx = make_float2(dot3_comp(kxx, ax.x, kxy, ay.x, kxz, az.x), dot3_comp(kxx, ax.y, kxy, ay.y, kxz, az.y));
        my = make_float2(dot3_comp(kxy, ax.x, kyy, ay.x, kyz, az.x), dot3_comp(kxy, ax.y, kyy, ay.y, kyz, az.y));
        mz = make_float2(dot3_comp(kxz, ax.x, kyz, ay.x, kzz, az.x), dot3_comp(kxz, ax.y, kyz, ay.y, kzz, az.y));
    } else {
        mx = make_float2(dot3_plain(kxx, ax.x, kxy, ay.x, kxz, az.x), dot3_plain(kxx, ax.y, kxy, ay.y, kxz, az.y));
        my = make_float2(dot3_plain(kxy, ax.x, kyy, ay.x, kyz, az.x), dot3_plain(kxy, ax.y, kyy, ay.y, kyz, az.y));
        mz = make_float2(dot3_plain(kxz, ax.x, kyz, ay.x, kzz, az.x), dot3_plain(kxz, ax.y, kyz, ay.y, kzz, az.y));
    }
}

template <int L, bool COMP, int V, bool TAB>
__global__ __launch_bounds__((ZShape<L, V>::THREADS)) void k_zconv(PassArg<ZDesc, TAB> A)
{
    using S = ZShape<L, V>;
    static_assert(!S::SEQ, "SEQ shapes run k_zconv_seq");
    constexpr int E = S::E, T = S::T, CB = S::CB;
    constexpr int NSUB = S::NSUB;
    extern __shared__ float2 sm[];
    // block (slot, kx) of the sample's own grid of (column tiles, kx)
    const ZDesc D = pass_desc(A);
    const Geo &g = D.g;
    int slot, kx, nst;
    if constexpr (TAB) {
        nst = (g.Py + CB * NSUB - 1) / (CB * NSUB);
        slot = (int)(blockIdx.x % nst);
        kx = (int)(blockIdx.x / nst);
    } else {
        slot = blockIdx.x;
        kx = blockIdx.y;
        nst = gridDim.x;
    }
    float2 *__restrict__ S2 = D.S2;
    const float *__restrict__ K = D.K;
    const int t = threadIdx.x / CB, col = threadIdx.x - t * CB;
    const int stile = zc_tile(slot, nst);
    if (kx >= g.Hx || stile * NSUB * CB >= g.Py) return;  // block-uniform, before any barrier
    // every exchange of an FFT ends with a block barrier after its LDS
    // reads, so the next tile's first LDS writes cannot overtake them
    for (int sub = 0; sub < NSUB; ++sub) {
        const int tile = stile * NSUB + sub;
        if (tile * CB >= g.Py) break;  // block-uniform
        const int ky = tile * CB + col;
        const bool ok = ky < g.Py;
        const long long zs = g.Py;                                // stride between z
        const long long cs = (long long)g.Hx * g.nz * g.Py;       // between components
        float2 *base = S2 + (long long)kx * g.nz * g.Py + ky;
        float2 v[3][E];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int zz = t + q * T;
                v[c][q] = (q < half_elems(E) && ok && zz < g.nz) ? base[c * cs + zz * zs]
                                                               : make_float2(0.f, 0.f);
            }
        // one twiddle set for both transforms, loaded while the data arrive
        TwSet<L, E> tw;
        load_twiddles<L, E>(tw, t);
        const int hy = g.Py / 2;
        const bool fy = ky > hy;
        const int kyf = fy ? g.Py - ky : ky;
        const float sy = fy ? -1.f : 1.f;
        // this column's octant entries: K[kx][kyf][kz][6], contiguous over kz,
        // loaded with the data, so that they arrive under the forward
        // transform (left to the compiler, they were loaded after it)
        const float *kcol = K + ((long long)kx * g.Hy + kyf) * g.Hz * 6;
        float2 kk[E][3];
#pragma unroll
        for (int q = 0; q < E; ++q) zc_kload(kk[q], kcol, ok, t + q * T, g.Pz);
        float2 *const lds[3] = {sm + (0 * CB + col) * lds_line(L), sm + (1 * CB + col) * lds_line(L),
                                sm + (2 * CB + col) * lds_line(L)};
        reg_fft<L, false>(v, lds, t, tw);
#pragma unroll
        for (int q = 0; q < E; ++q) zc_apply<COMP>(v[0][q], v[1][q], v[2][q], kk[q], t + q * T, g.Pz, sy);
        reg_fft<L, true>(v, lds, t, tw);
        if (ok) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < half_elems(E); ++q) {
                    const int zz = t + q * T;
                    if (zz < g.nz) base[c * cs + zz * zs] = v[c][q];
                }
        }
    }
}

// The z pass for 64-point transforms (the default shape for Pz = 64).  A
// block takes 16 adjacent ky columns; thread (col, r, w), lane 16 r + col of
// wavefront w, holds the points z = t + 16 q, q = 0..3, of column col, with
// t = 4 r + w.  Each component's forward transform is three radix-4 steps
// in decimation in frequency, with z = 16 n2 + 4 n1 + n0 and the frequency
// kz = k0 + 4 k1 + 16 k2, W = exp(-2 pi i / 64):
//   1. over n2 = q in registers -> k0; times W^(t k0);
//   2. the four rows of the wavefront (n1 = r) and the four registers (k0)
//      are transposed with permlane swaps, so that row r holds k0 = r;
//      over n1 in registers -> k1; times W^(4 n0 k1), n0 = w;
//   3. one LDS exchange: thread (r, w) takes k0 = r, k1 = w from the four
//      wavefronts n0; over n0 in registers -> k2.
// The tensor multiply takes register k2 at kz = r + 4 w + 16 k2 (left in
// this order), and the inverse runs the steps backwards with conjugate
// twiddles (unnormalised, as the other z passes).  One LDS exchange per
// transform instead of two, and three block barriers instead of eight.
__device__ __forceinline__ void pl32_swap(float2 &a, float2 &b)
{
    const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
    const auto y = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
    a = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
    b = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
}
__device__ __forceinline__ void pl16_swap(float2 &a, float2 &b)
{
    const auto x = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
    const auto y = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
    a = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
    b = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
}
// register j of row r <- register r of row j (rows of 16 lanes)
__device__ __forceinline__ void rows_transpose4(float2 (&v)[4])
{
    pl32_swap(v[0], v[2]);
    pl32_swap(v[1], v[3]);
    pl16_swap(v[0], v[1]);
    pl16_swap(v[2], v[3]);
}

template <bool COMP, bool TAB>
__global__ __launch_bounds__(256) void k_zconv64(PassArg<ZDesc, TAB> A)
{
    constexpr int L = 64, CB = 16;
    // [c][k0][k1][n0][col]; each k0 block padded by one 128-byte row, so
    // that the four lane rows of a wavefront (k0 = r, 2 KB apart unpadded)
    // fall on different halves of the LDS banks
    constexpr int K0S = 4 * 4 * CB + CB;
    __shared__ float2 ex[3 * 4 * K0S];
    const ZDesc D = pass_desc(A);
    const Geo &g = D.g;
    int slot, kx, nst;
    if constexpr (TAB) {
        nst = (g.Py + CB - 1) / CB;
        slot = (int)(blockIdx.x % nst);
        kx = (int)(blockIdx.x / nst);
    } else {
        slot = blockIdx.x;
        kx = blockIdx.y;
        nst = gridDim.x;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, r = lane >> 4;
    const int t = 4 * r + w;
    const int tile = zc_tile(slot, nst);
    if (kx >= g.Hx || tile * CB >= g.Py) return;  // block-uniform, before any barrier
    const int ky = tile * CB + col;
    const bool ok = ky < g.Py;
    const long long zs = g.Py;                           // stride between z
    const long long cs = (long long)g.Hx * g.nz * g.Py;  // between components
    float2 *__restrict__ base = D.S2 + (long long)kx * g.nz * g.Py + ky;
    // Every load is unconditional, so that each wait covers only what the
    // code needs next (a load under a branch makes the compiler wait for
    // all outstanding loads): points beyond nz read row 0 and are zeroed by
    // a lane mask; a column beyond Py reads column 0, and as columns never
    // mix and that column is not stored, its values do not matter.
    const float2 *lbase = D.S2 + (long long)kx * g.nz * g.Py + (ok ? ky : 0);
    float2 v[3][4];
    int mk[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int zz = t + 16 * q;
        const bool in = zz < g.nz;
        int zi = in ? zz : 0;
        mk[q] = in ? -1 : 0;
        asm volatile("" : "+v"(zi), "+v"(mk[q]));
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c][q] = lbase[c * cs + zi * zs];
    }
    // twiddles W^(t j) and W^(4 w j), j = 1..3, and the octant entries of
    // this thread's four frequencies, loaded with the data
    float2 w1[4], w2[4];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
        w1[j] = twiddle<false>(t * j, L);
        w2[j] = twiddle<false>(4 * w * j, L);
    }
    const bool fy = ky > g.Py / 2;
    const int kyf = fy ? g.Py - ky : ky;
    const float sy = fy ? -1.f : 1.f;
    const float *kcol = D.K + ((long long)kx * g.Hy + (ok ? kyf : 0)) * g.Hz * 6;
    float2 kk[4][3];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) zc_kload(kk[k2], kcol, true, r + 4 * w + 16 * k2, g.Pz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
            v[c][q] = make_float2(__int_as_float(__float_as_int(v[c][q].x) & mk[q]),
                                  __int_as_float(__float_as_int(v[c][q].y) & mk[q]));
        v[c][2] = v[c][3] = make_float2(0.f, 0.f);
    }
    auto slot_at = [&](int c, int k0, int k1, int n0) { return (c * 4 + k0) * K0S + (k1 * 4 + n0) * CB + col; };
    // forward
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Dft<4, false>::run(v[c]);
#pragma unroll
        for (int j = 1; j < 4; ++j) v[c][j] = cmul(v[c][j], w1[j]);
        rows_transpose4(v[c]);
        Dft<4, false>::run(v[c]);
#pragma unroll
        for (int j = 1; j < 4; ++j) v[c][j] = cmul(v[c][j], w2[j]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) ex[slot_at(c, r, k1, w)] = v[c][k1];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int n0 = 0; n0 < 4; ++n0) v[c][n0] = ex[slot_at(c, r, w, n0)];
        Dft<4, false>::run(v[c]);
    }
    __syncthreads();  // every exchange read before the inverse writes
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) zc_apply<COMP>(v[0][k2], v[1][k2], v[2][k2], kk[k2], r + 4 * w + 16 * k2, g.Pz, sy);
    // inverse
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Dft<4, true>::run(v[c]);
#pragma unroll
        for (int j = 1; j < 4; ++j) v[c][j] = cmul(v[c][j], cconj(w2[j]));
#pragma unroll
        for (int n0 = 0; n0 < 4; ++n0) ex[slot_at(c, r, w, n0)] = v[c][n0];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) v[c][k1] = ex[slot_at(c, r, k1, w)];
        Dft<4, true>::run(v[c]);
        rows_transpose4(v[c]);
#pragma unroll
        for (int j = 1; j < 4; ++j) v[c][j] = cmul(v[c][j], cconj(w1[j]));
        Dft<4, true>::run(v[c]);
    }
    if (ok) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int zz = t + 16 * q;
                if (zz < g.nz) base[c * cs + zz * zs] = v[c][q];
            }
    }
}

// SEQ blocks of G > 1 tiles per 128-byte row: the G tiles of row group j
// and the G tiles of its mirror group go to blocks 8 apart from each other
// (one XCD, dispatched back to back), lower tiles first.  A bijection on
// [0, ntiles) when ntiles is a multiple of 16 G; else zc_tile's order.
__device__ __forceinline__ int zc_tile_seq(int slot, int ntiles, int G)
{
    const int span = 2 * G;
    if (G < 2 || ntiles % (8 * span) != 0) return zc_tile(slot, ntiles);
    const int grp = slot / (8 * span), r = slot - grp * 8 * span;
    const int which = r >> 3, j = grp * 8 + (r & 7);
    return which < G ? j * G + which : ntiles - 1 - (j * G + (span - 1 - which));
}

// The z pass for long transforms (ZShape::SEQ): the same arithmetic as
// k_zconv, with the three components of a column transformed in turn through
// the column's one exchange buffer (each transform's last exchange ends with
// a barrier after its reads, so the next one's first writes cannot overtake
// them).  Each component is stored as soon as its inverse transform ends.
// Blocks of MMK_ZC_SEQ_THREADS threads held to MMK_ZC_SEQ_WAVES waves per
// SIMD: the form needs 160-168 VGPRs, and at 256^3 (512-point columns) 3
// waves per SIMD ran the pass in 718 us against 910 us at 2; at 4 the
// compiler spills 62-82 registers.
template <int L, bool COMP, int V, bool TAB>
__global__ __launch_bounds__((ZShape<L, V>::THREADS)) MMK_ZC_SEQ_ATTR void k_zconv_seq(PassArg<ZDesc, TAB> A)
{
    using S = ZShape<L, V>;
    static_assert(S::SEQ && S::NSUB == 1, "sequential-component form");
    constexpr int E = S::E, T = S::T, CB = S::CB, H = half_elems(E);
    extern __shared__ float2 sm[];
    const ZDesc D = pass_desc(A);
    const Geo &g = D.g;
    int slot, kx, nst;
    if constexpr (TAB) {
        nst = (g.Py + CB - 1) / CB;
        slot = (int)(blockIdx.x % nst);
        kx = (int)(blockIdx.x / nst);
    } else {
        slot = blockIdx.x;
        kx = blockIdx.y;
        nst = gridDim.x;
    }
    const int t = threadIdx.x / CB, col = threadIdx.x - t * CB;
    const int tile = S::G > 1 ? zc_tile_seq(slot, nst, S::G) : zc_tile(slot, nst);
    if (kx >= g.Hx || tile * CB >= g.Py) return;  // block-uniform, before any barrier
    const int ky = tile * CB + col;
    const bool ok = ky < g.Py;
    const long long zs = g.Py;                           // stride between z
    const long long cs = (long long)g.Hx * g.nz * g.Py;  // between components
    float2 *__restrict__ base = D.S2 + (long long)kx * g.nz * g.Py + ky;
    float2 v[3][E];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int zz = t + q * T;
            v[c][q] = (q < H && ok && zz < g.nz) ? base[c * cs + zz * zs] : make_float2(0.f, 0.f);
        }
    TwSet<L, E> tw;
    load_twiddles<L, E>(tw, t);
    // Each transform takes its thread index and buffer offset from an empty
    // asm statement: the three transforms address the same LDS slots, and
    // without this the compiler kept their common addresses in registers
    // from the first transform to the last.
    auto fft = [&](auto inv, int c) {
        int tt = t, off = col * lds_line(L);
        asm volatile("" : "+v"(tt), "+v"(off));
        float2 *const l1[1] = {sm + off};
        reg_fft<L, decltype(inv)::value>(*reinterpret_cast<float2(*)[1][E]>(&v[c][0]), l1, tt, tw);
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) fft(std::false_type{}, c);
    const bool fy = ky > g.Py / 2;
    const int kyf = fy ? g.Py - ky : ky;
    const float sy = fy ? -1.f : 1.f;
    const float *kcol = D.K + ((long long)kx * g.Hy + kyf) * g.Hz * 6;
#pragma unroll
    for (int q = 0; q < E; ++q) zc_point<COMP>(v[0][q], v[1][q], v[2][q], kcol, ok, t + q * T, g.Pz, sy);
    // store addresses and z indices computed afresh rather than kept from
    // the loads (held over the six transforms, the z indices of a 512-point
    // column were spilled to scratch memory)
    asm volatile("" : "+v"(base));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        fft(std::true_type{}, c);
        if (ok) {
            int ts = t;
            asm volatile("" : "+v"(ts));
#pragma unroll
            for (int q = 0; q < H; ++q) {
                const int zz = ts + q * T;
                if (zz < g.nz) base[c * cs + zz * zs] = v[c][q];
            }
        }
    }
}

// ------------------------------------------------------------------------
// a5: x-inverse real FFT (keep nx of Px outputs).  From the half spectrum
// X[0..L] (L = Px/2): Z'[k] = (X[k] + conj X[L-k]) + i (X[k] - conj X[L-k])
// exp(+2 pi i k/Px); the unnormalised inverse length-L FFT of Z' is
// x[2n] + i x[2n+1].
// ------------------------------------------------------------------------
template <int L, int V, bool TAB>
__global__ __launch_bounds__((XShape<L, V>::THREADS)) void k_xinv(PassArg<XinvDesc, TAB> A)
{
    using S = XShape<L, V>;
    constexpr int E = S::E, T = S::T, LPB = S::LPB, LD = lds_line(L);
    extern __shared__ float2 sm[];
    const XinvDesc D = pass_desc(A);
    const Geo &g = D.g;
    int row = 0, btile = 0;
    x_block(A, g, row, btile);
    const float2 *__restrict__ S1 = D.S1;
    float *__restrict__ Hd = D.Hd;
    const int c = row % 3, z = row / 3, y0 = btile * LPB;
    if (z >= g.nz || y0 >= g.ny) return;
    const int nl = min(LPB, g.ny - y0);
    const float2 *in = S1 + ((long long)(c * g.nz + z) * g.Hx) * g.ny + y0;
    float2 *const tw = sm + LPB * LD;
    load_half_twiddles<L, S::THREADS>(tw);
    constexpr int NIT = ((L + 1) * LPB + S::THREADS - 1) / S::THREADS;
    float2 tile[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * S::THREADS;
        const int kx = idx / LPB, yl = idx - kx * LPB;
        tile[it] = (idx < (L + 1) * LPB && yl < nl) ? in[(long long)kx * g.ny + yl] : make_float2(0.f, 0.f);
    }
    const int ll = threadIdx.x / T, t = threadIdx.x - ll * T;
    TwSet<L, E> twl;
    load_twiddles<L, E>(twl, t);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * S::THREADS;
        const int kx = idx / LPB, yl = idx - kx * LPB;
        if (idx < (L + 1) * LPB) sm[yl * LD + kx] = tile[it];
    }
    __syncthreads();
    float2 v[1][E];
    {
        const float2 *X = sm + ll * LD;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int k = t + q * T;
            const float2 xk = X[k], xc = cconj(X[L - k]);
            const float2 Ev = cadd(xk, xc);
            const float2 Od = cmul(csub(xk, xc), cconj(tw[k]));
            v[0][q] = cadd(Ev, mul_mi<true>(Od));
        }
    }
    __syncthreads();
    float2 *const lds[1] = {sm + ll * LD};
    reg_fft<L, true, MMK_WAVE_FFT && (T <= 64)>(v, lds, t, twl);
    if (ll < nl) {
        float *out = Hd + (long long)c * g.N + ((long long)z * g.ny + y0 + ll) * g.nx;
        const bool even = (g.nx & 1) == 0;
#pragma unroll
        for (int q = 0; q < half_elems(E); ++q) {
            const int x0 = 2 * (t + q * T);
            if (x0 < g.nx) {
                if (even) {
                    *reinterpret_cast<float2 *>(out + x0) = v[0][q];
                } else {
                    out[x0] = v[0][q].x;
                    if (x0 + 1 < g.nx) out[x0 + 1] = v[0][q].y;
                }
            }
        }
    }
}

// ------------------------------------------------------------------------
// a6-a8: local field terms and the explicit Euler LLG step, per cell.
//   H = H_demag + (2A/(mu0 Ms)) sum_nb (m_nb - m)/d^2 + (2Ku/(mu0 Ms)) (m.u) u + h_ext
//   f = c1 m x H + c2 m x (m x H),  c1 = -gamma0/(1+alpha^2), c2 = alpha c1
//   m' = m + dt f, then m' /= |m'| unless renormalisation is off.
// Free (Neumann) boundaries: a missing neighbour contributes nothing.
// V cells along x per thread (4 with 16-byte accesses when nx % 4 == 0).
// ------------------------------------------------------------------------
// Profile of the time-dependent external field (the field record of Sec. 5
// gives a start, a decay and a stop time; read as off, full strength, linear
// decay to zero, off).  FP64, so the switching times are decided exactly as
// on any other FP64 host.
__device__ __forceinline__ double field_scale(double t, double t_start, double t_decay, double t_stop)
{
    if (t < t_start) return 0.0;
    if (t <= t_decay) return 1.0;
    if (t >= t_stop) return 0.0;
    return (t_stop - t) / (t_stop - t_decay);
}

template <int V>
struct VecT;
template <>
struct VecT<1> {
    using T = float;
};
template <>
struct VecT<4> {
    using T = float4;
};

template <int V>
__device__ __forceinline__ void vload(const float *p, float (&o)[V])
{
    if constexpr (V == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    } else {
        o[0] = *p;
    }
}
template <int V>
__device__ __forceinline__ void vstore(float *p, const float (&o)[V])
{
    if constexpr (V == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
        *p = o[0];
    }
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// When a z-plane spans P = 8q blocks and the launch covers whole planes, XCD
// x takes blocks x*q .. x*q + q - 1 of every plane (q from the launcher):
// a block's z-neighbour rows (P blocks away) are then always, and its
// y-neighbour rows (the adjacent blocks) mostly, read through the same L2.
// q = 0 keeps the launch order.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int local_block(int b, int q)
{
    if (q <= 0) return b;
    const int k = b >> 3;
    return (k / q) * (8 * q) + (b & 7) * q + k % q;
}

// q for local_block: the z-plane of g spans P = 8q blocks of `cells` cells,
// and the nb blocks of the launch cover whole planes; else 0
static int local_perm_q(const Geo &g, long long cells, long long nb)
{
    const long long plane = (long long)g.nx * g.ny;
    if (plane % cells != 0) return 0;
    const long long P = plane / cells;
    if (P % 8 != 0 || nb % P != 0) return 0;
    return (int)(P / 8);
}

// Local field terms of V cells from cell i0 = (x0, y, z): loads m there into
// mc (unless LOADED) and adds exchange, anisotropy and the (scaled) external field to h, which
// holds H_demag (or zeros) on entry.  mag / inv_ms: magnetic cell, 1/Ms.
// MAPPED: the sample carries an Ms map (per-cell Ms, and vacuum where it is
// 0); without one this compiles to the uniform-Ms code alone.
// TILE (uniform Ms only): m of the caller's y-lines y - yl ... y - yl + nl - 1
// of this z-plane is also in LDS at st ([3][lpb][nx] floats), and the x and
// y neighbours inside it are read from there; the z neighbours come in zn,
// loaded by the caller.  The values are those the loads from m would
// return, taken in the same order, so the field is the same bit for bit.
// The z neighbours of V cells (the cells themselves where there is none),
// loaded by the caller ahead of their use (TILE).
template <int V>
struct ZNeighbours {
    float lo[3][V], hi[3][V];
};

template <int V, bool MAPPED, bool LOADED = false, bool TILE = false>
__device__ __forceinline__ void local_field(const LocalDesc &D, const LocalParams &p, uint32_t terms, float hsc,
                                            long long i0, int x0, int y, int z, float (&mc)[3][V],
                                            float (&h)[3][V], bool (&mag)[V], float (&inv_ms)[V],
                                            const float *st = nullptr, int yl = 0, int nl = 0, int lpb = 0,
                                            const ZNeighbours<V> *zn = nullptr)
{
    static_assert(!(TILE && MAPPED), "the LDS tile path takes a uniform Ms");
    const Geo &g = D.g;
    const long long N = g.N;
    const float *__restrict__ m = D.m;
    const float *__restrict__ ms_map = MAPPED ? D.ms_map : nullptr;
    const float *__restrict__ h_map = D.h_map;
    if constexpr (!LOADED) {  // else the caller has loaded m of these cells into mc
#pragma unroll
        for (int c = 0; c < 3; ++c) vload<V>(m + c * N + i0, mc[c]);
    }
    // With an Ms map, cells with Ms = 0 are vacuum (non-regular geometry):
    // no exchange or anisotropy field there, exchange skips vacuum
    // neighbours (a free surface), and their state never moves.
    if constexpr (MAPPED) {
        float s[V];
        vload<V>(ms_map + i0, s);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            mag[j] = s[j] > 0.f;
            inv_ms[j] = mag[j] ? 1.0f / s[j] : 0.f;
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            mag[j] = true;
            inv_ms[j] = 1.0f / p.ms;
        }
    }
    if (terms & 1u) {
        float lap[3][V];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < V; ++j) lap[c][j] = 0.f;
        // x neighbours: inside the vector, plus one scalar on each side.  All
        // neighbour loads are unconditional, so they issue together: where
        // there is no neighbour (the sample's free surface) the cell itself is
        // read, and its term is not added (x) or adds exactly zero (y, z).
        const bool gl = x0 > 0, gr = x0 + V < g.nx;
        const long long il = gl ? i0 - 1 : i0, ir = gr ? i0 + V : i0 + V - 1;
        bool has_l = gl, has_r = gr;
        if constexpr (MAPPED) {
            has_l = has_l && ms_map[il] > 0.f;
            has_r = has_r && ms_map[ir] > 0.f;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float left, right;
            if constexpr (TILE) {
                const float *row = st + (c * lpb + yl) * g.nx;
                left = row[gl ? x0 - 1 : x0];
                right = row[gr ? x0 + V : x0 + V - 1];
            } else {
                left = m[c * N + il];
                right = m[c * N + ir];
            }
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const float a = mc[c][j];
                float s = 0.f;
                if (j > 0) {
                    if (mag[j - 1]) s += mc[c][j - 1] - a;
                } else if (has_l) {
                    s += left - a;
                }
                if (j < V - 1) {
                    if (mag[j + 1]) s += mc[c][j + 1] - a;
                } else if (has_r) {
                    s += right - a;
                }
                lap[c][j] = p.ax * s;
            }
        }
        const long long sy = g.nx, sz = (long long)g.nx * g.ny;
        auto add = [&](long long off, float w) {
            bool nbm[V];
            if constexpr (MAPPED) {
                float sn[V];
                vload<V>(ms_map + i0 + off, sn);
#pragma unroll
                for (int j = 0; j < V; ++j) nbm[j] = sn[j] > 0.f;
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) nbm[j] = true;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float nb[V];
                vload<V>(m + c * N + i0 + off, nb);
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (nbm[j]) lap[c][j] = fmaf(w, nb[j] - mc[c][j], lap[c][j]);
            }
        };
        if constexpr (TILE) {
            // row yl + dy of the tile, or this row where there is no
            // neighbour; rows beyond the tile from m
            auto add_y = [&](bool has, int dy) {
                const int yt = has ? yl + dy : yl;
                if (yt < 0 || yt >= nl) {
                    add(dy * sy, p.ay);
                    return;
                }
                // an LDS-typed pointer, so that the compiler cannot merge
                // this read and the load from m into one flat load
                typedef __attribute__((address_space(3))) const float lds_float;
                const lds_float *sl = (const lds_float *)st;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
#pragma unroll
                    for (int j = 0; j < V; ++j)
                        lap[c][j] = fmaf(p.ay, sl[(c * lpb + yt) * g.nx + x0 + j] - mc[c][j], lap[c][j]);
                }
            };
            add_y(y > 0, -1);
            add_y(y < g.ny - 1, 1);
        } else {
            add(y > 0 ? -sy : 0, p.ay);
            add(y < g.ny - 1 ? sy : 0, p.ay);
        }
        if constexpr (TILE) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < V; ++j) lap[c][j] = fmaf(p.az, zn->lo[c][j] - mc[c][j], lap[c][j]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < V; ++j) lap[c][j] = fmaf(p.az, zn->hi[c][j] - mc[c][j], lap[c][j]);
        } else {
            add(z > 0 ? -sz : 0, p.az);
            add(z < g.nz - 1 ? sz : 0, p.az);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < V; ++j)
                if (mag[j]) h[c][j] = fmaf(lap[c][j], inv_ms[j], h[c][j]);
    }
    if (terms & 4u) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (!mag[j]) continue;
            const float k = p.ku2 * inv_ms[j] * (mc[0][j] * p.u0 + mc[1][j] * p.u1 + mc[2][j] * p.u2);
            h[0][j] = fmaf(k, p.u0, h[0][j]);
            h[1][j] = fmaf(k, p.u1, h[1][j]);
            h[2][j] = fmaf(k, p.u2, h[2][j]);
        }
    }
    if (terms & 8u) {
        if (h_map) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float e[V];
                vload<V>(h_map + c * N + i0, e);
#pragma unroll
                for (int j = 0; j < V; ++j) h[c][j] = fmaf(hsc, e[j], h[c][j]);
            }
        } else {
            const float e0 = hsc * D.h0, e1 = hsc * D.h1, e2 = hsc * D.h2;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                h[0][j] += e0;
                h[1][j] += e1;
                h[2][j] += e2;
            }
        }
    }
}

// Explicit Euler step of V cells with the field h (mode 1 of k_local): o =
// P(m + dt f), P the renormalisation unless renorm = 0; vacuum cells keep
// their state; bad is set on a non-finite result.  euler_store writes o to
// out_m and sets *flag.
template <int V>
__device__ __forceinline__ void euler_next(const LocalParams &p, float dt, int renorm, const float (&mc)[3][V],
                                           const float (&h)[3][V], const bool (&mag)[V], float (&o)[3][V],
                                           bool &bad)
{
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const float mx = mc[0][j], my = mc[1][j], mz = mc[2][j];
        if (!mag[j]) {  // vacuum: the state stays as it is
            o[0][j] = mx;
            o[1][j] = my;
            o[2][j] = mz;
            continue;
        }
        const float hx = h[0][j], hy = h[1][j], hz = h[2][j];
        // m x H and m x (m x H)
        const float ax = my * hz - mz * hy, ay = mz * hx - mx * hz, az = mx * hy - my * hx;
        const float bx = my * az - mz * ay, by = mz * ax - mx * az, bz = mx * ay - my * ax;
        float nx_ = mx + dt * (p.c1 * ax + p.c2 * bx);
        float ny_ = my + dt * (p.c1 * ay + p.c2 * by);
        float nz_ = mz + dt * (p.c1 * az + p.c2 * bz);
        if (renorm) {
            const float s = rsqrtf(nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
            nx_ *= s;
            ny_ *= s;
            nz_ *= s;
        }
        bad |= !(isfinite(nx_) && isfinite(ny_) && isfinite(nz_));
        o[0][j] = nx_;
        o[1][j] = ny_;
        o[2][j] = nz_;
    }
}

template <int V>
__device__ __forceinline__ void euler_store(const LocalParams &p, float dt, int renorm, const float (&mc)[3][V],
                                            const float (&h)[3][V], const bool (&mag)[V], float *__restrict__ out_m,
                                            long long N, long long i0, int *__restrict__ flag)
{
    float o[3][V];
    bool bad = false;
    euler_next<V>(p, dt, renorm, mc, h, mag, o, bad);
    if (bad) *flag = 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) vstore<V>(out_m + c * N + i0, o[c]);
}

// MAPPED: the samples carry an Ms map (per-cell Ms, and vacuum where it is 0);
// without one the kernel compiles to the uniform-Ms code alone.
template <int MODE, int V, bool TAB, bool MAPPED>
__global__ __launch_bounds__(kThreads) void k_local(PassArg<LocalDesc, TAB> A, LocalParams p, uint32_t terms,
                                                    float dt, int renorm, int *__restrict__ flag)
{
    const long long lb = blockIdx.x;
    const LocalDesc D = pass_desc(A);
    const Geo &g = D.g;
    const float *__restrict__ Hd = D.Hd;
    float *__restrict__ out_m = D.m_out;
    float *__restrict__ out_h = D.h_out;
    // time-dependent field: every block reads this step's time from one
    // clock slot; an Euler step writes the next step's time into the other
    float hsc = 1.f;
    if (p.sched) {
        const double t = p.clk[p.tslot];
        hsc = (float)field_scale(t, p.t_start, p.t_decay, p.t_stop);
        if (MODE == 1 && blockIdx.x == 0 && threadIdx.x == 0) p.clk[p.tslot ^ 1] = t + p.dt64;
    }
    const long long i0 = ((long long)local_block((int)lb, D.perm_q) * kThreads + threadIdx.x) * V;
    if (i0 >= g.N) return;
    const long long N = g.N;
    const int x0 = (int)(i0 % g.nx);
    const long long r = i0 / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    float mc[3][V], h[3][V];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if ((terms & 2u) && Hd) {
            vload<V>(Hd + c * N + i0, h[c]);
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) h[c][j] = 0.f;
        }
    }
    float inv_ms[V];
    bool mag[V];
    local_field<V, MAPPED>(D, p, terms, hsc, i0, x0, y, z, mc, h, mag, inv_ms);
    if (MODE == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vstore<V>(out_h + c * N + i0, h[c]);
        return;
    }
    if (MODE == 2) {
        // one explicit Runge-Kutta stage (coefficients in p; the stage
        // states, like the step result, are renormalised unless renorm = 0)
        const bool write_state = p.stage_last != 2;
        float base[3][V], acc[3][V], er[3][V], kv[3][V];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (write_state) {
                vload<V>(D.m_base + c * N + i0, base[c]);
                if (p.stage_first) {
#pragma unroll
                    for (int j = 0; j < V; ++j) acc[c][j] = base[c][j];
                } else {
                    vload<V>(D.acc + c * N + i0, acc[c]);
                }
            }
            if (p.stage_err) {
                if (p.stage_first) {
#pragma unroll
                    for (int j = 0; j < V; ++j) er[c][j] = 0.f;
                } else {
                    vload<V>(D.eacc + c * N + i0, er[c]);
                }
            }
        }
        // this stage's slope k = f(m, H(m)); zero in vacuum, where the state
        // stays as it is
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const float mx = mc[0][j], my = mc[1][j], mz = mc[2][j];
            const float hx = h[0][j], hy = h[1][j], hz = h[2][j];
            const float ax = my * hz - mz * hy, ay = mz * hx - mx * hz, az = mx * hy - my * hx;
            const float bx = my * az - mz * ay, by = mz * ax - mx * az, bz = mx * ay - my * ax;
            kv[0][j] = mag[j] ? p.c1 * ax + p.c2 * bx : 0.f;
            kv[1][j] = mag[j] ? p.c1 * ay + p.c2 * by : 0.f;
            kv[2][j] = mag[j] ? p.c1 * az + p.c2 * bz : 0.f;
        }
        if (p.stage_kstore >= 0) {  // kept for later stages' states
#pragma unroll
            for (int c = 0; c < 3; ++c) vstore<V>(D.kbuf + ((long long)p.stage_kstore * 3 + c) * N + i0, kv[c]);
        }
        const float wb = p.stage_b * dt, wa = p.stage_a * dt, we = p.stage_e * dt;
        float o[3][V], en[V] = {};
        if (p.stage_err) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                er[0][j] = fmaf(we, kv[0][j], er[0][j]);
                er[1][j] = fmaf(we, kv[1][j], er[1][j]);
                er[2][j] = fmaf(we, kv[2][j], er[2][j]);
                en[j] = sqrtf(er[0][j] * er[0][j] + er[1][j] * er[1][j] + er[2][j] * er[2][j]);
            }
        }
        bool bad = false;
        if (write_state) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    acc[c][j] = fmaf(wb, kv[c][j], acc[c][j]);
                    o[c][j] = p.stage_last ? acc[c][j] : fmaf(wa, kv[c][j], base[c][j]);
                }
            if (!p.stage_last) {
                // next state: m_base + dt (a k + sum_jj a_jj k_jj), earlier
                // slopes k_jj read back from the workspace
                for (int jj = 0; jj < p.stage_nprev; ++jj) {
                    const float w = p.stage_ap[jj] * dt;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float kp[V];
                        vload<V>(D.kbuf + ((long long)jj * 3 + c) * N + i0, kp);
#pragma unroll
                        for (int j = 0; j < V; ++j) o[c][j] = fmaf(w, kp[j], o[c][j]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < V; ++j) {
                if (!mag[j]) continue;
                if (renorm) {
                    const float sc = rsqrtf(o[0][j] * o[0][j] + o[1][j] * o[1][j] + o[2][j] * o[2][j]);
                    o[0][j] *= sc;
                    o[1][j] *= sc;
                    o[2][j] *= sc;
                }
                bad |= !(isfinite(o[0][j]) && isfinite(o[1][j]) && isfinite(o[2][j]));
            }
        }
        if (p.stage_err == 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) vstore<V>(D.eacc + c * N + i0, er[c]);
        } else if (p.stage_err == 2) {
            vstore<V>(D.eacc + i0, en);
        }
        if (!write_state) return;
        if (bad) *flag = 1;
        if (!p.stage_last) {
#pragma unroll
            for (int c = 0; c < 3; ++c) vstore<V>(D.acc + c * N + i0, acc[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) vstore<V>(out_m + c * N + i0, o[c]);
        return;
    }
    euler_store<V>(p, dt, renorm, mc, h, mag, out_m, N, i0, flag);
}

// ------------------------------------------------------------------------
// a5-a8 in one pass: the x-inverse real FFT of the three components of LPB
// y-lines of one z-plane (H_demag of those cells, which never goes to HBM),
// then the local terms and the explicit Euler step of the same cells.
//   Transforms: 3 LPB lines of L = Px/2 complex points, T = L/E threads per
//   line as in the x-inverse pass; each line lies within one wavefront.  The
//   S1 tile of every component is read in runs of LPB consecutive y.
//   Update: H_demag goes to LDS as [3][LPB][nx] floats.  V = 4 (nx % 4 ==
//   0): the first LPB nx/4 threads take 4 consecutive cells each and issue
//   the loads of m at their cells together with the S1 tile, so that they
//   complete under the transform (measured: 26.4 us against 28.0 us with
//   the loads after it, 256x256x32 block; tiles of 4 or 2 y-lines, 29.3 and
//   33.2 us).  V = 1: the threads take the tile's cells one at a time.
//   Both use k_local's device functions, so the result equals the two-kernel
//   step bit for bit.
// TAB: many samples, one per blockIdx.y (descriptors in device memory).
// Block order: G = 16/LPB tiles share the 128-byte lines of S1 (runs of LPB
// complex values).  Block b = 8 G K + 8 h + x (x the XCD) takes tile h of
// group P = 8 K + x, so the tiles of a group run back to back on one XCD, and
// each XCD keeps the same y-tiles in every z-plane (the z-neighbour rows of
// its cells stay in its L2).  When a plane has a multiple of 8 groups, the
// XCD's groups of a plane are adjacent (one y-range), so the y-neighbour rows
// at the edges between them are read once: measured on the 256x256x32 block,
// the pass fetched 79.5 MB against 81.5 MB with the groups 8 apart, at the
// same time within noise.
// ------------------------------------------------------------------------
#ifndef MMK_XE_LPB
#define MMK_XE_LPB 8
#endif
// The uniform-Ms forms, for lines of 128 points and more, are held to 6
// waves per SIMD (80 VGPRs), so that two 768-thread blocks share a CU.  The
// chained form then spills 3 VGPRs, but left at its 82 it ran one block per
// CU: 57.0 us against 44.0 us on the 256x256x32 block.
#define MMK_XE_ATTR(L, XF, MAPPED) __attribute__((amdgpu_waves_per_eu((!(MAPPED) && (L) >= 128) ? 6 : 1)))

template <int L, int LPB_>
struct XEShape {
    static constexpr int E = elems_per_thread(L), T = L / E;
    static constexpr int LPB = LPB_;     // y-lines per component
    static constexpr int G = 16 / LPB;   // tiles per 128-byte S1 line
    static constexpr int NL = 3 * LPB;   // lines per block
    static constexpr int THREADS = NL * T;
    static constexpr int LD = lds_line(L);
    static constexpr int LDS = NL * LD + L + 1;  // line buffers + unpack twiddles (complex)
    // H_demag and the next state of the block's cells ([3][LPB][nx] floats
    // each, nx <= L) fit in the line buffers
    static_assert(6 * LPB * L <= 2 * NL * LD, "H_demag and state tiles exceed the line buffers");
    // one thread per 4 cells of the LPB rows of nx <= L cells
    static_assert(LPB * L / 4 <= THREADS, "too few threads for the update");
};

// The front of the fused passes: the x-inverse of the block's tile (the
// three components of LPB y-lines from y0, z-plane z) into LDS as
// [3][LPB][nx] floats at sm.  `pre` runs once the tile's loads are issued
// (the caller's own loads, which then complete under the transform).
// Every thread of the block takes part; it ends with a barrier.
template <int L, int LPB_, typename Pre>
__device__ __forceinline__ void xe_front(const float2 *__restrict__ S1, const Geo &g, int z, int y0, int nl,
                                         float2 *sm, Pre &&pre)
{
    using S = XEShape<L, LPB_>;
    constexpr int E = S::E, T = S::T, LPB = S::LPB, NL = S::NL, LD = S::LD;
    float2 *const tw = sm + NL * LD;
    load_half_twiddles<L, S::THREADS>(tw);
    // the three components' tiles, (L + 1) x NL entries, line r = c LPB + yl
    constexpr int NIT = ((L + 1) * NL + S::THREADS - 1) / S::THREADS;
    float2 tile_v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * S::THREADS;
        const int kx = idx / NL, r = idx - kx * NL;
        const int c = r / LPB, yl = r - c * LPB;
        tile_v[it] = (idx < (L + 1) * NL && yl < nl)
                         ? S1[(((long long)c * g.nz + z) * g.Hx + kx) * g.ny + y0 + yl]
                         : make_float2(0.f, 0.f);
    }
    pre();
    const int ll = threadIdx.x / T, t = threadIdx.x - ll * T;
    TwSet<L, E> twl;
    load_twiddles<L, E>(twl, t);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * S::THREADS;
        const int kx = idx / NL, r = idx - kx * NL;
        if (idx < (L + 1) * NL) sm[r * LD + kx] = tile_v[it];
    }
    __syncthreads();
    float2 v[1][E];
    {
        const float2 *X = sm + ll * LD;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int k = t + q * T;
            const float2 xk = X[k], xc = cconj(X[L - k]);
            const float2 Ev = cadd(xk, xc);
            const float2 Od = cmul(csub(xk, xc), cconj(tw[k]));
            v[0][q] = cadd(Ev, mul_mi<true>(Od));
        }
    }
    __syncthreads();
    float2 *const lds[1] = {sm + ll * LD};
    reg_fft<L, true, MMK_WAVE_FFT && (T <= 64)>(v, lds, t, twl);
    __syncthreads();  // every line is done with its buffer before H_demag overwrites them
    float *const sH = reinterpret_cast<float *>(sm);
    {
        const int c = ll / LPB, yl = ll - c * LPB;
        if (yl < nl) {
            float *row = sH + (c * LPB + yl) * g.nx;
            const bool even = (g.nx & 1) == 0;
#pragma unroll
            for (int q = 0; q < half_elems(E); ++q) {
                const int xx = 2 * (t + q * T);
                if (xx < g.nx) {
                    if (even) {
                        *reinterpret_cast<float2 *>(row + xx) = v[0][q];
                    } else {
                        row[xx] = v[0][q].x;
                        if (xx + 1 < g.nx) row[xx + 1] = v[0][q].y;
                    }
                }
            }
        }
    }
    __syncthreads();
}

// z-plane and y-tile of block b of a fused pass (the block order above)
template <int LPB, int G>
__device__ __forceinline__ void xe_tile(const Geo &g, int b, int &z, int &tile)
{
    const int ntiles = (g.ny + LPB - 1) / LPB, groups = ntiles / G;
    if (ntiles % G == 0 && ((long long)g.nz * groups) % 8 == 0) {
        const int P = 8 * (b / (8 * G)) + (b & 7);
        z = P / groups;
        int gi = P - z * groups;
        if (groups % 8 == 0) {  // the XCD's groups of a plane: one y-range
            const int r = groups / 8;
            gi = (gi & 7) * r + (gi >> 3);
        }
        tile = G * gi + (b / 8) % G;
    } else {
        z = b / ntiles;
        tile = b - z * ntiles;
    }
}

template <int L, int LPB_, int V, bool TAB, bool XF, bool MAPPED>
__global__ __launch_bounds__((XEShape<L, LPB_>::THREADS)) MMK_XE_ATTR(L, XF, MAPPED) void k_xinv_euler(PassArg<XeDesc, TAB> A, LocalParams p,
                                                                           float dt, int renorm,
                                                                           int *__restrict__ flag)
{
    using S = XEShape<L, LPB_>;
    constexpr int E = S::E, T = S::T, LPB = S::LPB, NL = S::NL, LD = S::LD, G = S::G;
    extern __shared__ float2 sm[];
    const XeDesc D = pass_desc(A);
    const Geo &g = D.g;
    const float2 *__restrict__ S1 = D.S1;
    float hsc = 1.f;
    if (p.sched) {  // time-dependent field, as in k_local's Euler step
        const double t = p.clk[p.tslot];
        hsc = (float)field_scale(t, p.t_start, p.t_decay, p.t_stop);
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) p.clk[p.tslot ^ 1] = t + p.dt64;
    }
    const int ntiles = (g.ny + LPB - 1) / LPB;
    if constexpr (TAB) {
        if ((long long)blockIdx.x >= (long long)g.nz * ntiles) return;  // block-uniform, before any barrier
    }
    int z, tile;
    xe_tile<LPB, G>(g, blockIdx.x, z, tile);
    static_assert(!(XF && MAPPED), "the chained x-forward takes a uniform Ms");
    const LocalDesc DL{g, D.m, nullptr, MAPPED ? D.ms_map : nullptr, D.h_map, D.m_out, nullptr, D.h0, D.h1, D.h2};
    const int y0 = tile * LPB;
    const int nl = min(LPB, g.ny - y0);
    // V = 4: this thread's update cells, 4 from (x0, y, z), if it has any
    const int q4 = g.nx / 4;
    const int w = threadIdx.x;
    const int yl_u = V == 4 ? w / q4 : 0, x0 = V == 4 ? (w - yl_u * q4) * 4 : 0, y = y0 + yl_u;
    const bool upd = V == 4 && w < LPB * q4 && y < g.ny;
    const long long i0 = ((long long)z * g.ny + y) * g.nx + x0;
    float mc[3][4];
    xe_front<L, LPB_>(S1, g, z, y0, nl, sm, [&] {
        if (upd) {
#pragma unroll
            for (int c = 0; c < 3; ++c) vload<4>(D.m + c * g.N + i0, mc[c]);
        }
    });
    float *const sH = reinterpret_cast<float *>(sm);
    constexpr int NIT = ((L + 1) * NL + S::THREADS - 1) / S::THREADS;
    float2 *const tw = sm + NL * LD;
    // [3][LPB][nx] floats after H_demag: with XF the next state of the
    // tile's cells, for the next step's x-forward below; otherwise, with a
    // uniform Ms, the tile's present state, for the neighbours of the update
    float *const sM = sH + 3 * LPB * g.nx;
    if constexpr (V == 4) {
        // uniform Ms without the chained x-forward: the tile's m also goes
        // to LDS, where the x and y neighbours inside the tile are read
        // instead of from m (with XF the form took 88 VGPRs against 82)
        constexpr bool TILE = !MAPPED && !XF;
        ZNeighbours<4> zn;
        if constexpr (TILE) {
            if (upd) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    *reinterpret_cast<float4 *>(sM + (c * LPB + yl_u) * g.nx + x0) =
                        make_float4(mc[c][0], mc[c][1], mc[c][2], mc[c][3]);
                // the z neighbours, issued before the barrier so that they
                // arrive while the tile is read
                const long long sz = (long long)g.nx * g.ny;
                const long long lo = z > 0 ? -sz : 0, hi = z < g.nz - 1 ? sz : 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) vload<4>(D.m + c * g.N + i0 + lo, zn.lo[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c) vload<4>(D.m + c * g.N + i0 + hi, zn.hi[c]);
            }
            __syncthreads();
        }
        if (upd) {
            float h[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 hv = *reinterpret_cast<const float4 *>(sH + (c * LPB + yl_u) * g.nx + x0);
                h[c][0] = hv.x;
                h[c][1] = hv.y;
                h[c][2] = hv.z;
                h[c][3] = hv.w;
                if (D.hd_out) vstore<4>(D.hd_out + c * g.N + i0, h[c]);
            }
            bool mag[4];
            float inv_ms[4];
            local_field<4, MAPPED, true, TILE>(DL, p, 15u, hsc, i0, x0, y, z, mc, h, mag, inv_ms, sM, yl_u, nl,
                                               LPB, &zn);
            if constexpr (XF) {
                float o[3][4];
                bool bad = false;
                euler_next<4>(p, dt, renorm, mc, h, mag, o, bad);
                if (bad) *flag = 1;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    vstore<4>(D.m_out + c * g.N + i0, o[c]);
                    vstore<4>(sM + (c * LPB + yl_u) * g.nx + x0, o[c]);
                }
            } else {
                euler_store<4>(p, dt, renorm, mc, h, mag, D.m_out, g.N, i0, flag);
            }
        }
    } else {
        for (int wi = threadIdx.x; wi < nl * g.nx; wi += S::THREADS) {
            const int yl = wi / g.nx, x = wi - yl * g.nx;
            const long long i = ((long long)z * g.ny + y0 + yl) * g.nx + x;
            float m1[3][1], h1[3][1];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                h1[c][0] = sH[(c * LPB + yl) * g.nx + x];
                if (D.hd_out) D.hd_out[c * g.N + i] = h1[c][0];
            }
            bool mag[1];
            float inv_ms[1];
            local_field<1, MAPPED>(DL, p, 15u, hsc, i, x, y0 + yl, z, m1, h1, mag, inv_ms);
            if constexpr (XF) {
                float o[3][1];
                bool bad = false;
                euler_next<1>(p, dt, renorm, m1, h1, mag, o, bad);
                if (bad) *flag = 1;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    D.m_out[c * g.N + i] = o[c][0];
                    sM[(c * LPB + yl) * g.nx + x] = o[c][0];
                }
            } else {
                euler_store<1>(p, dt, renorm, m1, h1, mag, D.m_out, g.N, i, flag);
            }
        }
    }
    if constexpr (XF) {
        // the next step's x-forward of the tile (the arithmetic of k_xfwd):
        // line ll = (c, yl) packs Ms m into z[k] = r[2k] + i r[2k+1], is
        // transformed, unpacked to the half spectrum and stored in place of
        // this step's S1 tile, which only this block reads
        __syncthreads();
        // this phase's thread index comes from an empty asm statement: the
        // compiler then recomputes its addresses and twiddles here instead of
        // keeping those of the tile load and the first transform live
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int l2 = tid / T, t2 = tid - l2 * T;
        TwSet<L, E> tw2;
        load_twiddles<L, E>(tw2, t2);
        float2 u[1][E];
        {
            const int c = l2 / LPB, yl = l2 - c * LPB;
            const float *row = sM + (c * LPB + yl) * g.nx;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int xx = 2 * (t2 + q * T);
                float2 a = make_float2(0.f, 0.f);
                if (q < half_elems(E) && yl < nl && xx < g.nx) {
                    a.x = row[xx];
                    if (xx + 1 < g.nx) a.y = row[xx + 1];
                }
                u[0][q] = q < half_elems(E) ? make_float2(a.x * p.ms, a.y * p.ms) : make_float2(0.f, 0.f);
            }
        }
        __syncthreads();  // every row is read before the transforms reuse the buffers
        float2 *const lds2[1] = {sm + l2 * LD};
        reg_fft<L, false, MMK_WAVE_FFT && (T <= 64)>(u, lds2, t2, tw2);
#pragma unroll
        for (int q = 0; q < E; ++q) sm[l2 * LD + t2 + q * T] = u[0][q];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = tid + it * S::THREADS;
            const int kx = idx / NL, r = idx - kx * NL;
            const int c = r / LPB, yl = r - c * LPB;
            if (idx >= (L + 1) * NL || yl >= nl) continue;
            const float2 *Z = sm + r * LD;
            const float2 zk = Z[kx & (L - 1)];
            const float2 zc = cconj(Z[(L - kx) & (L - 1)]);
            const float2 Ev = cscale(cadd(zk, zc), 0.5f);
            const float2 Od = mul_mi<false>(cscale(csub(zk, zc), 0.5f));
            D.S1w[(((long long)c * g.nz + z) * g.Hx + kx) * g.ny + y0 + yl] = cadd(Ev, cmul(tw[kx], Od));
        }
    }
}

// ------------------------------------------------------------------------
// Adjoint of one Euler step (exact transpose of the discrete step above).
// Forward: H = H_demag(m) + H_ex(m) + H_an(m) + h_ext; f = c1 m x H +
// c2 m x (m x H); v = m + dt f; m' = v/|v|.  Given lam' = dL/dm':
//   w   = (lam' - (m'.lam') m')/|v|            (lam' without renormalisation)
//   g_H = dt [c1 (w x m) + c2 m x (m x w)]     (= (df/dH)^T w dt)
//   lam = w + dt [c1 H x w + c2 ((m x H) x w + H x (w x m))]
//         + (2A/mu0) L(g_H/Ms) - Ms (N * g_H) + (2Ku/(mu0 Ms)) (u.g_H) u
//   dL/dh_ext += g_H
//   dL/dMs    += -(H_ex + H_an).g_H / Ms - m.(N * g_H)
// L is the symmetric Neumann Laplacian, N* the demag convolution, which is
// self-adjoint (N(-r) = N(r), each N symmetric), so N * g_H is the forward
// demag pipeline run on g_H with unit Ms (it returns -N * g_H).
// k_adj_a does everything except the two non-local terms; k_adj_b adds them.
// ------------------------------------------------------------------------
__device__ __forceinline__ void cross3f(float ax, float ay, float az, float bx, float by, float bz, float &cx,
                                        float &cy, float &cz)
{
    cx = ay * bz - az * by;
    cy = az * bx - ax * bz;
    cz = ax * by - ay * bx;
}

__global__ __launch_bounds__(kThreads) void k_adj_a(Geo g, LocalParams p, const float *__restrict__ m,
                                                    const float *__restrict__ Hd,
                                                    const float *__restrict__ ms_map,
                                                    const float *__restrict__ h_map,
                                                    const float *__restrict__ lam1, float dt, int renorm,
                                                    float *__restrict__ gH, float *__restrict__ lam_loc,
                                                    float *__restrict__ g_hext, float *__restrict__ g_ms)
{
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= g.N) return;
    const long long N = g.N;
    const int x = (int)(i % g.nx);
    const long long r = i / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const float mx = m[i], my = m[N + i], mz = m[2 * N + i];
    const float ms = ms_map ? ms_map[i] : p.ms;
    const float inv_ms = 1.0f / ms;
    // exchange and anisotropy fields (kept apart for dL/dMs)
    float ex = 0.f, ey = 0.f, ez = 0.f;
    {
        const long long sy = g.nx, sz = (long long)g.nx * g.ny;
        auto add = [&](long long j, float w) {
            ex = fmaf(w, m[j] - mx, ex);
            ey = fmaf(w, m[N + j] - my, ey);
            ez = fmaf(w, m[2 * N + j] - mz, ez);
        };
        if (x > 0) add(i - 1, p.ax);
        if (x < g.nx - 1) add(i + 1, p.ax);
        if (y > 0) add(i - sy, p.ay);
        if (y < g.ny - 1) add(i + sy, p.ay);
        if (z > 0) add(i - sz, p.az);
        if (z < g.nz - 1) add(i + sz, p.az);
        ex *= inv_ms;
        ey *= inv_ms;
        ez *= inv_ms;
    }
    const float mu = mx * p.u0 + my * p.u1 + mz * p.u2;
    const float ka = p.ku2 * inv_ms;
    const float anx = ka * mu * p.u0, any = ka * mu * p.u1, anz = ka * mu * p.u2;
    float hx = Hd[i] + ex + anx, hy = Hd[N + i] + ey + any, hz = Hd[2 * N + i] + ez + anz;
    if (h_map) {
        hx += h_map[i];
        hy += h_map[N + i];
        hz += h_map[2 * N + i];
    } else {
        hx += p.h0;
        hy += p.h1;
        hz += p.h2;
    }
    // forward step, recomputed
    float ax, ay, az, bx, by, bz;
    cross3f(mx, my, mz, hx, hy, hz, ax, ay, az);  // m x H
    cross3f(mx, my, mz, ax, ay, az, bx, by, bz);  // m x (m x H)
    const float vx = mx + dt * (p.c1 * ax + p.c2 * bx);
    const float vy = my + dt * (p.c1 * ay + p.c2 * by);
    const float vz = mz + dt * (p.c1 * az + p.c2 * bz);
    float wx = lam1[i], wy = lam1[N + i], wz = lam1[2 * N + i];
    if (renorm) {
        const float inv = rsqrtf(vx * vx + vy * vy + vz * vz);
        const float px = vx * inv, py = vy * inv, pz = vz * inv;
        const float d = px * wx + py * wy + pz * wz;
        wx = (wx - d * px) * inv;
        wy = (wy - d * py) * inv;
        wz = (wz - d * pz) * inv;
    }
    // g_H = dt [c1 (w x m) + c2 m x (m x w)]
    float wmx, wmy, wmz, mwx, mwy, mwz, mmwx, mmwy, mmwz;
    cross3f(wx, wy, wz, mx, my, mz, wmx, wmy, wmz);
    cross3f(mx, my, mz, wx, wy, wz, mwx, mwy, mwz);
    cross3f(mx, my, mz, mwx, mwy, mwz, mmwx, mmwy, mmwz);
    const float gx = dt * (p.c1 * wmx + p.c2 * mmwx);
    const float gy = dt * (p.c1 * wmy + p.c2 * mmwy);
    const float gz = dt * (p.c1 * wmz + p.c2 * mmwz);
    // lam_loc = w + dt [c1 H x w + c2 ((m x H) x w + H x (w x m))] + aniso^T g_H
    float hwx, hwy, hwz, mhwx, mhwy, mhwz, hwmx, hwmy, hwmz;
    cross3f(hx, hy, hz, wx, wy, wz, hwx, hwy, hwz);
    cross3f(ax, ay, az, wx, wy, wz, mhwx, mhwy, mhwz);
    cross3f(hx, hy, hz, wmx, wmy, wmz, hwmx, hwmy, hwmz);
    const float ug = p.u0 * gx + p.u1 * gy + p.u2 * gz;
    lam_loc[i] = wx + dt * (p.c1 * hwx + p.c2 * (mhwx + hwmx)) + ka * ug * p.u0;
    lam_loc[N + i] = wy + dt * (p.c1 * hwy + p.c2 * (mhwy + hwmy)) + ka * ug * p.u1;
    lam_loc[2 * N + i] = wz + dt * (p.c1 * hwz + p.c2 * (mhwz + hwmz)) + ka * ug * p.u2;
    gH[i] = gx;
    gH[N + i] = gy;
    gH[2 * N + i] = gz;
    if (g_hext) {
        g_hext[i] += gx;
        g_hext[N + i] += gy;
        g_hext[2 * N + i] += gz;
    }
    if (g_ms) g_ms[i] -= ((ex + anx) * gx + (ey + any) * gy + (ez + anz) * gz) * inv_ms;
}

// lam = lam_loc + (2A/mu0) L(g_H/Ms) + Ms D,  dL/dMs += m.D,  D = -(N * g_H)
// The completion of one cell i = (x, y, z) of the adjoint step: lam = lam_loc
// + (exchange transpose of g_H / Ms) + Ms d and g_ms += m.d, where d = (dx,
// dy, dz) = -(N * g_H) at the cell (the demag pipeline's output for g_H
// with unit Ms).
__device__ __forceinline__ void adjb_cell(const Geo &g, const LocalParams &p, const float *__restrict__ m,
                                          const float *__restrict__ gH, const float *__restrict__ ms_map,
                                          const float *__restrict__ lam_loc, float *__restrict__ lam,
                                          float *__restrict__ g_ms, long long i, float dx, float dy, float dz)
{
    const long long N = g.N;
    const int x = (int)(i % g.nx);
    const long long r = i / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const float ms = ms_map ? ms_map[i] : p.ms;
    const float inv_ms = 1.0f / ms;
    const float qx = gH[i] * inv_ms, qy = gH[N + i] * inv_ms, qz = gH[2 * N + i] * inv_ms;
    float lx = 0.f, ly = 0.f, lz = 0.f;
    const long long sy = g.nx, sz = (long long)g.nx * g.ny;
    auto add = [&](long long j, float w) {
        const float inv_j = ms_map ? 1.0f / ms_map[j] : inv_ms;
        lx = fmaf(w, gH[j] * inv_j - qx, lx);
        ly = fmaf(w, gH[N + j] * inv_j - qy, ly);
        lz = fmaf(w, gH[2 * N + j] * inv_j - qz, lz);
    };
    if (x > 0) add(i - 1, p.ax);
    if (x < g.nx - 1) add(i + 1, p.ax);
    if (y > 0) add(i - sy, p.ay);
    if (y < g.ny - 1) add(i + sy, p.ay);
    if (z > 0) add(i - sz, p.az);
    if (z < g.nz - 1) add(i + sz, p.az);
    lam[i] = lam_loc[i] + lx + ms * dx;
    lam[N + i] = lam_loc[N + i] + ly + ms * dy;
    lam[2 * N + i] = lam_loc[2 * N + i] + lz + ms * dz;
    if (g_ms) g_ms[i] += m[i] * dx + m[N + i] * dy + m[2 * N + i] * dz;
}

__global__ __launch_bounds__(kThreads) void k_adj_b(Geo g, LocalParams p, const float *__restrict__ m,
                                                    const float *__restrict__ gH, const float *__restrict__ D,
                                                    const float *__restrict__ ms_map,
                                                    const float *__restrict__ lam_loc, float *__restrict__ lam,
                                                    float *__restrict__ g_ms)
{
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= g.N) return;
    const long long N = g.N;
    adjb_cell(g, p, m, gH, ms_map, lam_loc, lam, g_ms, i, D[i], D[N + i], D[2 * N + i]);
}

// ------------------------------------------------------------------------
// a9: FP64 energy terms and mean magnetisation.  Per-block partial sums in a
// fixed order, then one block sums the partials: deterministic.
// ------------------------------------------------------------------------
constexpr int kEq = 8;  // e_ex, e_d, e_an, e_z, sum mx, sum my, sum mz, magnetic cells

// NV values reduced over the kThreads threads of a block by an associative
// op: shuffles within each wavefront, then the wavefronts' results in order
// by thread 0 (a fixed order, so sums are deterministic).  The result is
// valid in thread 0; lds holds kThreads / 64 * NV values.
template <int NV, typename T, typename Op>
__device__ __forceinline__ void block_reduce(T (&v)[NV], T *lds, Op op)
{
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] = op(v[q], __shfl_down(v[q], off, 64));
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[(threadIdx.x >> 6) * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            T r = lds[q];
            for (int w = 1; w < kThreads / 64; ++w) r = op(r, lds[w * NV + q]);
            v[q] = r;
        }
    }
}

struct OpAdd {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a + b; }
};

__global__ __launch_bounds__(kThreads) void k_energy(Geo g, EnergyParams p, const float *__restrict__ m,
                                                     const float *__restrict__ Hd,
                                                     const float *__restrict__ ms_map,
                                                     const float *__restrict__ h_map,
                                                     double *__restrict__ partials)
{
    __shared__ double red[kThreads / 64 * kEq];
    double acc[kEq] = {0, 0, 0, 0, 0, 0, 0, 0};
    const long long N = g.N;
    // the external field at the clock's time, scaled as in the step (FP32
    // scale, so the energy sees the field the step applies)
    const double hsc = p.sched ? (double)(float)field_scale(p.clk[p.tslot], p.t_start, p.t_decay, p.t_stop) : 1.0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < N;
         i += (long long)gridDim.x * kThreads) {
        const double mx = m[i], my = m[N + i], mz = m[2 * N + i];
        const int x = (int)(i % g.nx);
        const long long r = i / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        const double ms = ms_map ? (double)ms_map[i] : p.ms;
        if (!(ms > 0.0)) continue;  // vacuum: no energy, not in the mean
        if (p.terms & 1u) {
            auto pair = [&](long long j, double w) {
                if (ms_map && !(ms_map[j] > 0.f)) return;  // pairs of magnetic cells only
                const double dx = m[j] - mx, dy = m[N + j] - my, dz = m[2 * N + j] - mz;
                acc[0] += w * (dx * dx + dy * dy + dz * dz);
            };
            if (x < g.nx - 1) pair(i + 1, p.cx);
            if (y < g.ny - 1) pair(i + g.nx, p.cy);
            if (z < g.nz - 1) pair(i + (long long)g.nx * g.ny, p.cz);
        }
        if ((p.terms & 2u) && Hd) acc[1] += ms * (mx * Hd[i] + my * Hd[N + i] + mz * Hd[2 * N + i]);
        if (p.terms & 4u) {
            const double mu = mx * p.u0 + my * p.u1 + mz * p.u2;
            acc[2] += 1.0 - mu * mu;
        }
        if (p.terms & 8u) {
            double h0 = p.h0, h1 = p.h1, h2 = p.h2;
            if (h_map) {
                h0 = h_map[i];
                h1 = h_map[N + i];
                h2 = h_map[2 * N + i];
            }
            acc[3] += hsc * ms * (mx * h0 + my * h1 + mz * h2);
        }
        acc[4] += mx;
        acc[5] += my;
        acc[6] += mz;
        acc[7] += 1.0;
    }
    block_reduce<kEq>(acc, red, OpAdd{});
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kEq; ++q) partials[(long long)blockIdx.x * kEq + q] = acc[q];
    }
}

__global__ __launch_bounds__(kThreads) void k_energy_final(int nblk, EnergyParams p, long long N,
                                                           const double *__restrict__ partials,
                                                           double *__restrict__ out)
{
    __shared__ double red[kThreads / 64 * kEq];
    double acc[kEq] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += kThreads)
#pragma unroll
        for (int q = 0; q < kEq; ++q) acc[q] += partials[(long long)b * kEq + q];
    block_reduce<kEq>(acc, red, OpAdd{});
    if (threadIdx.x == 0) {
        const double eex = (p.terms & 1u) ? p.A * p.V * acc[0] : 0.0;
        const double ed = (p.terms & 2u) ? -0.5 * p.mu0 * p.V * acc[1] : 0.0;
        const double ean = (p.terms & 4u) ? p.Ku * p.V * acc[2] : 0.0;
        const double ez = (p.terms & 8u) ? -p.mu0 * p.V * acc[3] : 0.0;
        out[0] = eex;
        out[1] = ed;
        out[2] = ean;
        out[3] = ez;
        out[4] = eex + ed + ean + ez;
        const double cells = acc[7];  // magnetic cells (all N without vacuum)
        out[5] = cells > 0.0 ? acc[4] / cells : 0.0;
        out[6] = cells > 0.0 ? acc[5] / cells : 0.0;
        out[7] = cells > 0.0 ? acc[6] / cells : 0.0;
    }
}

// ------------------------------------------------------------------------
// a0: FP64 demag tensor.  N(o) between two cells o cells apart:
//  near (every |o_a| d_a <= 8 max(dx, dy, dz)): Newell's closed form, the
//    second difference over the 27-point stencil of the auxiliary functions
//    f (diagonal) and g (off-diagonal), divided by 4 pi V;
//  far: (1/V) integral over s in [-d,d]^3 of the dipole kernel
//    K(r) = (I/r^3 - 3 r r^T/r^5)/(4 pi) at r = o d + s, weighted by
//    prod (d_a - |s_a|); each half-axis with 4-point Gauss-Legendre.
// The split is in lengths, not cells: with flat cells (say 5 x 5 x 1 nm) an
// offset of 9 cells along the thin axis is under two cell widths away, where
// 4 nodes are accurate to ~1e-7 only, while Newell's form holds to ~1e-12
// out to 8 of the largest cell dimension.
// ------------------------------------------------------------------------
constexpr double kNearWidths = 8.0;

__device__ double nf(double x, double y, double z)
{
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double xx = x * x, yy = y * y, zz = z * z, R = sqrt(xx + yy + zz);
    if (R == 0.0) return 0.0;
    double acc = (2.0 * xx - yy - zz) * R * (1.0 / 6.0);
    const double p1 = 0.5 * y * (zz - xx), p2 = 0.5 * z * (yy - xx), p3 = x * y * z;
    if (p1 != 0.0) acc += p1 * asinh(y / sqrt(xx + zz));
    if (p2 != 0.0) acc += p2 * asinh(z / sqrt(xx + yy));
    if (p3 != 0.0) acc -= p3 * atan(y * z / (x * R));
    return acc;
}

__device__ double ng(double x, double y, double z)
{
    double sg = 1.0;
    if (x < 0.0) sg = -sg;
    if (y < 0.0) sg = -sg;
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double xx = x * x, yy = y * y, zz = z * z, R = sqrt(xx + yy + zz);
    if (R == 0.0) return 0.0;
    double acc = -x * y * R * (1.0 / 3.0);
    const double q1 = x * y * z, q2 = y * (3.0 * zz - yy) * (1.0 / 6.0), q3 = x * (3.0 * zz - xx) * (1.0 / 6.0);
    const double q4 = z * zz * (1.0 / 6.0), q5 = 0.5 * z * yy, q6 = 0.5 * z * xx;
    if (q1 != 0.0) acc += q1 * asinh(z / sqrt(xx + yy));
    if (q2 != 0.0) acc += q2 * asinh(x / sqrt(yy + zz));
    if (q3 != 0.0) acc += q3 * asinh(y / sqrt(xx + zz));
    if (q4 != 0.0) acc -= q4 * atan(x * y / (z * R));
    if (q5 != 0.0) acc -= q5 * atan(x * z / (y * R));
    if (q6 != 0.0) acc -= q6 * atan(y * z / (x * R));
    return sg * acc;
}

template <bool G>
__device__ double newell27(double X, double Y, double Z, double dx, double dy, double dz)
{
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double wa = a == 1 ? 2.0 : -1.0;
        for (int b = 0; b < 3; ++b) {
            const double wb = b == 1 ? 2.0 : -1.0;
            for (int c = 0; c < 3; ++c) {
                const double wc = c == 1 ? 2.0 : -1.0;
                const double px = X + (a - 1) * dx, py = Y + (b - 1) * dy, pz = Z + (c - 1) * dz;
                s += wa * wb * wc * (G ? ng(px, py, pz) : nf(px, py, pz));
            }
        }
    }
    return s / (4.0 * M_PI * dx * dy * dz);
}

__global__ __launch_bounds__(kThreads) void k_tensor_octant(Geo g, double dx, double dy, double dz,
                                                            double *__restrict__ T)
{
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= g.N) return;
    const int ox = (int)(i % g.nx);
    const long long r = i / g.nx;
    const int oy = (int)(r % g.ny), oz = (int)(r / g.ny);
    const double X = ox * dx, Y = oy * dy, Z = oz * dz;
    double v[6];
    const double reach = kNearWidths * fmax(dx, fmax(dy, dz)) * (1.0 + 1e-12);
    if (X <= reach && Y <= reach && Z <= reach) {
        v[0] = newell27<false>(X, Y, Z, dx, dy, dz);
        v[1] = newell27<false>(Y, X, Z, dy, dx, dz);
        v[2] = newell27<false>(Z, Y, X, dz, dy, dx);
        v[3] = newell27<true>(X, Y, Z, dx, dy, dz);
        v[4] = newell27<true>(X, Z, Y, dx, dz, dy);
        v[5] = newell27<true>(Y, Z, X, dy, dz, dx);
    } else {
        // 4-point Gauss-Legendre on [-1,1]
        const double gx[4] = {-0.86113631159405257522, -0.33998104358485626480,
                              0.33998104358485626480, 0.86113631159405257522};
        const double gw[4] = {0.34785484513745385737, 0.65214515486254614263,
                              0.65214515486254614263, 0.34785484513745385737};
        // nodes of the tent on [-d, d]: s = +-d t, t = (1+x)/2, weight (w/2)(1-t)
        double sx[8], sy[8], sz[8], w[8];
        for (int q = 0; q < 4; ++q) {
            const double t = 0.5 * (1.0 + gx[q]);
            const double wt = 0.5 * gw[q] * (1.0 - t);
            sx[q] = t * dx; sx[q + 4] = -t * dx;
            sy[q] = t * dy; sy[q + 4] = -t * dy;
            sz[q] = t * dz; sz[q + 4] = -t * dz;
            w[q] = wt; w[q + 4] = wt;
        }
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
        for (int p = 0; p < 8; ++p) {
            const double px = X + sx[p];
            for (int q = 0; q < 8; ++q) {
                const double py = Y + sy[q];
                const double wpq = w[p] * w[q];
                for (int s = 0; s < 8; ++s) {
                    const double pz = Z + sz[s];
                    const double r2 = px * px + py * py + pz * pz;
                    const double ir = rsqrt(r2);
                    const double ir2 = ir * ir;
                    const double k = wpq * w[s] * ir * ir2 * ir2;  // w / r^5
                    a0 += k * (r2 - 3.0 * px * px);
                    a1 += k * (r2 - 3.0 * py * py);
                    a2 += k * (r2 - 3.0 * pz * pz);
                    a3 -= k * 3.0 * px * py;
                    a4 -= k * 3.0 * px * pz;
                    a5 -= k * 3.0 * py * pz;
                }
            }
        }
        const double f = dx * dy * dz / (4.0 * M_PI);
        v[0] = a0 * f; v[1] = a1 * f; v[2] = a2 * f;
        v[3] = a3 * f; v[4] = a4 * f; v[5] = a5 * f;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) T[(long long)c * g.N + i] = v[c];
}

// Real transform of one axis of an octant-symmetric table (FP64):
//   out[o][k][in] = sum_{j < nj} w(j) cs(2 pi k j / P) src[o][j][in],  k < nk
// even: cs = cos, w(0) = 1, w(j>0) = 2 (the +-j pair); odd: cs = sin, w = 2.
// The full signed DFT of an odd-odd-even table is minus the product of these
// transforms (a factor -i per odd axis); the sign is applied when packing.
__global__ __launch_bounds__(kThreads) void k_axis_transform(const double *__restrict__ src,
                                                             double *__restrict__ out, int n_outer,
                                                             int nj, int n_inner, int P, int nk, int odd)
{
    __shared__ double cs[MAXL];
    for (int t = threadIdx.x; t < P; t += kThreads) {
        double s, c;
        sincospi(2.0 * (double)t / (double)P, &s, &c);
        cs[t] = odd ? s : c;
    }
    __syncthreads();
    const long long total = (long long)n_outer * nk * n_inner;
    for (long long idx = (long long)blockIdx.x * kThreads + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * kThreads) {
        const int in = (int)(idx % n_inner);
        const long long r = idx / n_inner;
        const int k = (int)(r % nk);
        const long long o = r / nk;
        const double *s = src + o * nj * (long long)n_inner + in;
        double acc = 0.0;
        for (int j = 0; j < nj; ++j) {
            const double w = (odd || j > 0) ? 2.0 : 1.0;
            acc += w * cs[(k * j) & (P - 1)] * s[(long long)j * n_inner];
        }
        out[idx] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void k_pack(Geo g, const double *__restrict__ T, int comp,
                                                   double scale, float *__restrict__ K)
{
    const long long total = (long long)g.Hx * g.Hy * g.Hz;
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= total) return;
    // T is [Hz][Hy][Hx]; K is [Hx][Hy][Hz][6]
    const int kx = (int)(idx % g.Hx);
    const long long r = idx / g.Hx;
    const int ky = (int)(r % g.Hy), kz = (int)(r / g.Hy);
    K[(((long long)kx * g.Hy + ky) * g.Hz + kz) * 6 + comp] = (float)(scale * T[idx]);
}

// ---------------------------------------------------------------- launchers

#define MM_LEN_CASES(X) X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

// Start/stop events for the next timed launch on this host thread.  The
// dispatch records them itself (hipExtLaunchKernelGGL), so their interval is
// the kernel's own execution, as a profiler's kernel trace reports it, without
// the gaps that event records around the launch would add.
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

void set_launch_events(hipEvent_t start, hipEvent_t stop)
{
    t_ev_start = start;
    t_ev_stop = stop;
}

bool launch_events_pending() { return t_ev_start != nullptr; }

void clear_launch_events() { t_ev_start = t_ev_stop = nullptr; }

#define MMK_LAUNCH(KERNEL, GRID, BLOCK, LDS, STREAM, ...)                                     \
    do {                                                                                    \
        if (t_ev_start) {                                                                   \
            hipEvent_t a_ = t_ev_start, b_ = t_ev_stop;                                     \
            t_ev_start = t_ev_stop = nullptr;                                               \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, a_, b_, 0, __VA_ARGS__); \
        } else {                                                                            \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);              \
        }                                                                                   \
    } while (0)

// Runs go(integral_constant<int, V>) for the variant to use: `var` for lines
// of kTuneMinL points or more, V = 0 otherwise.
template <int LL, typename F>
static void with_variant(int var, F &&go)
{
    if constexpr (LL >= kTuneMinL) {
        if (var == 1) return go(std::integral_constant<int, 1>{});
        if (var == 2) return go(std::integral_constant<int, 2>{});
    }
    go(std::integral_constant<int, 0>{});
}

// One z launch: the sequential-component kernel for SEQ shapes, else the
// concurrent one.
template <int LL, int VV, bool COMP, bool TAB>
static void zc_launch(dim3 grid, const PassArg<ZDesc, TAB> &a, hipStream_t s)
{
    using S = ZShape<LL, VV>;
    const size_t lds = S::LDS * sizeof(float2);
    if constexpr (S::SEQ)
        MMK_LAUNCH((k_zconv_seq<LL, COMP, VV, TAB>), grid, dim3(S::THREADS), lds, s, a);
    else if constexpr (LL == 64 && VV == 0 && S::CB == 16 && S::THREADS == 256 && S::NSUB == 1)
        MMK_LAUNCH((k_zconv64<COMP, TAB>), grid, dim3(256), 0, s, a);
    else
        MMK_LAUNCH((k_zconv<LL, COMP, VV, TAB>), grid, dim3(S::THREADS), lds, s, a);
}

int pass_variant(int pass, int L, int var)
{
    (void)pass;
    return (L >= kTuneMinL && var >= 0 && var < kVariants) ? var : 0;
}

// Per-sample grids.  x passes: (3 nz rows, y tiles); y passes: line blocks;
// z pass: (column tiles, kx); all shapes from the structs above.
template <int LL>
static long long x_blocks(const Geo &g, int var)
{
    long long n = 0;
    with_variant<LL>(var, [&](auto vt) {
        using S = XShape<LL, decltype(vt)::value>;
        n = 3LL * g.nz * ((g.ny + S::LPB - 1) / S::LPB);
    });
    return n;
}
template <int LL>
static long long y_blocks(const Geo &g, int var)
{
    long long n = 0;
    with_variant<LL>(var, [&](auto vt) {
        using S = YShape<LL, decltype(vt)::value>;
        n = (3LL * g.nz * g.Hx + S::LPB - 1) / S::LPB;
    });
    return n;
}
template <int LL>
static long long z_blocks(const Geo &g, int var)
{
    long long n = 0;
    with_variant<LL>(var, [&](auto vt) {
        using S = ZShape<LL, decltype(vt)::value>;
        constexpr int CT = S::CB * S::NSUB;
        n = (long long)((g.Py + CT - 1) / CT) * g.Hx;
    });
    return n;
}

long long pass_blocks(int pass, const Geo &g, int var)
{
    const int L = pass == 0 ? g.Px / 2 : (pass == 1 ? g.Py : g.Pz);
    switch (L) {
#define CASE(LL)                                                                              \
    case LL:                                                                                  \
        if constexpr (LL <= 512) {                                                            \
            if (pass == 0) return x_blocks<LL>(g, var);                                       \
        }                                                                                     \
        if (pass == 1) return y_blocks<LL>(g, var);                                           \
        return z_blocks<LL>(g, var);
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return -1;
    }
}

long long local_blocks(const Geo &g, bool vec)
{
    const long long items = vec ? g.N / 4 : g.N;
    return (items + kThreads - 1) / kThreads;
}

int local_perm(const Geo &g, bool vec) { return local_perm_q(g, (long long)kThreads * (vec ? 4 : 1), local_blocks(g, vec)); }

// ---- single sample: descriptor by value, the sample's own grid

hipError_t launch_xfwd(const Geo &g, const float *m, const float *ms_map, float ms, float2 *S1, hipStream_t s, int var)
{
    const PassArg<XfwdDesc, false> a{{g, m, ms_map, S1, ms}};
    switch (g.Px / 2) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        if constexpr (LL <= 512) {                                                            \
            with_variant<LL>(var, [&](auto vt) {                                              \
                using S = XShape<LL, decltype(vt)::value>;                                    \
                dim3 grid(3 * g.nz, (g.ny + S::LPB - 1) / S::LPB);                            \
                MMK_LAUNCH((k_xfwd<LL, decltype(vt)::value, false>), grid, dim3(S::THREADS),  \
                           S::LDS * sizeof(float2), s, a);                                    \
            });                                                                               \
        }                                                                                     \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xinv(const Geo &g, const float2 *S1, float *Hd, hipStream_t s, int var)
{
    const PassArg<XinvDesc, false> a{{g, S1, Hd}};
    switch (g.Px / 2) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        if constexpr (LL <= 512) {                                                            \
            with_variant<LL>(var, [&](auto vt) {                                              \
                using S = XShape<LL, decltype(vt)::value>;                                    \
                dim3 grid(3 * g.nz, (g.ny + S::LPB - 1) / S::LPB);                            \
                MMK_LAUNCH((k_xinv<LL, decltype(vt)::value, false>), grid, dim3(S::THREADS),  \
                           S::LDS * sizeof(float2), s, a);                                    \
            });                                                                               \
        }                                                                                     \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_y(const Geo &g, const float2 *in, float2 *out, bool inverse, hipStream_t s, int var)
{
    const PassArg<YDesc, false> a{{g, in, out}};
    switch (g.Py) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        with_variant<LL>(var, [&](auto vt) {                                                  \
            using S = YShape<LL, decltype(vt)::value>;                                        \
            dim3 grid((unsigned)((3LL * g.nz * g.Hx + S::LPB - 1) / S::LPB));                \
            if (inverse)                                                                      \
                MMK_LAUNCH((k_yinv<LL, decltype(vt)::value, false>), grid, dim3(kThreads),    \
                           S::LDS * sizeof(float2), s, a);                                    \
            else                                                                              \
                MMK_LAUNCH((k_yfwd<LL, decltype(vt)::value, false>), grid, dim3(kThreads),    \
                           S::LDS * sizeof(float2), s, a);                                    \
        });                                                                                   \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_yfwd(const Geo &g, const float2 *S1, float2 *S2, hipStream_t s, int var)
{
    return launch_y(g, S1, S2, false, s, var);
}
hipError_t launch_yinv(const Geo &g, const float2 *S2, float2 *S1, hipStream_t s, int var)
{
    return launch_y(g, S2, S1, true, s, var);
}

hipError_t launch_zconv(const Geo &g, float2 *S2, const float *K, bool comp, hipStream_t s, int var)
{
    const PassArg<ZDesc, false> a{{g, S2, K}};
    switch (g.Pz) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        with_variant<LL>(comp ? 0 : var, [&](auto vt) {                                       \
            constexpr int VV = decltype(vt)::value;                                           \
            using S = ZShape<LL, VV>;                                                         \
            constexpr int CT = S::CB * S::NSUB;                                               \
            const dim3 grid((g.Py + CT - 1) / CT, g.Hx);                                      \
            if (comp) {                                                                       \
                if constexpr (VV == 0) zc_launch<LL, 0, true, false>(grid, a, s);             \
            } else {                                                                          \
                zc_launch<LL, VV, false, false>(grid, a, s);                                  \
            }                                                                                 \
        });                                                                                   \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- many samples: descriptors and block map in device memory

template <typename Dsc>
static PassArg<Dsc, true> targ(const Table<Dsc> &t)
{
    return PassArg<Dsc, true>{t.desc};
}

template <typename Dsc>
static bool table_ok(const Table<Dsc> &t)
{
    return t.desc && t.width >= 1 && t.width <= 0x7fffffffLL && t.count >= 1 && t.count <= 65535;
}

template <typename Dsc>
static dim3 tgrid(const Table<Dsc> &t)
{
    return dim3((unsigned)t.width, (unsigned)t.count);
}

hipError_t launch_xfwd_table(const Table<XfwdDesc> &t, int Px, hipStream_t s, int var)
{
    if (!table_ok(t)) return hipErrorInvalidValue;
    const auto a = targ(t);
    switch (Px / 2) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        if constexpr (LL <= 512) {                                                            \
            with_variant<LL>(var, [&](auto vt) {                                              \
                using S = XShape<LL, decltype(vt)::value>;                                    \
                MMK_LAUNCH((k_xfwd<LL, decltype(vt)::value, true>), tgrid(t), \
                           dim3(S::THREADS), S::LDS * sizeof(float2), s, a);                  \
            });                                                                               \
        }                                                                                     \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xinv_table(const Table<XinvDesc> &t, int Px, hipStream_t s, int var)
{
    if (!table_ok(t)) return hipErrorInvalidValue;
    const auto a = targ(t);
    switch (Px / 2) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        if constexpr (LL <= 512) {                                                            \
            with_variant<LL>(var, [&](auto vt) {                                              \
                using S = XShape<LL, decltype(vt)::value>;                                    \
                MMK_LAUNCH((k_xinv<LL, decltype(vt)::value, true>), tgrid(t), \
                           dim3(S::THREADS), S::LDS * sizeof(float2), s, a);                  \
            });                                                                               \
        }                                                                                     \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_y_table(const Table<YDesc> &t, int Py, bool inverse, hipStream_t s, int var)
{
    if (!table_ok(t)) return hipErrorInvalidValue;
    const auto a = targ(t);
    switch (Py) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        with_variant<LL>(var, [&](auto vt) {                                                  \
            using S = YShape<LL, decltype(vt)::value>;                                        \
            if (inverse)                                                                      \
                MMK_LAUNCH((k_yinv<LL, decltype(vt)::value, true>), tgrid(t), \
                           dim3(kThreads), S::LDS * sizeof(float2), s, a);                    \
            else                                                                              \
                MMK_LAUNCH((k_yfwd<LL, decltype(vt)::value, true>), tgrid(t), \
                           dim3(kThreads), S::LDS * sizeof(float2), s, a);                    \
        });                                                                                   \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_yfwd_table(const Table<YDesc> &t, int Py, hipStream_t s, int var)
{
    return launch_y_table(t, Py, false, s, var);
}
hipError_t launch_yinv_table(const Table<YDesc> &t, int Py, hipStream_t s, int var)
{
    return launch_y_table(t, Py, true, s, var);
}

hipError_t launch_zconv_table(const Table<ZDesc> &t, int Pz, bool comp, hipStream_t s, int var)
{
    if (!table_ok(t)) return hipErrorInvalidValue;
    const auto a = targ(t);
    switch (Pz) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        with_variant<LL>(comp ? 0 : var, [&](auto vt) {                                       \
            constexpr int VV = decltype(vt)::value;                                           \
            if (comp) {                                                                       \
                if constexpr (VV == 0) zc_launch<LL, 0, true, true>(tgrid(t), a, s);          \
            } else {                                                                          \
                zc_launch<LL, VV, false, true>(tgrid(t), a, s);                               \
            }                                                                                 \
        });                                                                                   \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- local kernel

template <bool TAB>
static hipError_t launch_local_any(const PassArg<LocalDesc, TAB> &a, dim3 grid, bool vec, bool mapped,
                                   const LocalParams &p, uint32_t terms, int mode, float dt, int renorm,
                                   int *flag, hipStream_t s)
{
#define LOCAL(MODE, V)                                                                        \
    do {                                                                                      \
        if (mapped)                                                                           \
            MMK_LAUNCH((k_local<MODE, V, TAB, true>), grid, dim3(kThreads), 0, s, a, p, terms, dt, renorm, flag); \
        else                                                                                  \
            MMK_LAUNCH((k_local<MODE, V, TAB, false>), grid, dim3(kThreads), 0, s, a, p, terms, dt, renorm, flag); \
    } while (0)
    if (mode == 0) {
        if (vec) LOCAL(0, 4); else LOCAL(0, 1);
    } else if (mode == 1) {
        if (vec) LOCAL(1, 4); else LOCAL(1, 1);
    } else {
        if (vec) LOCAL(2, 4); else LOCAL(2, 1);
    }
#undef LOCAL
    return hipGetLastError();
}

hipError_t launch_local_table(const Table<LocalDesc> &t, bool vec, bool mapped, const LocalParams &p,
                              uint32_t terms, int mode, float dt, int renorm, int *flag, hipStream_t s)
{
    if (!table_ok(t)) return hipErrorInvalidValue;
    return launch_local_any(targ(t), tgrid(t), vec, mapped, p, terms, mode, dt, renorm, flag, s);
}

static hipError_t launch_local_one(LocalDesc d, const LocalParams &p, uint32_t terms, int mode, float dt,
                                   int renorm, int *flag, hipStream_t s)
{
    const bool vec = d.g.nx % 4 == 0;
    d.perm_q = local_perm(d.g, vec);
    const PassArg<LocalDesc, false> a{d};
    return launch_local_any(a, dim3((unsigned)local_blocks(d.g, vec)), vec, d.ms_map != nullptr, p, terms, mode, dt,
                            renorm, flag, s);
}

hipError_t launch_local(const Geo &g, const LocalParams &p, const float *m, const float *Hd,
                        const float *ms_map, const float *h_map, uint32_t terms, int mode, float dt,
                        int renorm, float *out_m, float *out_h, int *flag, hipStream_t s)
{
    LocalDesc d{g, m, Hd, ms_map, h_map, out_m, out_h, p.h0, p.h1, p.h2};
    return launch_local_one(d, p, terms, mode, dt, renorm, flag, s);
}

hipError_t launch_stage(const Geo &g, const LocalParams &p, const float *m, const float *Hd, const float *ms_map,
                        const float *h_map, const float *m_base, float *acc, float *eacc, float *kbuf, float dt,
                        int renorm, float *out_m, int *flag, hipStream_t s)
{
    LocalDesc d{g, m, Hd, ms_map, h_map, out_m, nullptr, p.h0, p.h1, p.h2, m_base, acc, eacc, kbuf};
    return launch_local_one(d, p, 15u, 2, dt, renorm, flag, s);
}

bool fused_xinv_euler_ok(const Geo &g)
{
    const int L = g.Px / 2;
    return L >= 4 && L <= 256 && g.nx <= L;
}

long long xe_blocks(const Geo &g)
{
    return (long long)g.nz * ((g.ny + MMK_XE_LPB - 1) / MMK_XE_LPB);
}

template <bool TAB, bool XF, bool MAPPED>
static hipError_t launch_xe_any(const PassArg<XeDesc, TAB> &a, dim3 grid, int Px, bool vec, const LocalParams &p,
                                float dt, int renorm, int *flag, hipStream_t s)
{
    switch (Px / 2) {
#define CASE(LL)                                                                              \
    case LL: {                                                                                \
        if constexpr (LL >= 4 && LL <= 256) {                                                 \
            using S = XEShape<LL, MMK_XE_LPB>;                                                \
            const size_t lds = S::LDS * sizeof(float2);                                       \
            if (vec)                                                                          \
                MMK_LAUNCH((k_xinv_euler<LL, MMK_XE_LPB, 4, TAB, XF, MAPPED>), grid, dim3(S::THREADS), lds, \
                           s, a, p, dt, renorm, flag);                                        \
            else                                                                              \
                MMK_LAUNCH((k_xinv_euler<LL, MMK_XE_LPB, 1, TAB, XF, MAPPED>), grid, dim3(S::THREADS), lds, \
                           s, a, p, dt, renorm, flag);                                        \
            return hipGetLastError();                                                         \
        }                                                                                     \
        break;                                                                                \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_xinv_euler(const Geo &g, const LocalParams &p, const float2 *S1, const float *m,
                             const float *ms_map, const float *h_map, float dt, int renorm, float *out_m,
                             float *hd_out, int *flag, hipStream_t s, float2 *S1_next)
{
    if (!fused_xinv_euler_ok(g) || (S1_next && (S1_next != S1 || ms_map))) return hipErrorInvalidValue;
    const PassArg<XeDesc, false> a{XeDesc{g, S1, m, h_map, ms_map, out_m, S1_next, hd_out, p.h0, p.h1, p.h2, 0}};
    const dim3 grid((unsigned)xe_blocks(g));
    const bool vec = g.nx % 4 == 0;
    if (S1_next) return launch_xe_any<false, true, false>(a, grid, g.Px, vec, p, dt, renorm, flag, s);
    if (ms_map) return launch_xe_any<false, false, true>(a, grid, g.Px, vec, p, dt, renorm, flag, s);
    return launch_xe_any<false, false, false>(a, grid, g.Px, vec, p, dt, renorm, flag, s);
}

hipError_t launch_xinv_euler_table(const Table<XeDesc> &t, int Px, bool vec, const LocalParams &p, float dt,
                                   int renorm, int *flag, hipStream_t s)
{
    if (!table_ok(t)) return hipErrorInvalidValue;
    return launch_xe_any<true, false, false>(targ(t), tgrid(t), Px, vec, p, dt, renorm, flag, s);
}

struct OpMax {
    __device__ unsigned operator()(unsigned a, unsigned b) const { return a > b ? a : b; }
};
struct OpOr {
    __device__ unsigned operator()(unsigned a, unsigned b) const { return a | b; }
};

// Maximum of n non-negative floats (NaN propagates): grid-stride loop,
// wavefront shuffles and the wavefronts' results per block, one atomicMax on
// the bit pattern per block.
__global__ __launch_bounds__(kThreads) void k_errmax(const float *__restrict__ e, long long n,
                                                     unsigned *__restrict__ out)
{
    __shared__ unsigned red[kThreads / 64];
    unsigned mx[1] = {0u};
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const unsigned v = __float_as_uint(e[i]);
        mx[0] = v > mx[0] ? v : mx[0];
    }
    block_reduce<1>(mx, red, OpMax{});
    if (threadIdx.x == 0) atomicMax(out, mx[0]);
}

// Checks an Ms map: out[0] |= 1 if some value is negative, NaN or infinite
// (its bit pattern is above that of the largest finite float), out[1] |= 1
// if some value is zero (a vacuum cell).
__global__ __launch_bounds__(kThreads) void k_map_check(const float *__restrict__ v, long long n,
                                                        unsigned *__restrict__ out)
{
    __shared__ unsigned red[kThreads / 64 * 2];
    unsigned f[2] = {0u, 0u};  // bad, zero
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const unsigned b = __float_as_uint(v[i]);
        f[0] |= b > 0x7f7fffffu ? 1u : 0u;
        f[1] |= b == 0u ? 1u : 0u;
    }
    block_reduce<2>(f, red, OpOr{});
    if (threadIdx.x == 0) {
        if (f[0]) atomicOr(out, 1u);
        if (f[1]) atomicOr(out + 1, 1u);
    }
}

hipError_t launch_map_check(const float *v, long long n, unsigned *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_map_check, dim3((unsigned)blocks), dim3(kThreads), 0, s, v, n, out);
    return hipGetLastError();
}

hipError_t launch_errmax(const float *e, long long n, unsigned *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_errmax, dim3((unsigned)blocks), dim3(kThreads), 0, s, e, n, out);
    return hipGetLastError();
}

hipError_t launch_diag_dot3(const float *in, float *out, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag_dot3, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, in, out,
                       n);
    return hipGetLastError();
}

hipError_t launch_adj_a(const Geo &g, const LocalParams &p, const float *m, const float *Hd, const float *ms_map,
                        const float *h_map, const float *lam1, float dt, int renorm, float *gH, float *lam_loc,
                        float *g_hext, float *g_ms, hipStream_t s)
{
    dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads));
    MMK_LAUNCH(k_adj_a, grid, dim3(kThreads), 0, s, g, p, m, Hd, ms_map, h_map, lam1, dt, renorm, gH,
                       lam_loc, g_hext, g_ms);
    return hipGetLastError();
}

hipError_t launch_adj_b(const Geo &g, const LocalParams &p, const float *m, const float *gH, const float *D,
                        const float *ms_map, const float *lam_loc, float *lam, float *g_ms, hipStream_t s)
{
    dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads));
    MMK_LAUNCH(k_adj_b, grid, dim3(kThreads), 0, s, g, p, m, gH, D, ms_map, lam_loc, lam, g_ms);
    return hipGetLastError();
}

hipError_t launch_energy(const Geo &g, const EnergyParams &p, const float *m, const float *Hd,
                         const float *ms_map, const float *h_map, double *partials, double *out,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(kEnergyBlocks), dim3(kThreads), 0, s, g, p, m, Hd, ms_map, h_map,
                       partials);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kThreads), 0, s, kEnergyBlocks, p, g.N, partials, out);
    return hipGetLastError();
}

hipError_t launch_tensor_octant(const Geo &g, double dx, double dy, double dz, double *T, hipStream_t s)
{
    dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_tensor_octant, grid, dim3(kThreads), 0, s, g, dx, dy, dz, T);
    return hipGetLastError();
}

static unsigned grid_for(long long total)
{
    long long b = (total + kThreads - 1) / kThreads;
    return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

hipError_t launch_tensor_spectrum(const Geo &g, const double *T, double *tmpA, double *tmpB, float *K,
                                  hipStream_t s)
{
    // parity per component along (x, y, z): 1 = odd
    static const int par[6][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    const double inv = 1.0 / ((double)g.Px * g.Py * g.Pz);
    for (int c = 0; c < 6; ++c) {
        const double *src = T + (long long)c * g.N;
        long long tot = (long long)g.nz * g.ny * g.Hx;
        hipLaunchKernelGGL(k_axis_transform, dim3(grid_for(tot)), dim3(kThreads), 0, s, src, tmpA,
                           g.nz * g.ny, g.nx, 1, g.Px, g.Hx, par[c][0]);
        tot = (long long)g.nz * g.Hy * g.Hx;
        hipLaunchKernelGGL(k_axis_transform, dim3(grid_for(tot)), dim3(kThreads), 0, s, tmpA, tmpB, g.nz,
                           g.ny, g.Hx, g.Py, g.Hy, par[c][1]);
        tot = (long long)g.Hz * g.Hy * g.Hx;
        hipLaunchKernelGGL(k_axis_transform, dim3(grid_for(tot)), dim3(kThreads), 0, s, tmpB, tmpA, 1, g.nz,
                           g.Hy * g.Hx, g.Pz, g.Hz, par[c][2]);
        // H = -IFFT(F . FFT(M)), IFFT carrying 1/(Px Py Pz); F = +product for the
        // diagonal components and -product for the odd-odd ones
        const double scale = (c < 3) ? -inv : inv;
        hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, g,
                           tmpA, c, scale, K);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Clock of the time-dependent external field: both slots set to t.  A kernel
// rather than a host copy, so it is ordered on the stream like the steps.
// ------------------------------------------------------------------------
__global__ void k_set_clock(double *clk, double t)
{
    if (threadIdx.x < 2) clk[threadIdx.x] = t;
}

hipError_t launch_set_clock(double *clk, double t, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, s, clk, t);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// FP64 loss L = 1/2 sum_i (m_i - t_i)^2 (the L2 mismatch of a final state
// to a target) and its gradient m - t.  Block b takes the kLossChunk values
// [b kLossChunk, (b+1) kLossChunk): each thread adds its values in order,
// the wavefront adds across lanes by shuffles, then the 4 wavefronts' sums
// are added in order.  The difference of two FP32 values is exact in FP64.
// ------------------------------------------------------------------------
constexpr int kLossItems = (int)(kLossChunk / kThreads);
static_assert(kLossChunk % kThreads == 0, "loss chunk is whole rows of the block");

__device__ __forceinline__ double block_sum256(double v, double *lds)
{
    double r[1] = {v};
    block_reduce<1>(r, lds, OpAdd{});
    return r[0];  // valid in thread 0
}

__global__ __launch_bounds__(kThreads) void k_loss(const float *__restrict__ m, const float *__restrict__ t,
                                                   long long n, float *__restrict__ grad,
                                                   double *__restrict__ partials)
{
    __shared__ double red[kThreads / 64];
    const long long base = (long long)blockIdx.x * kLossChunk + threadIdx.x;
    float a[kLossItems], b[kLossItems];
#pragma unroll
    for (int k = 0; k < kLossItems; ++k) {
        const long long i = base + (long long)k * kThreads;
        a[k] = i < n ? m[i] : 0.f;
        b[k] = i < n ? t[i] : 0.f;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kLossItems; ++k) {
        const double d = (double)a[k] - (double)b[k];
        acc = fma(d, d, acc);
        const long long i = base + (long long)k * kThreads;
        if (grad && i < n) grad[i] = a[k] - b[k];
    }
    const double r = block_sum256(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void k_loss_final(const double *__restrict__ partials, long long nblk,
                                                         double *__restrict__ out)
{
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    for (long long b = threadIdx.x; b < nblk; b += kThreads) acc += partials[b];
    const double r = block_sum256(acc, red);
    if (threadIdx.x == 0) out[0] = 0.5 * r;
}

hipError_t launch_loss(const float *m, const float *t, long long n, float *grad, double *partials, double *out,
                       hipStream_t s)
{
    const long long nb = loss_partials(n);
    if (n < 1 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_loss, dim3((unsigned)nb), dim3(kThreads), 0, s, m, t, n, grad, partials);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

}  // namespace mmk
