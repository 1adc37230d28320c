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

hipError_t init_tables(hipStream_t s)
{
    hipLaunchKernelGGL(k_init_tw, dim3(MAXL / 256), dim3(256), 0, s);
    return hipGetLastError();
}

constexpr int kThreads = 256;
constexpr int kLdsComplex = 4096;  // complex values per LDS buffer (32 KB)

__host__ __device__ constexpr int pow2floor(int v)
{
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}
__host__ __device__ constexpr int lines_per_block(int L, int cap)
{
    return (kLdsComplex / L) < cap ? (kLdsComplex / L) : cap;
}

// ------------------------------------------------------------------------
// a1: x-forward real FFT.  A real line x[0..Px) (nx non-zeros) is packed as
// z[k] = x[2k] + i x[2k+1], k < L = Px/2, transformed with a length-L complex
// FFT, and unpacked with X[k] = E[k] + exp(-2 pi i k/Px) O[k],
// E[k] = (Z[k] + conj Z[L-k])/2, O[k] = (Z[k] - conj Z[L-k])/(2i).
// ------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(kThreads) void k_xfwd(Geo g, const float *__restrict__ m,
                                                   const float *__restrict__ ms_map, float ms,
                                                   float2 *__restrict__ S1)
{
    constexpr int TL = lines_per_block(L, 64);
    extern __shared__ float2 sm[];
    float2 *a = sm, *b = sm + TL * L;
    const int c = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * TL;
    const int nl = min(TL, g.ny - y0);
    const long long cell0 = ((long long)z * g.ny + y0) * g.nx;
    const float *mrow = m + (long long)c * g.N + cell0;
    const float *srow = ms_map ? ms_map + cell0 : nullptr;
    for (int idx = threadIdx.x; idx < TL * L; idx += kThreads) {
        const int t = idx / L, k = idx - t * L;
        float2 v = make_float2(0.f, 0.f);
        const int x0 = 2 * k;
        if (t < nl) {
            const long long o = (long long)t * g.nx + x0;
            if (x0 < g.nx) v.x = (srow ? srow[o] : ms) * mrow[o];
            if (x0 + 1 < g.nx) v.y = (srow ? srow[o + 1] : ms) * mrow[o + 1];
        }
        a[idx] = v;
    }
    const float2 *r = lds_fft<L, false>(a, b, TL, L);
    float2 *out = S1 + ((long long)(c * g.nz + z) * g.Hx) * g.ny + y0;
    for (int idx = threadIdx.x; idx < (L + 1) * TL; idx += kThreads) {
        const int kx = idx / TL, t = idx - kx * TL;
        if (t >= nl) continue;
        const float2 *Z = r + t * L;
        const float2 zk = Z[kx & (L - 1)];
        const float2 zc = cconj(Z[(L - kx) & (L - 1)]);
        const float2 E = cscale(cadd(zk, zc), 0.5f);
        const float2 O = mul_mi<false>(cscale(csub(zk, zc), 0.5f));
        out[(long long)kx * g.ny + t] = cadd(E, cmul(twiddle<false>(kx, 2 * L), O));
    }
}

// ------------------------------------------------------------------------
// a2 / a4: FFT along y of contiguous columns (length Py, ny non-zeros in /
// ny kept out).
// ------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(kThreads) void k_yfwd(Geo g, const float2 *__restrict__ S1,
                                                   float2 *__restrict__ S2)
{
    constexpr int TK = lines_per_block(L, 64);
    extern __shared__ float2 sm[];
    float2 *a = sm, *b = sm + TK * L;
    const int c = blockIdx.z, z = blockIdx.y, k0 = blockIdx.x * TK;
    const int nk = min(TK, g.Hx - k0);
    const long long col0 = (long long)(c * g.nz + z) * g.Hx + k0;
    const float2 *in = S1 + col0 * g.ny;
    for (int idx = threadIdx.x; idx < TK * L; idx += kThreads) {
        const int t = idx / L, y = idx - t * L;
        a[idx] = (t < nk && y < g.ny) ? in[(long long)t * g.ny + y] : make_float2(0.f, 0.f);
    }
    const float2 *r = lds_fft<L, false>(a, b, TK, L);
    float2 *out = S2 + col0 * L;
    for (int idx = threadIdx.x; idx < nk * L; idx += kThreads) out[idx] = r[idx];
}

template <int L>
__global__ __launch_bounds__(kThreads) void k_yinv(Geo g, const float2 *__restrict__ S2,
                                                   float2 *__restrict__ S1)
{
    constexpr int TK = lines_per_block(L, 64);
    extern __shared__ float2 sm[];
    float2 *a = sm, *b = sm + TK * L;
    const int c = blockIdx.z, z = blockIdx.y, k0 = blockIdx.x * TK;
    const int nk = min(TK, g.Hx - k0);
    const long long col0 = (long long)(c * g.nz + z) * g.Hx + k0;
    const float2 *in = S2 + col0 * L;
    for (int idx = threadIdx.x; idx < TK * L; idx += kThreads)
        a[idx] = idx < nk * L ? in[idx] : make_float2(0.f, 0.f);
    const float2 *r = lds_fft<L, true>(a, b, TK, L);
    float2 *out = S1 + col0 * g.ny;
    for (int idx = threadIdx.x; idx < TK * g.ny; idx += kThreads) {
        const int t = idx / g.ny, y = idx - t * g.ny;
        if (t < nk) out[(long long)t * g.ny + y] = r[t * L + y];
    }
}

// ------------------------------------------------------------------------
// a3: z transform + tensor multiply + inverse z transform, per (kx, ky).
// K holds the octant kx in [0,Hx), ky in [0,Hy), kz in [0,Hz) as
// K[kx][ky][kz][6] (xx, yy, zz, xy, xz, yz).  Components odd in y (xy, yz)
// change sign for ky > Py/2, components odd in z (xz, yz) for kz > Pz/2.
// Compensated form: each of the six real dot products of three terms is
// accumulated with an error-free product (fma) and two-sum and rounded once.
// ------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ float dot3_comp(float k0, float x0, float k1, float x1, float k2, float x2)
{
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

template <int L, bool COMP>
__global__ __launch_bounds__(kThreads) void k_zconv(Geo g, float2 *__restrict__ S2,
                                                    const float *__restrict__ K)
{
    constexpr int TYr = pow2floor(1365 / L);
    constexpr int TY = TYr > 256 ? 256 : (TYr < 1 ? 1 : TYr);
    extern __shared__ float2 sm[];
    float2 *a = sm, *b = sm + 3 * TY * L;
    const int kx = blockIdx.y, ky0 = blockIdx.x * TY;
    const int nyl = min(TY, g.Py - ky0);
    const long long plane = (long long)g.Hx * g.Py;  // stride between z planes
    float2 *base = S2 + (long long)kx * g.Py + ky0;
    for (int idx = threadIdx.x; idx < 3 * TY * L; idx += kThreads) {
        const int t = idx % TY, rest = idx / TY;
        const int zz = rest % L, c = rest / L;
        float2 v = make_float2(0.f, 0.f);
        if (t < nyl && zz < g.nz) v = base[((long long)c * g.nz + zz) * plane + t];
        a[(c * TY + t) * L + zz] = v;
    }
    float2 *r = lds_fft<L, false>(a, b, 3 * TY, L);
    float2 *o = (r == a) ? b : a;
    const int hy = g.Py / 2, hz = g.Pz / 2;
    for (int idx = threadIdx.x; idx < TY * L; idx += kThreads) {
        const int kz = idx / TY, t = idx - kz * TY;
        if (t >= nyl) continue;
        const int ky = ky0 + t;
        const bool fy = ky > hy, fz = kz > hz;
        const int kyf = fy ? g.Py - ky : ky, kzf = fz ? g.Pz - kz : kz;
        const float *k6 = K + (((long long)kx * g.Hy + kyf) * g.Hz + kzf) * 6;
        const float sy = fy ? -1.f : 1.f, sz = fz ? -1.f : 1.f;
        const float kxx = k6[0], kyy = k6[1], kzz = k6[2];
        const float kxy = sy * k6[3], kxz = sz * k6[4], kyz = sy * sz * k6[5];
        float2 *px = r + (0 * TY + t) * L + kz;
        float2 *py = r + (1 * TY + t) * L + kz;
        float2 *pz = r + (2 * TY + t) * L + kz;
        const float2 mx = *px, my = *py, mz = *pz;
        float2 hx, hy2, hz2;
        if (COMP) {
            hx = make_float2(dot3_comp(kxx, mx.x, kxy, my.x, kxz, mz.x), dot3_comp(kxx, mx.y, kxy, my.y, kxz, mz.y));
            hy2 = make_float2(dot3_comp(kxy, mx.x, kyy, my.x, kyz, mz.x), dot3_comp(kxy, mx.y, kyy, my.y, kyz, mz.y));
            hz2 = make_float2(dot3_comp(kxz, mx.x, kyz, my.x, kzz, mz.x), dot3_comp(kxz, mx.y, kyz, my.y, kzz, mz.y));
        } else {
            hx = make_float2(fmaf(kxx, mx.x, fmaf(kxy, my.x, kxz * mz.x)), fmaf(kxx, mx.y, fmaf(kxy, my.y, kxz * mz.y)));
            hy2 = make_float2(fmaf(kxy, mx.x, fmaf(kyy, my.x, kyz * mz.x)), fmaf(kxy, mx.y, fmaf(kyy, my.y, kyz * mz.y)));
            hz2 = make_float2(fmaf(kxz, mx.x, fmaf(kyz, my.x, kzz * mz.x)), fmaf(kxz, mx.y, fmaf(kyz, my.y, kzz * mz.y)));
        }
        *px = hx;
        *py = hy2;
        *pz = hz2;
    }
    const float2 *q = lds_fft<L, true>(r, o, 3 * TY, L);
    for (int idx = threadIdx.x; idx < 3 * TY * g.nz; idx += kThreads) {
        const int t = idx % TY, rest = idx / TY;
        const int zz = rest % g.nz, c = rest / g.nz;
        if (t < nyl) base[((long long)c * g.nz + zz) * plane + t] = q[(c * TY + t) * L + zz];
    }
}

// ------------------------------------------------------------------------
// a5: x-inverse real FFT (keep nx of Px outputs).  From the half spectrum
// X[0..L] (L = Px/2): Z'[k] = (X[k] + conj X[L-k]) + i (X[k] - conj X[L-k])
// exp(+2 pi i k/Px); the unnormalised inverse length-L FFT of Z' is
// x[2n] + i x[2n+1].
// ------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(kThreads) void k_xinv(Geo g, const float2 *__restrict__ S1,
                                                   float *__restrict__ Hd)
{
    constexpr int TL = lines_per_block(L, 64);
    extern __shared__ float2 sm[];
    float2 *a = sm, *b = sm + TL * L;
    const int c = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * TL;
    const int nl = min(TL, g.ny - y0);
    const float2 *in = S1 + ((long long)(c * g.nz + z) * g.Hx) * g.ny + y0;
    // pairs (k, L-k) for k in [0, L/2]; k = 0 pairs X[0] with X[L]
    constexpr int HP = L / 2 + 1;
    for (int idx = threadIdx.x; idx < HP * TL; idx += kThreads) {
        const int k = idx / TL, t = idx - k * TL;
        float2 xk = make_float2(0.f, 0.f), xl = make_float2(0.f, 0.f);
        if (t < nl) {
            xk = in[(long long)k * g.ny + t];
            xl = in[(long long)(L - k) * g.ny + t];
        }
        {
            const float2 xc = cconj(xl);
            const float2 E = cadd(xk, xc);
            const float2 O = cmul(csub(xk, xc), twiddle<true>(k, 2 * L));
            a[t * L + (k & (L - 1))] = cadd(E, mul_mi<true>(O));
        }
        if (k > 0 && 2 * k < L) {
            const float2 xc = cconj(xk);
            const float2 E = cadd(xl, xc);
            const float2 O = cmul(csub(xl, xc), twiddle<true>(L - k, 2 * L));
            a[t * L + (L - k)] = cadd(E, mul_mi<true>(O));
        }
    }
    const float2 *r = lds_fft<L, true>(a, b, TL, L);
    float *out = Hd + (long long)c * g.N + ((long long)z * g.ny + y0) * g.nx;
    for (int idx = threadIdx.x; idx < nl * g.nx; idx += kThreads) {
        const int t = idx / g.nx, x = idx - t * g.nx;
        const float2 v = r[t * L + (x >> 1)];
        out[(long long)t * g.nx + x] = (x & 1) ? v.y : v.x;
    }
}

// ------------------------------------------------------------------------
// a6-a8: local field terms and the explicit Euler LLG step, per cell.
//   H = H_demag + (2A/(mu0 Ms)) sum_nb (m_nb - m)/d^2 + (2Ku/(mu0 Ms)) (m.u) u + h_ext
//   f = c1 m x H + c2 m x (m x H),  c1 = -gamma0/(1+alpha^2), c2 = alpha c1
//   m' = m + dt f, then m' /= |m'| unless renormalisation is off.
// Free (Neumann) boundaries: a missing neighbour contributes nothing.
// ------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_local(Geo g, LocalParams p, const float *__restrict__ m,
                                                    const float *__restrict__ Hd,
                                                    const float *__restrict__ ms_map,
                                                    const float *__restrict__ h_map, uint32_t terms,
                                                    float dt, int renorm, float *__restrict__ out_m,
                                                    float *__restrict__ out_h, int *__restrict__ flag)
{
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= g.N) return;
    const long long N = g.N;
    const int x = (int)(i % g.nx);
    const long long r = i / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const float mx = m[i], my = m[N + i], mz = m[2 * N + i];
    float hx = 0.f, hy = 0.f, hz = 0.f;
    if ((terms & 2u) && Hd) {
        hx = Hd[i];
        hy = Hd[N + i];
        hz = Hd[2 * N + i];
    }
    const float ms = ms_map ? ms_map[i] : p.ms;
    const float inv_ms = 1.0f / ms;
    if (terms & 1u) {
        float lx = 0.f, ly = 0.f, lz = 0.f;
        const long long sy = g.nx, sz = (long long)g.nx * g.ny;
        auto add = [&](long long j, float w) {
            lx = fmaf(w, m[j] - mx, lx);
            ly = fmaf(w, m[N + j] - my, ly);
            lz = fmaf(w, m[2 * N + j] - mz, lz);
        };
        if (x > 0) add(i - 1, p.ax);
        if (x < g.nx - 1) add(i + 1, p.ax);
        if (y > 0) add(i - sy, p.ay);
        if (y < g.ny - 1) add(i + sy, p.ay);
        if (z > 0) add(i - sz, p.az);
        if (z < g.nz - 1) add(i + sz, p.az);
        hx = fmaf(lx, inv_ms, hx);
        hy = fmaf(ly, inv_ms, hy);
        hz = fmaf(lz, inv_ms, hz);
    }
    if (terms & 4u) {
        const float k = p.ku2 * inv_ms * (mx * p.u0 + my * p.u1 + mz * p.u2);
        hx = fmaf(k, p.u0, hx);
        hy = fmaf(k, p.u1, hy);
        hz = fmaf(k, p.u2, hz);
    }
    if (terms & 8u) {
        if (h_map) {
            hx += h_map[i];
            hy += h_map[N + i];
            hz += h_map[2 * N + i];
        } else {
            hx += p.h0;
            hy += p.h1;
            hz += p.h2;
        }
    }
    if (MODE == 0) {
        out_h[i] = hx;
        out_h[N + i] = hy;
        out_h[2 * N + i] = hz;
        return;
    }
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
    if (!(isfinite(nx_) && isfinite(ny_) && isfinite(nz_))) *flag = 1;
    out_m[i] = nx_;
    out_m[N + i] = ny_;
    out_m[2 * N + i] = nz_;
}

// ------------------------------------------------------------------------
// a9: FP64 energy terms and mean magnetisation.  Per-block partial sums in a
// fixed order, then one block sums the partials: deterministic.
// ------------------------------------------------------------------------
constexpr int kEq = 7;  // e_ex, e_d, e_an, e_z, sum mx, sum my, sum mz

__global__ __launch_bounds__(kThreads) void k_energy(Geo g, EnergyParams p, const float *__restrict__ m,
                                                     const float *__restrict__ Hd,
                                                     const float *__restrict__ ms_map,
                                                     const float *__restrict__ h_map,
                                                     double *__restrict__ partials)
{
    __shared__ double red[kEq][kThreads];
    double acc[kEq] = {0, 0, 0, 0, 0, 0, 0};
    const long long N = g.N;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < N;
         i += (long long)gridDim.x * kThreads) {
        const double mx = m[i], my = m[N + i], mz = m[2 * N + i];
        const int x = (int)(i % g.nx);
        const long long r = i / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        const double ms = ms_map ? (double)ms_map[i] : p.ms;
        if (p.terms & 1u) {
            auto pair = [&](long long j, double w) {
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
            acc[3] += ms * (mx * h0 + my * h1 + mz * h2);
        }
        acc[4] += mx;
        acc[5] += my;
        acc[6] += mz;
    }
#pragma unroll
    for (int q = 0; q < kEq; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < kEq; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < kEq) partials[(long long)blockIdx.x * kEq + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kThreads) void k_energy_final(int nblk, EnergyParams p, long long N,
                                                           const double *__restrict__ partials,
                                                           double *__restrict__ out)
{
    __shared__ double red[kEq][kThreads];
    double acc[kEq] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += kThreads)
#pragma unroll
        for (int q = 0; q < kEq; ++q) acc[q] += partials[(long long)b * kEq + q];
#pragma unroll
    for (int q = 0; q < kEq; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < kEq; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double eex = (p.terms & 1u) ? p.A * p.V * red[0][0] : 0.0;
        const double ed = (p.terms & 2u) ? -0.5 * p.mu0 * p.V * red[1][0] : 0.0;
        const double ean = (p.terms & 4u) ? p.Ku * p.V * red[2][0] : 0.0;
        const double ez = (p.terms & 8u) ? -p.mu0 * p.V * red[3][0] : 0.0;
        out[0] = eex;
        out[1] = ed;
        out[2] = ean;
        out[3] = ez;
        out[4] = eex + ed + ean + ez;
        out[5] = red[4][0] / (double)N;
        out[6] = red[5][0] / (double)N;
        out[7] = red[6][0] / (double)N;
    }
}

// ------------------------------------------------------------------------
// a0: FP64 demag tensor.  N(o) between two cells o cells apart:
//  near (all |o_a| <= 8): Newell's closed form, the second difference over
//    the 27-point stencil of the auxiliary functions f (diagonal) and g
//    (off-diagonal), divided by 4 pi V;
//  far: (1/V) integral over s in [-d,d]^3 of the dipole kernel
//    K(r) = (I/r^3 - 3 r r^T/r^5)/(4 pi) at r = o d + s, weighted by
//    prod (d_a - |s_a|); each half-axis with 4-point Gauss-Legendre.
// ------------------------------------------------------------------------
constexpr int kNearCells = 8;

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
    if (ox <= kNearCells && oy <= kNearCells && oz <= kNearCells) {
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

hipError_t launch_xfwd(const Geo &g, const float *m, const float *ms_map, float ms, float2 *S1, hipStream_t s)
{
    const int L = g.Px / 2;
    switch (L) {
#define CASE(LL)                                                                          \
    case LL: {                                                                            \
        if constexpr (LL <= 512) {                                                        \
            constexpr int TL = lines_per_block(LL, 64);                                   \
            dim3 grid((g.ny + TL - 1) / TL, g.nz, 3);                                     \
            hipLaunchKernelGGL(k_xfwd<LL>, grid, dim3(kThreads), 2 * TL * LL * sizeof(float2), s, \
                               g, m, ms_map, ms, S1);                                     \
        }                                                                                 \
        break;                                                                            \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xinv(const Geo &g, const float2 *S1, float *Hd, hipStream_t s)
{
    const int L = g.Px / 2;
    switch (L) {
#define CASE(LL)                                                                          \
    case LL: {                                                                            \
        if constexpr (LL <= 512) {                                                        \
            constexpr int TL = lines_per_block(LL, 64);                                   \
            dim3 grid((g.ny + TL - 1) / TL, g.nz, 3);                                     \
            hipLaunchKernelGGL(k_xinv<LL>, grid, dim3(kThreads), 2 * TL * LL * sizeof(float2), s, \
                               g, S1, Hd);                                                \
        }                                                                                 \
        break;                                                                            \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_yfwd(const Geo &g, const float2 *S1, float2 *S2, hipStream_t s)
{
    switch (g.Py) {
#define CASE(LL)                                                                          \
    case LL: {                                                                            \
        constexpr int TK = lines_per_block(LL, 64);                                       \
        dim3 grid((g.Hx + TK - 1) / TK, g.nz, 3);                                         \
        hipLaunchKernelGGL(k_yfwd<LL>, grid, dim3(kThreads), 2 * TK * LL * sizeof(float2), s, g, \
                           S1, S2);                                                       \
        break;                                                                            \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_yinv(const Geo &g, const float2 *S2, float2 *S1, hipStream_t s)
{
    switch (g.Py) {
#define CASE(LL)                                                                          \
    case LL: {                                                                            \
        constexpr int TK = lines_per_block(LL, 64);                                       \
        dim3 grid((g.Hx + TK - 1) / TK, g.nz, 3);                                         \
        hipLaunchKernelGGL(k_yinv<LL>, grid, dim3(kThreads), 2 * TK * LL * sizeof(float2), s, g, \
                           S2, S1);                                                       \
        break;                                                                            \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zconv(const Geo &g, float2 *S2, const float *K, bool comp, hipStream_t s)
{
    switch (g.Pz) {
#define CASE(LL)                                                                          \
    case LL: {                                                                            \
        constexpr int TYr = pow2floor(1365 / LL);                                         \
        constexpr int TY = TYr > 256 ? 256 : (TYr < 1 ? 1 : TYr);                         \
        dim3 grid((g.Py + TY - 1) / TY, g.Hx, 1);                                         \
        const size_t lds = 2 * 3 * TY * LL * sizeof(float2);                              \
        if (comp)                                                                         \
            hipLaunchKernelGGL((k_zconv<LL, true>), grid, dim3(kThreads), lds, s, g, S2, K); \
        else                                                                              \
            hipLaunchKernelGGL((k_zconv<LL, false>), grid, dim3(kThreads), lds, s, g, S2, K); \
        break;                                                                            \
    }
        MM_LEN_CASES(CASE)
#undef CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_local(const Geo &g, const LocalParams &p, const float *m, const float *Hd,
                        const float *ms_map, const float *h_map, uint32_t terms, int mode, float dt,
                        int renorm, float *out_m, float *out_h, int *flag, hipStream_t s)
{
    dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads));
    if (mode == 0)
        hipLaunchKernelGGL(k_local<0>, grid, dim3(kThreads), 0, s, g, p, m, Hd, ms_map, h_map, terms, dt,
                           renorm, out_m, out_h, flag);
    else
        hipLaunchKernelGGL(k_local<1>, grid, dim3(kThreads), 0, s, g, p, m, Hd, ms_map, h_map, terms, dt,
                           renorm, out_m, out_h, flag);
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

}  // namespace mmk
