// launch.hpp -- host-side launchers of the gfx950 kernels (kernels.hip).
// Every launcher enqueues on `s` and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmk {

// Grid sizes and padded FFT sizes of one sample.
struct Geo {
    int nx, ny, nz;   // cells
    int Px, Py, Pz;   // padded lengths (powers of two, or 1 for a single-cell axis)
    int Hx, Hy, Hz;   // stored spectral lengths P/2 + 1 (1 when P = 1)
    long long N;      // nx*ny*nz
};

// Coefficients of the local field terms and of the LLG update, FP32.
struct LocalParams {
    float ms;            // uniform Ms (A/m), used when no map is given
    float ax, ay, az;    // 2A/(mu0 d^2) per axis: exchange field = (a/Ms) * sum (m_nb - m)
    float ku2;           // 2Ku/mu0: anisotropy field = (ku2/Ms) (m.u) u
    float u0, u1, u2;    // easy axis
    float h0, h1, h2;    // uniform external field (A/m)
    float c1, c2;        // LLG: f = c1 m x H + c2 m x (m x H)
    // mode 2, one Runge-Kutta stage with k = f(m, H(m)) at this stage's state:
    //   acc' = (first ? m_base : acc) + stage_b dt k
    //   last: m_out = P(acc');  else: acc = acc', m_out = P(m_base + stage_a dt k)
    //   stage_last = 2: error-only stage (no acc / m_out writes)
    // with the embedded error estimate (stage_err = 1 or 2):
    //   e' = (first ? 0 : eacc) + stage_e dt k;  1: eacc = e';  2: eacc[0][i] = |e'_i|
    float stage_a, stage_b, stage_e;
    int stage_first, stage_last, stage_err;
    // full tableau rows: the next state also adds dt sum_{jj < stage_nprev}
    // stage_ap[jj] kbuf[jj]; stage_kstore >= 0 stores this stage's k there
    float stage_ap[6];
    int stage_nprev, stage_kstore;
    // time-dependent external field (sched != 0): the field is scaled by
    // field_scale(t) with t = clk[tslot]; an Euler step (mode 1) also writes
    // clk[tslot ^ 1] = t + dt64 for the next step
    int sched, tslot;
    double *clk;
    double t_start, t_decay, t_stop, dt64;
};

// Per-sample arguments of one pass.
struct XfwdDesc {
    Geo g;
    const float *m;       // state [3][nz][ny][nx]
    const float *ms_map;  // per-cell Ms or NULL
    float2 *S1;           // x spectrum [3][nz][Hx][ny]
    float ms;             // uniform Ms (M = ms m when no map; 1 for a plain field)
};
struct YDesc {
    Geo g;
    const float2 *in;
    float2 *out;
};
struct ZDesc {
    Geo g;
    float2 *S2;      // [3][nz][Hx][Py], transformed in place
    const float *K;  // tensor spectrum of this padded size
};
struct XinvDesc {
    Geo g;
    const float2 *S1;
    float *Hd;  // H_demag [3][nz][ny][nx]
};
struct LocalDesc {
    Geo g;
    const float *m, *Hd, *ms_map, *h_map;
    float *m_out;  // Euler step output (mode 1), next stage state or step result (mode 2)
    float *h_out;  // field output (mode 0)
    float h0, h1, h2;  // uniform external field of this sample
    const float *m_base;  // mode 2: state at the start of the step
    float *acc;           // mode 2: m_base + dt sum_j b_j k_j so far (3N floats)
    float *eacc;          // mode 2: dt sum_j e_j k_j so far (3N floats); per-cell norm at the error stage
    float *kbuf;          // mode 2: stored slopes k_0, k_1, ... (3N floats each) for tableaus with full rows
    int perm_q;           // set by the launcher: blocks per XCD per z-plane of the block order (0: launch order)
};
// The fused x-inverse + Euler update of one sample: H_demag's x spectrum S1
// in, the state m read, the next state m_out written; with the chained
// x-forward, the next step's S1 (of m_out) written to S1w (the same array).
struct XeDesc {
    Geo g;
    const float2 *S1;
    const float *m, *h_map, *ms_map;
    float *m_out;
    float2 *S1w;
    float *hd_out;     // H_demag of every cell, when not NULL
    float h0, h1, h2;  // uniform external field of this sample (no map)
    int pad;
};
// Where a pass kernel finds its sample and its block within the sample.
//   TAB = false: one sample, its descriptor by value, the grid is the
//     sample's own (2-D for the x and z passes).
//   TAB = true: many samples; their descriptors live in device memory and
//     the grid is (blocks, samples): blockIdx.y is the sample, blockIdx.x
//     the block within that sample's own grid, flattened x-fastest.  The
//     grid is as wide as the launch's largest sample (a multiple of 8, so
//     every sample starts on the same XCD); a block beyond its sample's own
//     grid exits after reading the descriptor.
template <typename D, bool TAB>
struct PassArg;
template <typename D>
struct PassArg<D, false> {
    D d;
};
template <typename D>
struct PassArg<D, true> {
    const D *desc;
};

// A table launch: `count` descriptors in device memory, `width` blocks per
// sample (the grid is width x count).
template <typename D>
struct Table {
    const D *desc;
    long long width;
    int count;
};

// FP64 energy coefficients.
struct EnergyParams {
    double A, Ku, u0, u1, u2, ms, h0, h1, h2;
    double cx, cy, cz;  // 1/d^2
    double V;           // cell volume
    double mu0;
    uint32_t terms;
    // time-dependent external field as in LocalParams (read only)
    int sched, tslot;
    const double *clk;
    double t_start, t_decay, t_stop;
};

constexpr int kEnergyBlocks = 512;

// Partial sums the static scratch of the loss reduction holds: up to
// kScratchPartials * kLossChunk values (2 796 202 cells of 3 components).
constexpr long long kScratchPartials = 4096;

// once per device, with that device current: device tables, and the
// address of the static scratch array on this device
hipError_t init_tables(hipStream_t s, double **scratch_dev);

// Table launches of many samples.  Every sample of one launch has the
// transform length given (x: Px, y: Py, z: Pz); `var` selects a
// launch-shape variant (0 = default, 1, 2; see the shape structs in
// kernels.hip) for lines of 64 points or more, 0 otherwise, and the block map
// must be at least the largest sample's pass_blocks for that variant.
hipError_t launch_xfwd_table(const Table<XfwdDesc> &t, int Px, hipStream_t s, int var = 0);
hipError_t launch_yfwd_table(const Table<YDesc> &t, int Py, hipStream_t s, int var = 0);
hipError_t launch_zconv_table(const Table<ZDesc> &t, int Pz, bool compensated, hipStream_t s, int var = 0);
hipError_t launch_yinv_table(const Table<YDesc> &t, int Py, hipStream_t s, int var = 0);
hipError_t launch_xinv_table(const Table<XinvDesc> &t, int Px, hipStream_t s, int var = 0);
// local terms + Euler step (mode 1) or field output (mode 0) of many samples;
// vec: every sample has nx % 4 == 0 (4 cells per thread); mapped: some
// sample has an Ms map
hipError_t launch_local_table(const Table<LocalDesc> &t, bool vec, bool mapped, const LocalParams &p,
                              uint32_t terms, int mode, float dt, int renorm, int *flag, hipStream_t s);

// Blocks of one sample's own grid (what its map entries count) for a pass
// (0: x passes, 1: y passes, 2: z pass) with launch-shape variant var, and
// for the local kernel (vec as above); local_perm: the XCD block order of
// that sample's local grid (LocalDesc::perm_q).
long long pass_blocks(int pass, const Geo &g, int var);
long long local_blocks(const Geo &g, bool vec);
int local_perm(const Geo &g, bool vec);
// the variant a table launch of this pass and length actually uses
int pass_variant(int pass, int L, int var);

// Timing: events that the next launch of a timed kernel on this host thread
// records itself at dispatch start and end.  launch_events_pending() tells
// whether they are still unused after a launcher returned.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();
void clear_launch_events();

// single-sample forms
hipError_t launch_xfwd(const Geo &g, const float *m, const float *ms_map, float ms, float2 *S1, hipStream_t s,
                       int var = 0);
hipError_t launch_yfwd(const Geo &g, const float2 *S1, float2 *S2, hipStream_t s, int var = 0);
hipError_t launch_zconv(const Geo &g, float2 *S2, const float *K, bool compensated, hipStream_t s, int var = 0);
hipError_t launch_yinv(const Geo &g, const float2 *S2, float2 *S1, hipStream_t s, int var = 0);
hipError_t launch_xinv(const Geo &g, const float2 *S1, float *Hd, hipStream_t s, int var = 0);

// local terms: mode 0 writes H to out_h, mode 1 writes the Euler step to out_m
hipError_t launch_local(const Geo &g, const LocalParams &p, const float *m, const float *Hd,
                        const float *ms_map, const float *h_map, uint32_t terms, int mode,
                        float dt, int renorm, float *out_m, float *out_h, int *flag, hipStream_t s);
// a5-a8 in one launch: x-inverse of S1 (H_demag kept on chip) + local terms +
// Euler step of m into out_m; for 8 <= Px <= 512 and nx <= Px/2
// (fused_xinv_euler_ok)
bool fused_xinv_euler_ok(const Geo &g);
// ms_map: per-cell Ms (vacuum where 0) or NULL; hd_out != NULL also stores
// H_demag of every cell there.  S1_next != NULL (uniform Ms only): the
// launch also runs the next step's x-forward of out_m (as launch_xfwd with
// Ms = p.ms) into S1_next, which must be S1 itself
hipError_t launch_xinv_euler(const Geo &g, const LocalParams &p, const float2 *S1, const float *m,
                             const float *ms_map, const float *h_map, float dt, int renorm, float *out_m,
                             float *hd_out, int *flag, hipStream_t s, float2 *S1_next = nullptr);
// the same for many samples of one padded x length Px and one update width
// (vec: nx % 4 == 0); every sample fused_xinv_euler_ok
hipError_t launch_xinv_euler_table(const Table<XeDesc> &t, int Px, bool vec, const LocalParams &p, float dt,
                                   int renorm, int *flag, hipStream_t s);
// blocks of one sample's own grid of the fused pass
long long xe_blocks(const Geo &g);
// one Runge-Kutta stage (all field terms; coefficients in p.stage_*): reads
// m (the stage state), Hd = H_demag(m), m_base and acc; writes out_m and acc
hipError_t launch_stage(const Geo &g, const LocalParams &p, const float *m, const float *Hd, const float *ms_map,
                        const float *h_map, const float *m_base, float *acc, float *eacc, float *kbuf, float dt,
                        int renorm, float *out_m, int *flag, hipStream_t s);
// out (one unsigned, zeroed by the caller) <- bits of max(e[0..n)) for e >= 0
// or NaN (NaN wins: its bit pattern orders above every finite value)
hipError_t launch_errmax(const float *e, long long n, unsigned *out, hipStream_t s);
hipError_t launch_diag_dot3(const float *in, float *out, long long n, hipStream_t s);
// out[0] |= 1 if a value of v[0..n) is negative or not finite, out[1] |= 1
// if a value is zero (out zeroed by the caller)
hipError_t launch_map_check(const float *v, long long n, unsigned *out, hipStream_t s);

// adjoint of one Euler step: local part (a) and the non-local completion (b)
hipError_t launch_adj_a(const Geo &g, const LocalParams &p, const float *m, const float *Hd, const float *ms_map,
                        const float *h_map, const float *lam1, float dt, int renorm, float *gH, float *lam_loc,
                        float *g_hext, float *g_ms, hipStream_t s);
hipError_t launch_adj_b(const Geo &g, const LocalParams &p, const float *m, const float *gH, const float *D,
                        const float *ms_map, const float *lam_loc, float *lam, float *g_ms, hipStream_t s);

// FP64 reductions
hipError_t launch_energy(const Geo &g, const EnergyParams &p, const float *m, const float *Hd,
                         const float *ms_map, const float *h_map, double *partials, double *out,
                         hipStream_t s);

// device clock of the time-dependent field: clk[0] = clk[1] = t
hipError_t launch_set_clock(double *clk, double t, hipStream_t s);

// FP64 loss 1/2 sum_i (m_i - t_i)^2 over n values into out[0], and m - t
// into grad (FP32) when grad is not null.  Each block reduces one chunk of
// kLossChunk consecutive values into partials[b] (loss_partials(n) slots),
// one block then adds the partials in block order: deterministic.
constexpr long long kLossChunk = 2048;
constexpr long long loss_partials(long long n) { return (n + kLossChunk - 1) / kLossChunk; }
hipError_t launch_loss(const float *m, const float *t, long long n, float *grad, double *partials, double *out,
                       hipStream_t s);

// FP64 tensor build
hipError_t launch_tensor_octant(const Geo &g, double dx, double dy, double dz, double *T, hipStream_t s);
hipError_t launch_tensor_spectrum(const Geo &g, const double *T, double *tmpA, double *tmpB, float *K,
                                  hipStream_t s);

}  // namespace mmk
