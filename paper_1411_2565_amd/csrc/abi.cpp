// abi.cpp -- the C ABI of include/mm.h: argument checks, padded sizes,
// workspace carving and the order of kernel launches for one step.
//
// Paper: Zhu, "Grace" (arXiv:1411.2565).  Sec. 3: every step evaluates the
// demagnetising field by zero-padded FFT convolution, adds the six-neighbour
// exchange field, anisotropy and external field, and applies one explicit
// Euler step of eq. (3); the data stays on the GPU between steps and only
// the caller's explicit reads cross to the host.
#include "mm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"

namespace {

constexpr double kMu0 = 4.0e-7 * M_PI;
constexpr int kMaxN = 512;

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

}  // namespace

struct mm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    mmk::Geo g{};
    double d[3] = {0, 0, 0};
    mm_material mat{};
    bool have_mat = false;
    double hext[3] = {0, 0, 0};
    bool ms_map = false, h_map = false, tensor = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    // workspace layout (byte offsets)
    size_t o_K = 0, o_S1 = 0, o_S2 = 0, o_mtmp = 0, o_rk = 0, o_T = 0, o_tA = 0, o_tB = 0;
    size_t o_ms = 0, o_h = 0, o_part = 0, o_lpart = 0, o_flag = 0, o_adj = 0, total = 0;
    bool compensated = false;  // compensated spectral multiply in every demag evaluation
    int fusion = 1;            // Euler steps: 0 two kernels, 1 x-inverse + update fused, 2 also the next x-forward
    bool vacuum = false;       // the Ms map holds vacuum cells (Ms = 0)
    int tune[3] = {0, 0, 0};   // launch-shape variants of the x, y and z passes
    // time-dependent external field: profile times, and which slot of the
    // device clock holds the time of the next step (toggled per Euler step)
    bool sched = false;
    double sched_t[3] = {0, 0, 0};
    int tslot = 0;
    std::string err;
    // captured step chunks (MM_F_GRAPH): kernel arguments (state pointer,
    // material, fields, maps, dt) are baked in, so every setter drops them
    struct GraphEntry {
        const float *m;
        int64_t n;
        double dt;
        uint32_t flags;
        hipStream_t stream;
        int tslot;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    void drop_graphs()
    {
        for (auto &e : graphs) (void)hipGraphExecDestroy(e.exec);
        graphs.clear();
    }
    // diagnostic per-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev_free;
    struct Pending { int kernel; hipEvent_t a, b; };
    std::vector<Pending> pending;
    double t_ms[MM_K_COUNT] = {0};
    int64_t t_n[MM_K_COUNT] = {0};

    ~mm_ctx()
    {
        drop_graphs();
        for (auto &p : pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (auto e : ev_free) (void)hipEventDestroy(e);
    }

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

mm_status fail(mm_ctx *c, mm_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

mm_status hipcheck(mm_ctx *c, hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(c, MM_EHIP, "%s: %s", what, hipGetErrorString(e));
    return MM_OK;
}

#define MM_TRY(expr)                        \
    do {                                    \
        mm_status _s = (expr);              \
        if (_s != MM_OK) return _s;         \
    } while (0)

int padded(int n)
{
    if (n == 1) return 1;
    int p = 1;
    while (p < 2 * n - 1) p *= 2;
    return p;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

std::mutex g_init_mu;
bool g_init_done[64] = {false};
// per device: address of the library's static scratch array (see
// mm_reduce_loss_noalloc), looked up once with that device current
double *g_scratch[64] = {nullptr};

// device tables (twiddles) once per device, with that device current
mm_status init_device(mm_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (c->device < 0 || c->device >= 64) return fail(c, MM_EINVAL, "device index %d out of range", c->device);
    if (g_init_done[c->device]) return MM_OK;
    double *sc = nullptr;
    MM_TRY(hipcheck(c, mmk::init_tables(c->stream, &sc), "init_tables"));
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "init_tables sync"));
    if (!sc) return fail(c, MM_EHIP, "no device address for the static scratch");
    g_scratch[c->device] = sc;
    g_init_done[c->device] = true;
    return MM_OK;
}

void layout(mm_ctx *c)
{
    const mmk::Geo &g = c->g;
    const size_t N = (size_t)g.N;
    Carve cv;
    c->o_K = cv.take(sizeof(float) * 6 * (size_t)g.Hx * g.Hy * g.Hz);
    c->o_ms = cv.take(sizeof(float) * N);
    c->o_h = cv.take(sizeof(float) * 3 * N);
    c->o_part = cv.take(sizeof(double) * 8 * mmk::kEnergyBlocks + sizeof(double) * 8);
    c->o_lpart = cv.take(sizeof(double) * (size_t)mmk::loss_partials(3 * (long long)N));
    c->o_flag = cv.take(256);
    c->o_adj = cv.take(sizeof(float) * 6 * N);  // adjoint: g_H and the local part of lambda
    // region shared by the step buffers and the tensor-build temporaries
    const size_t region = cv.off;
    Carve st;
    st.off = region;
    c->o_S1 = st.take(sizeof(float2) * 3 * (size_t)g.nz * g.Hx * g.ny);
    c->o_S2 = st.take(sizeof(float2) * 3 * (size_t)g.nz * g.Hx * g.Py);
    c->o_mtmp = st.take(sizeof(float) * 3 * N);
    // Runge-Kutta: two stage states, accumulator, error accumulator, four stored slopes
    c->o_rk = st.take(sizeof(float) * 24 * N);
    Carve tb;
    tb.off = region;
    c->o_T = tb.take(sizeof(double) * 6 * N);
    size_t a1 = (size_t)g.nz * g.ny * g.Hx, a2 = (size_t)g.Hz * g.Hy * g.Hx;
    c->o_tA = tb.take(sizeof(double) * (a1 > a2 ? a1 : a2));
    c->o_tB = tb.take(sizeof(double) * (size_t)g.nz * g.Hy * g.Hx);
    c->total = st.off > tb.off ? st.off : tb.off;
}

// fold completed event pairs into the per-kernel totals (stream synchronised)
mm_status drain_timing(mm_ctx *c)
{
    if (c->pending.empty()) return MM_OK;
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "timing sync"));
    for (auto &p : c->pending) {
        float ms = 0.f;
        MM_TRY(hipcheck(c, hipEventElapsedTime(&ms, p.a, p.b), "event elapsed"));
        c->t_ms[p.kernel] += ms;
        c->t_n[p.kernel] += 1;
        c->ev_free.push_back(p.a);
        c->ev_free.push_back(p.b);
    }
    c->pending.clear();
    return MM_OK;
}

hipEvent_t take_event(mm_ctx *c)
{
    if (c->ev_free.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
}

// run one single-kernel launcher; when timing is on, the kernel's dispatch
// records a start and a stop event (its own execution interval)
template <typename F>
mm_status timed(mm_ctx *c, int kernel, const char *what, F &&launch)
{
    if (!c->timing) return hipcheck(c, launch(), what);
    // folding needs a synchronisation: only when many pairs are pending, so a
    // timed region of a few thousand launches runs without one
    if (c->pending.size() >= 16384) MM_TRY(drain_timing(c));
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return fail(c, MM_EHIP, "hipEventCreate failed");
    mmk::set_launch_events(a, b);
    const hipError_t e = launch();
    const bool used = !mmk::launch_events_pending();
    mmk::clear_launch_events();
    if (e != hipSuccess || !used) {
        c->ev_free.push_back(a);
        c->ev_free.push_back(b);
        if (e == hipSuccess) return fail(c, MM_EHIP, "%s: timed launcher did not take the dispatch events", what);
        return hipcheck(c, e, what);
    }
    c->pending.push_back({kernel, a, b});
    return MM_OK;
}

mm_status need_ws(mm_ctx *c)
{
    if (!c->ws) return fail(c, MM_ESTATE, "no workspace set (mm_set_workspace)");
    return MM_OK;
}

mm_status set_device(mm_ctx *c) { return hipcheck(c, hipSetDevice(c->device), "hipSetDevice"); }

// the device clock of the time-dependent field: two FP64 slots in the flag block
double *clock_ptr(const mm_ctx *c) { return reinterpret_cast<double *>(c->at<char>(c->o_flag) + 192); }

mmk::LocalParams local_params(const mm_ctx *c)
{
    mmk::LocalParams p{};
    const mm_material &m = c->mat;
    p.ms = (float)m.Ms;
    p.ax = (float)(2.0 * m.A / (kMu0 * c->d[0] * c->d[0]));
    p.ay = (float)(2.0 * m.A / (kMu0 * c->d[1] * c->d[1]));
    p.az = (float)(2.0 * m.A / (kMu0 * c->d[2] * c->d[2]));
    p.ku2 = (float)(2.0 * m.Ku / kMu0);
    p.u0 = (float)m.u[0];
    p.u1 = (float)m.u[1];
    p.u2 = (float)m.u[2];
    p.h0 = (float)c->hext[0];
    p.h1 = (float)c->hext[1];
    p.h2 = (float)c->hext[2];
    const double c1 = -m.gamma0 / (1.0 + m.alpha * m.alpha);
    p.c1 = (float)c1;
    p.c2 = (float)(m.alpha * c1);
    p.stage_kstore = -1;  // no stored slopes unless a tableau asks for them
    p.stage_nprev = 0;
    p.sched = c->sched ? 1 : 0;
    p.tslot = c->tslot;
    p.clk = c->ws ? clock_ptr(c) : nullptr;
    p.t_start = c->sched_t[0];
    p.t_decay = c->sched_t[1];
    p.t_stop = c->sched_t[2];
    return p;
}

const float *ms_map_ptr(const mm_ctx *c) { return c->ms_map ? c->at<float>(c->o_ms) : nullptr; }
const float *h_map_ptr(const mm_ctx *c) { return c->h_map ? c->at<float>(c->o_h) : nullptr; }

// The demag spectrum of m (M = Ms m, or M = m when unit_ms): the x-forward,
// y-forward, z-convolution and y-inverse passes, leaving H_demag's x spectrum
// in S1.
mm_status demag_spectrum(mm_ctx *c, const float *m, bool comp, bool unit_ms = false, bool have_s1 = false)
{
    const mmk::Geo &g = c->g;
    float2 *S1 = c->at<float2>(c->o_S1), *S2 = c->at<float2>(c->o_S2);
    const float *K = c->at<float>(c->o_K);
    hipStream_t s = c->stream;
    const float *msm = unit_ms ? nullptr : ms_map_ptr(c);
    const float ms = unit_ms ? 1.0f : (float)c->mat.Ms;
    comp = comp || c->compensated;
    const int *tv = c->tune;
    if (!have_s1)  // else S1 already holds m's x spectrum (the previous step's chained x-forward)
        MM_TRY(timed(c, MM_K_XFWD, "xfwd", [&] { return mmk::launch_xfwd(g, m, msm, ms, S1, s, tv[0]); }));
    MM_TRY(timed(c, MM_K_YFWD, "yfwd", [&] { return mmk::launch_yfwd(g, S1, S2, s, tv[1]); }));
    MM_TRY(timed(c, MM_K_ZCONV, "zconv", [&] { return mmk::launch_zconv(g, S2, K, comp, s, tv[2]); }));
    MM_TRY(timed(c, MM_K_YINV, "yinv", [&] { return mmk::launch_yinv(g, S2, S1, s, tv[1]); }));
    return MM_OK;
}

// H_demag of m into `out` or, if NULL, the S2 region (aliased, 3N floats);
// *Hd receives the pointer
mm_status demag(mm_ctx *c, const float *m, bool comp, float **Hd, float *out = nullptr, bool unit_ms = false)
{
    MM_TRY(demag_spectrum(c, m, comp, unit_ms));
    float *H = out ? out : c->at<float>(c->o_S2);
    const float2 *S1 = c->at<float2>(c->o_S1);
    MM_TRY(timed(c, MM_K_XINV, "xinv", [&] { return mmk::launch_xinv(c->g, S1, H, c->stream, c->tune[0]); }));
    *Hd = H;
    return MM_OK;
}

mm_status check_step_args(mm_ctx *c, const float *m, int64_t nsteps, double dt, uint32_t flags)
{
    if (!m || !aligned16(m)) return fail(c, MM_EINVAL, "m must be a 16-byte aligned device pointer");
    if (nsteps < 0) return fail(c, MM_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, MM_EINVAL, "dt must be finite and > 0");
    if (flags & ~uint32_t(MM_F_NO_RENORM | MM_F_COMPENSATED | MM_F_HEUN | MM_F_RK4))
        return fail(c, MM_EINVAL, "unknown flag bits 0x%x", flags);
    if ((flags & MM_F_HEUN) && (flags & MM_F_RK4)) return fail(c, MM_EINVAL, "MM_F_HEUN and MM_F_RK4 together");
    MM_TRY(need_ws(c));
    if (!c->have_mat) return fail(c, MM_ESTATE, "material not set");
    if (!c->tensor) return fail(c, MM_ESTATE, "mm_build_tensor has not been called");
    return MM_OK;
}

}  // namespace

extern "C" {

mm_status mm_create(mm_ctx **out, const mm_geometry *geo, int device, void *hip_stream)
{
    if (!out || !geo) return MM_EINVAL;
    *out = nullptr;
    if (geo->nx < 2 || geo->nx > kMaxN || geo->ny < 1 || geo->ny > kMaxN || geo->nz < 1 || geo->nz > kMaxN)
        return MM_EINVAL;
    if (!(geo->dx > 0) || !(geo->dy > 0) || !(geo->dz > 0) || !std::isfinite(geo->dx) ||
        !std::isfinite(geo->dy) || !std::isfinite(geo->dz))
        return MM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MM_EINVAL;
    mm_ctx *c = new (std::nothrow) mm_ctx();
    if (!c) return MM_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    mmk::Geo &g = c->g;
    g.nx = geo->nx;
    g.ny = geo->ny;
    g.nz = geo->nz;
    g.Px = padded(g.nx);
    g.Py = padded(g.ny);
    g.Pz = padded(g.nz);
    g.Hx = g.Px / 2 + 1;
    g.Hy = g.Py == 1 ? 1 : g.Py / 2 + 1;
    g.Hz = g.Pz == 1 ? 1 : g.Pz / 2 + 1;
    g.N = (long long)g.nx * g.ny * g.nz;
    c->d[0] = geo->dx;
    c->d[1] = geo->dy;
    c->d[2] = geo->dz;
    layout(c);
    mm_status s = set_device(c);
    if (s == MM_OK) s = init_device(c);
    if (s != MM_OK) {
        delete c;
        return s;
    }
    *out = c;
    return MM_OK;
}

mm_status mm_destroy(mm_ctx *c)
{
    if (!c) return MM_EINVAL;
    delete c;
    return MM_OK;
}

mm_status mm_set_stream(mm_ctx *c, void *hip_stream)
{
    if (!c) return MM_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return MM_OK;
}

mm_status mm_workspace_size(const mm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return MM_EINVAL;
    *bytes = c->total;
    return MM_OK;
}

mm_status mm_set_workspace(mm_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c) return MM_EINVAL;
    if (!dev_ptr) return fail(c, MM_EINVAL, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) return fail(c, MM_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < c->total)
        return fail(c, MM_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", bytes, c->total);
    c->ws = static_cast<char *>(dev_ptr);
    c->ws_bytes = bytes;
    c->drop_graphs();
    c->tensor = false;
    c->ms_map = false;
    c->h_map = false;
    MM_TRY(set_device(c));
    MM_TRY(hipcheck(c, hipMemsetAsync(c->at<int>(c->o_flag), 0, sizeof(int), c->stream), "clear flag"));
    c->tslot = 0;
    return hipcheck(c, mmk::launch_set_clock(clock_ptr(c), 0.0, c->stream), "set clock");
}

mm_status mm_set_material(mm_ctx *c, const mm_material *m)
{
    if (!c) return MM_EINVAL;
    if (!m) return fail(c, MM_EINVAL, "material is NULL");
    const double un = std::sqrt(m->u[0] * m->u[0] + m->u[1] * m->u[1] + m->u[2] * m->u[2]);
    if (!(m->Ms > 0) || !std::isfinite(m->Ms)) return fail(c, MM_EINVAL, "Ms must be > 0");
    if (!(m->A >= 0) || !std::isfinite(m->A)) return fail(c, MM_EINVAL, "A must be >= 0");
    if (!(m->Ku >= 0) || !std::isfinite(m->Ku)) return fail(c, MM_EINVAL, "Ku must be >= 0");
    if (!(un > 0) || !std::isfinite(un)) return fail(c, MM_EINVAL, "anisotropy axis must be non-zero");
    if (!(m->alpha >= 0) || !std::isfinite(m->alpha)) return fail(c, MM_EINVAL, "alpha must be >= 0");
    if (!(m->gamma0 > 0) || !std::isfinite(m->gamma0)) return fail(c, MM_EINVAL, "gamma0 must be > 0");
    c->mat = *m;
    for (int i = 0; i < 3; ++i) c->mat.u[i] = m->u[i] / un;
    c->have_mat = true;
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_set_ms_map(mm_ctx *c, const float *ms)
{
    if (!c) return MM_EINVAL;
    MM_TRY(need_ws(c));
    if (!ms) {
        c->ms_map = false;
        c->drop_graphs();
        return MM_OK;
    }
    if (!aligned16(ms)) return fail(c, MM_EINVAL, "Ms map must be 16-byte aligned");
    MM_TRY(set_device(c));
    c->drop_graphs();
    c->ms_map = false;
    MM_TRY(hipcheck(c, hipMemcpyAsync(c->at<float>(c->o_ms), ms, sizeof(float) * c->g.N, hipMemcpyDeviceToDevice,
                                      c->stream), "copy Ms map"));
    unsigned *chk = reinterpret_cast<unsigned *>(c->at<char>(c->o_flag) + 128);
    unsigned res[2] = {0u, 0u};
    MM_TRY(hipcheck(c, hipMemsetAsync(chk, 0, sizeof(res), c->stream), "clear map check"));
    MM_TRY(hipcheck(c, mmk::launch_map_check(c->at<float>(c->o_ms), c->g.N, chk, c->stream), "check Ms map"));
    MM_TRY(hipcheck(c, hipMemcpyAsync(res, chk, sizeof(res), hipMemcpyDeviceToHost, c->stream), "read map check"));
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "map check sync"));
    if (res[0]) return fail(c, MM_EINVAL, "Ms map values must be finite and >= 0 (0 marks vacuum)");
    c->ms_map = true;
    c->vacuum = res[1] != 0;
    return MM_OK;
}

mm_status mm_set_hext(mm_ctx *c, const double h[3])
{
    if (!c) return MM_EINVAL;
    if (!h) return fail(c, MM_EINVAL, "field is NULL");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(h[i])) return fail(c, MM_EINVAL, "field must be finite");
    for (int i = 0; i < 3; ++i) c->hext[i] = h[i];
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_set_hext_map(mm_ctx *c, const float *h)
{
    if (!c) return MM_EINVAL;
    MM_TRY(need_ws(c));
    if (!h) {
        c->h_map = false;
        c->drop_graphs();
        return MM_OK;
    }
    if (!aligned16(h)) return fail(c, MM_EINVAL, "field map must be 16-byte aligned");
    MM_TRY(set_device(c));
    MM_TRY(hipcheck(c, hipMemcpyAsync(c->at<float>(c->o_h), h, sizeof(float) * 3 * c->g.N, hipMemcpyDeviceToDevice,
                                      c->stream), "copy field map"));
    c->h_map = true;
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_set_field_schedule(mm_ctx *c, const double sched[3])
{
    if (!c) return MM_EINVAL;
    if (!sched) {
        c->sched = false;
        c->drop_graphs();
        return MM_OK;
    }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(sched[i])) return fail(c, MM_EINVAL, "schedule times must be finite");
    if (!(sched[0] <= sched[1] && sched[1] <= sched[2]))
        return fail(c, MM_EINVAL, "schedule needs t_start <= t_decay <= t_stop");
    for (int i = 0; i < 3; ++i) c->sched_t[i] = sched[i];
    c->sched = true;
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_set_time(mm_ctx *c, double t)
{
    if (!c) return MM_EINVAL;
    if (!std::isfinite(t)) return fail(c, MM_EINVAL, "time must be finite");
    MM_TRY(need_ws(c));
    MM_TRY(set_device(c));
    return hipcheck(c, mmk::launch_set_clock(clock_ptr(c), t, c->stream), "set clock");
}

mm_status mm_get_time(mm_ctx *c, double *t)
{
    if (!c) return MM_EINVAL;
    if (!t) return fail(c, MM_EINVAL, "t is NULL");
    MM_TRY(need_ws(c));
    MM_TRY(set_device(c));
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "clock sync"));
    return hipcheck(c, hipMemcpy(t, clock_ptr(c) + c->tslot, sizeof(double), hipMemcpyDeviceToHost), "read clock");
}

mm_status mm_tensor_table(mm_ctx *c, double *tab)
{
    if (!c) return MM_EINVAL;
    if (!tab || !aligned16(tab)) return fail(c, MM_EINVAL, "table pointer must be non-NULL and 16-byte aligned");
    MM_TRY(set_device(c));
    MM_TRY(hipcheck(c, mmk::launch_tensor_octant(c->g, c->d[0], c->d[1], c->d[2], tab, c->stream), "tensor octant"));
    return hipcheck(c, hipStreamSynchronize(c->stream), "tensor table sync");
}

mm_status mm_diag_dot3(mm_ctx *c, const float *in, float *out, int64_t n)
{
    if (!c) return MM_EINVAL;
    if (n < 0 || n > ((int64_t)1 << 31)) return fail(c, MM_EINVAL, "n must be in [0, 2^31]");
    if (n == 0) return MM_OK;
    if (!in || !out) return fail(c, MM_EINVAL, "in and out must be non-NULL");
    MM_TRY(set_device(c));
    MM_TRY(hipcheck(c, mmk::launch_diag_dot3(in, out, n, c->stream), "dot3 diagnostic"));
    return hipcheck(c, hipStreamSynchronize(c->stream), "dot3 diagnostic sync");
}

mm_status mm_build_tensor(mm_ctx *c)
{
    if (!c) return MM_EINVAL;
    MM_TRY(need_ws(c));
    MM_TRY(set_device(c));
    double *T = c->at<double>(c->o_T);
    MM_TRY(hipcheck(c, mmk::launch_tensor_octant(c->g, c->d[0], c->d[1], c->d[2], T, c->stream), "tensor octant"));
    MM_TRY(hipcheck(c, mmk::launch_tensor_spectrum(c->g, T, c->at<double>(c->o_tA), c->at<double>(c->o_tB),
                                                   c->at<float>(c->o_K), c->stream),
                    "tensor spectrum"));
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "tensor build sync"));
    c->tensor = true;
    return MM_OK;
}

mm_status mm_compute_heff(mm_ctx *c, const float *m, float *h, uint32_t terms)
{
    if (!c) return MM_EINVAL;
    if (!m || !h || !aligned16(m) || !aligned16(h)) return fail(c, MM_EINVAL, "m and h must be 16-byte aligned device pointers");
    if (m == h) return fail(c, MM_EINVAL, "h may not alias m");
    if (terms & ~uint32_t(MM_T_ALL)) return fail(c, MM_EINVAL, "unknown term bits 0x%x", terms);
    MM_TRY(need_ws(c));
    if (!c->have_mat) return fail(c, MM_ESTATE, "material not set");
    if ((terms & MM_T_DEMAG) && !c->tensor) return fail(c, MM_ESTATE, "demag requested before mm_build_tensor");
    MM_TRY(set_device(c));
    float *Hd = nullptr;
    if (terms & MM_T_DEMAG) MM_TRY(demag(c, m, false, &Hd));
    const mmk::LocalParams p = local_params(c);
    return timed(c, MM_K_LOCAL, "local field", [&] {
        return mmk::launch_local(c->g, p, m, Hd, ms_map_ptr(c), h_map_ptr(c), terms, 0, 0.f, 0, nullptr, h,
                                 c->at<int>(c->o_flag), c->stream);
    });
}

}  // extern "C"

namespace {

// Enqueue nsteps Euler steps: step s reads src(s), writes the new state to
// dst(s) and, when hd(s) is not null, H_demag of src(s) there.  mm_step_llg
// and mm_forward_store both go through here, so a replay from a stored state
// reproduces the forward run bit for bit.
template <class Src, class Dst, class HdOut>
mm_status run_steps(mm_ctx *c, int64_t nsteps, double dt, uint32_t flags, Src src, Dst dst, HdOut hd)
{
    mmk::LocalParams p = local_params(c);
    const bool comp = flags & MM_F_COMPENSATED;
    const int renorm = (flags & MM_F_NO_RENORM) ? 0 : 1;
    int *flag = c->at<int>(c->o_flag);
    if (flags & (MM_F_HEUN | MM_F_RK4)) {
        // explicit Runge-Kutta with a_{i+1} = A[i+1][i] the only nonzero
        // entry of each row (true of Heun and classic RK4): stage i reads
        // state i, writes state i+1 from m_base and its own k_i
        const bool heun = flags & MM_F_HEUN;
        const int ns = heun ? 2 : 4;
        static const float a_heun[2] = {1.f, 0.f}, b_heun[2] = {0.5f, 0.5f};
        static const float a_rk4[4] = {0.5f, 0.5f, 1.f, 0.f};
        static const float b_rk4[4] = {1.f / 6.f, 1.f / 3.f, 1.f / 3.f, 1.f / 6.f};
        const size_t S = 3 * (size_t)c->g.N;
        float *stage[2] = {c->at<float>(c->o_rk), c->at<float>(c->o_rk) + S};
        float *acc = c->at<float>(c->o_rk) + 2 * S;
        for (int64_t s = 0; s < nsteps; ++s) {
            const float *base = src(s);
            const float *eval = base;
            for (int i = 0; i < ns; ++i) {
                float *Hd = nullptr;
                MM_TRY(demag(c, eval, comp, &Hd, hd(s)));
                p.stage_a = heun ? a_heun[i] : a_rk4[i];
                p.stage_b = heun ? b_heun[i] : b_rk4[i];
                p.stage_first = i == 0;
                p.stage_last = i == ns - 1;
                float *out = p.stage_last ? dst(s) : stage[i & 1];
                MM_TRY(timed(c, MM_K_LOCAL, "runge-kutta stage", [&] {
                    return mmk::launch_stage(c->g, p, eval, Hd, ms_map_ptr(c), h_map_ptr(c), base, acc, nullptr,
                                             nullptr, (float)dt, renorm, out, flag, c->stream);
                }));
                eval = out;
            }
        }
        return MM_OK;
    }
    p.dt64 = dt;
    // the x-inverse and the update as one pass (H_demag stays on chip, and
    // goes to hd(s) too where that is asked for); at fusion level 2 and a
    // uniform Ms that pass also runs the next step's x-forward of the state
    // it writes, so the next step skips its own x-forward
    const bool fuse = c->fusion >= 1 && mmk::fused_xinv_euler_ok(c->g);
    const bool chain = fuse && c->fusion >= 2 && !c->ms_map;
    bool have_s1 = false;
    for (int64_t s = 0; s < nsteps; ++s) {
        float *hs = hd(s);
        if (fuse) {
            MM_TRY(demag_spectrum(c, src(s), comp, false, have_s1));
            p.tslot = c->tslot;
            if (c->sched) c->tslot ^= 1;  // this step's kernel writes the next step's time
            const bool xf = chain && s + 1 < nsteps;
            float2 *S1 = c->at<float2>(c->o_S1);
            MM_TRY(timed(c, xf ? MM_K_XINV_LOCAL_XFWD : MM_K_XINV_LOCAL, "x-inverse + llg step", [&] {
                return mmk::launch_xinv_euler(c->g, p, S1, src(s), ms_map_ptr(c), h_map_ptr(c), (float)dt, renorm,
                                              dst(s), hs, flag, c->stream, xf ? S1 : nullptr);
            }));
            have_s1 = xf;
            continue;
        }
        have_s1 = false;
        float *Hd = nullptr;
        MM_TRY(demag(c, src(s), comp, &Hd, hs));
        p.tslot = c->tslot;
        if (c->sched) c->tslot ^= 1;  // this step's kernel writes the next step's time
        MM_TRY(timed(c, MM_K_LOCAL, "llg step", [&] {
            return mmk::launch_local(c->g, p, src(s), Hd, ms_map_ptr(c), h_map_ptr(c), MM_T_ALL, 1, (float)dt,
                                     renorm, dst(s), nullptr, flag, c->stream);
        }));
    }
    return MM_OK;
}

// One attempted step of an embedded pair from `base` to `out` with step h;
// the stream is synchronised and *err receives max over cells of the local
// error estimate |h sum_i (b_i - bh_i) k_i|.
//   2(1) Heun / Euler:      a = (1), b = (1/2, 1/2), bh = (1, 0)
//   3(2) Bogacki-Shampine:  a = (1/2, 3/4), b = (2/9, 1/3, 4/9), a fourth
//                           stage at the result, bh = (7/24, 1/4, 1/3, 1/8)
//   5(4) Dormand-Prince:    the published 1980 tableau, seven stages, the
//                           seventh at the result; rows with several
//                           nonzero entries read earlier slopes back
enum class Pair { HeunEuler, BS23, DP54 };

mm_status embedded_step(mm_ctx *c, const float *base, float *out, double h, Pair pair, uint32_t flags, float *err)
{
    mmk::LocalParams p = local_params(c);
    const bool comp = flags & MM_F_COMPENSATED;
    const int renorm = (flags & MM_F_NO_RENORM) ? 0 : 1;
    int *flag = c->at<int>(c->o_flag);
    unsigned *emax = reinterpret_cast<unsigned *>(c->at<char>(c->o_flag) + 64);
    const size_t S = 3 * (size_t)c->g.N;
    float *rk = c->at<float>(c->o_rk);
    float *stage[2] = {rk, rk + S};
    float *acc = rk + 2 * S, *eacc = rk + 3 * S, *kbuf = rk + 4 * S;  // kbuf: 4 slopes
    // a: weight of this stage's k in the next state; ap: weights of the
    // stored slopes k_0..k_{nprev-1}; last: 0 next state, 1 result, 2 error
    // only; err: 1 accumulate, 2 accumulate and reduce; kstore: slot or -1
    struct St {
        double a, b, e;
        int last, err, kstore, nprev;
        double ap[4];
    };
    static const St heun[2] = {{1.0, 0.5, -0.5, 0, 1, -1, 0, {0}}, {0.0, 0.5, 0.5, 1, 2, -1, 0, {0}}};
    static const St bs[4] = {{0.5, 2.0 / 9.0, 2.0 / 9.0 - 7.0 / 24.0, 0, 1, -1, 0, {0}},
                             {0.75, 1.0 / 3.0, 1.0 / 3.0 - 0.25, 0, 1, -1, 0, {0}},
                             {0.0, 4.0 / 9.0, 4.0 / 9.0 - 1.0 / 3.0, 1, 1, -1, 0, {0}},
                             {0.0, 0.0, -0.125, 2, 2, -1, 0, {0}}};
    static const St dp[7] = {
        {1.0 / 5.0, 35.0 / 384.0, 35.0 / 384.0 - 5179.0 / 57600.0, 0, 1, 0, 0, {0}},
        {9.0 / 40.0, 0.0, 0.0, 0, 1, 1, 1, {3.0 / 40.0}},
        {32.0 / 9.0, 500.0 / 1113.0, 500.0 / 1113.0 - 7571.0 / 16695.0, 0, 1, 2, 2, {44.0 / 45.0, -56.0 / 15.0}},
        {-212.0 / 729.0, 125.0 / 192.0, 125.0 / 192.0 - 393.0 / 640.0, 0, 1, 3, 3,
         {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0}},
        {-5103.0 / 18656.0, -2187.0 / 6784.0, -2187.0 / 6784.0 + 92097.0 / 339200.0, 0, 1, -1, 4,
         {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0}},
        {0.0, 11.0 / 84.0, 11.0 / 84.0 - 187.0 / 2100.0, 1, 1, -1, 0, {0}},
        {0.0, 0.0, -1.0 / 40.0, 2, 2, -1, 0, {0}}};
    const St *tab = pair == Pair::HeunEuler ? heun : (pair == Pair::BS23 ? bs : dp);
    const int ns = pair == Pair::HeunEuler ? 2 : (pair == Pair::BS23 ? 4 : 7);
    MM_TRY(hipcheck(c, hipMemsetAsync(emax, 0, sizeof(unsigned), c->stream), "clear error maximum"));
    const float *eval = base;
    for (int i = 0; i < ns; ++i) {
        float *Hd = nullptr;
        MM_TRY(demag(c, eval, comp, &Hd));
        const St &t = tab[i];
        p.stage_a = (float)t.a;
        p.stage_b = (float)t.b;
        p.stage_e = (float)t.e;
        p.stage_first = i == 0;
        p.stage_last = t.last;
        p.stage_err = t.err;
        p.stage_kstore = t.kstore;
        p.stage_nprev = t.nprev;
        for (int jj = 0; jj < 6; ++jj) p.stage_ap[jj] = jj < 4 ? (float)t.ap[jj] : 0.f;
        float *o = t.last == 1 ? out : (t.last == 2 ? nullptr : stage[i & 1]);
        MM_TRY(timed(c, MM_K_LOCAL, "embedded stage", [&] {
            return mmk::launch_stage(c->g, p, eval, Hd, ms_map_ptr(c), h_map_ptr(c), base, acc, eacc, kbuf, (float)h,
                                     renorm, o, flag, c->stream);
        }));
        if (o) eval = o;
    }
    MM_TRY(hipcheck(c, mmk::launch_errmax(eacc, c->g.N, emax, c->stream), "error maximum"));
    unsigned bits = 0;
    MM_TRY(hipcheck(c, hipMemcpyAsync(&bits, emax, sizeof(bits), hipMemcpyDeviceToHost, c->stream), "read error"));
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "step sync"));
    float e;
    std::memcpy(&e, &bits, sizeof(e));
    *err = e;
    return MM_OK;
}

// nsteps Euler steps of m in place, through the context's state buffer
mm_status enqueue_steps(mm_ctx *c, float *m, int64_t nsteps, double dt, uint32_t flags)
{
    float *buf[2] = {m, c->at<float>(c->o_mtmp)};
    MM_TRY(run_steps(
        c, nsteps, dt, flags, [&](int64_t s) { return buf[s & 1]; }, [&](int64_t s) { return buf[(s + 1) & 1]; },
        [](int64_t) { return (float *)nullptr; }));
    if (nsteps & 1)
        MM_TRY(hipcheck(c, hipMemcpyAsync(m, buf[1], sizeof(float) * 3 * c->g.N, hipMemcpyDeviceToDevice, c->stream),
                        "copy back state"));
    return MM_OK;
}

// captured chunk of n (even) steps for this state pointer, dt and flags
mm_status graph_for(mm_ctx *c, float *m, int64_t n, double dt, uint32_t flags, hipGraphExec_t *out)
{
    for (auto &e : c->graphs)
        if (e.m == m && e.n == n && e.dt == dt && e.flags == flags && e.stream == c->stream && e.tslot == c->tslot) {
            *out = e.exec;
            return MM_OK;
        }
    const bool was_timing = c->timing;
    const int tslot0 = c->tslot;
    c->timing = false;
    MM_TRY(hipcheck(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture"));
    mm_status st = enqueue_steps(c, m, n, dt, flags);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(c->stream, &graph);
    c->timing = was_timing;
    if (st != MM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    MM_TRY(hipcheck(c, e_end, "end capture"));
    hipGraphExec_t exec = nullptr;
    const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    MM_TRY(hipcheck(c, e_inst, "instantiate graph"));
    c->tslot = tslot0;  // n is even: a replay leaves the clock slot where it found it
    c->graphs.push_back({m, n, dt, flags, c->stream, tslot0, exec});
    *out = exec;
    return MM_OK;
}

constexpr int64_t kGraphChunk = 32;  // steps per captured graph

}  // namespace

extern "C" {

mm_status mm_step_llg(mm_ctx *c, float *m, int64_t nsteps, double dt, uint32_t flags)
{
    if (!c) return MM_EINVAL;
    const uint32_t step_flags = flags & ~uint32_t(MM_F_GRAPH);
    MM_TRY(check_step_args(c, m, nsteps, dt, step_flags));
    if (c->sched && (step_flags & (MM_F_HEUN | MM_F_RK4)))
        return fail(c, MM_EUNSUP, "a time-dependent field is applied by Euler steps only");
    MM_TRY(set_device(c));
    if (!(flags & MM_F_GRAPH)) return enqueue_steps(c, m, nsteps, dt, step_flags);
    if (!c->stream) return fail(c, MM_EINVAL, "MM_F_GRAPH needs a non-null stream (capture is not allowed on it)");
    int64_t chunk = nsteps >= kGraphChunk ? kGraphChunk : (nsteps & ~int64_t(1));
    int64_t done = 0;
    if (chunk >= 2) {
        hipGraphExec_t exec = nullptr;
        MM_TRY(graph_for(c, m, chunk, dt, step_flags, &exec));
        for (; done + chunk <= nsteps; done += chunk)
            MM_TRY(hipcheck(c, hipGraphLaunch(exec, c->stream), "graph launch"));
    }
    return enqueue_steps(c, m, nsteps - done, dt, step_flags);
}

mm_status mm_step_adaptive(mm_ctx *c, float *m, double t_end, double *dt_io, double tol, uint32_t flags,
                           int64_t max_steps, int64_t *accepted, int64_t *rejected)
{
    if (!c) return MM_EINVAL;
    if (!dt_io || !(*dt_io > 0) || !std::isfinite(*dt_io)) return fail(c, MM_EINVAL, "*dt must be finite and > 0");
    if (!(t_end >= 0) || !std::isfinite(t_end)) return fail(c, MM_EINVAL, "t_end must be finite and >= 0");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(c, MM_EINVAL, "tol must be finite and > 0");
    if (max_steps < 1) return fail(c, MM_EINVAL, "max_steps must be >= 1");
    const int heun = (flags & MM_F_HEUN) ? 1 : 0, bs23 = (flags & MM_F_BS23) ? 1 : 0,
              dp54 = (flags & MM_F_DP54) ? 1 : 0;
    if (heun + bs23 + dp54 != 1)
        return fail(c, MM_EINVAL, "exactly one of MM_F_HEUN, MM_F_BS23 and MM_F_DP54 selects the pair");
    if (flags & ~uint32_t(MM_F_NO_RENORM | MM_F_COMPENSATED | MM_F_HEUN | MM_F_BS23 | MM_F_DP54))
        return fail(c, MM_EINVAL, "unsupported flag bits 0x%x for adaptive steps", flags);
    MM_TRY(check_step_args(c, m, 0, *dt_io, flags & uint32_t(MM_F_NO_RENORM | MM_F_COMPENSATED)));
    if (c->sched) return fail(c, MM_EUNSUP, "a time-dependent field is applied by Euler steps only");
    MM_TRY(set_device(c));
    const Pair pair = heun ? Pair::HeunEuler : (bs23 ? Pair::BS23 : Pair::DP54);
    const int q = heun ? 1 : (bs23 ? 2 : 4);  // order of the lower member
    float *buf[2] = {m, c->at<float>(c->o_mtmp)};
    int cur = 0;
    double t = 0.0, dt = *dt_io;
    int64_t acc = 0, rej = 0;
    mm_status st = MM_OK;
    while (t < t_end) {
        if (acc + rej >= max_steps) {
            st = fail(c, MM_ESTATE, "max_steps (%lld) attempts did not reach t_end", (long long)max_steps);
            break;
        }
        const double h = (t + dt > t_end) ? t_end - t : dt;
        float err = 0.f;
        st = embedded_step(c, buf[cur], buf[cur ^ 1], h, pair, flags, &err);
        if (st != MM_OK) break;
        if (!(err == err)) {
            st = fail(c, MM_ENONFINITE, "non-finite error estimate at t = %g s", t);
            break;
        }
        if ((double)err <= tol) {
            cur ^= 1;
            t += h;
            ++acc;
        } else {
            ++rej;
        }
        double f = err > 0.f ? 0.9 * std::pow(tol / (double)err, 1.0 / (q + 1)) : 5.0;
        f = std::min(5.0, std::max(0.2, f));
        dt = h * f;
    }
    if (cur == 1)
        MM_TRY(hipcheck(c, hipMemcpyAsync(m, buf[1], sizeof(float) * 3 * c->g.N, hipMemcpyDeviceToDevice, c->stream),
                        "copy back state"));
    *dt_io = dt;
    if (accepted) *accepted = acc;
    if (rejected) *rejected = rej;
    return st;
}

mm_status mm_set_tuning(mm_ctx *c, const int32_t choice[3])
{
    if (!c || !choice) return MM_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (choice[k] < 0 || choice[k] >= MM_TUNE_VARIANTS)
            return fail(c, MM_EINVAL, "tuning choice %d out of range [0, %d)", choice[k], MM_TUNE_VARIANTS);
    for (int k = 0; k < 3; ++k) c->tune[k] = choice[k];
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_get_tuning(const mm_ctx *c, int32_t choice[3])
{
    if (!c || !choice) return MM_EINVAL;
    for (int k = 0; k < 3; ++k) choice[k] = c->tune[k];
    return MM_OK;
}

mm_status mm_autotune(mm_ctx *c, const char *cache_path, int32_t choice_out[3])
{
    if (!c) return MM_EINVAL;
    MM_TRY(need_ws(c));
    MM_TRY(set_device(c));
    hipDeviceProp_t prop;
    MM_TRY(hipcheck(c, hipGetDeviceProperties(&prop, c->device), "device properties"));
    std::string arch(prop.gcnArchName);
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    const mmk::Geo &g = c->g;
    int best[3] = {0, 0, 0};
    bool found = false;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char a[256];
            int nx, ny, nz, v0, v1, v2;
            while (std::fscanf(f, "%255s %d %d %d %d %d %d", a, &nx, &ny, &nz, &v0, &v1, &v2) == 7) {
                if (arch == a && nx == g.nx && ny == g.ny && nz == g.nz && v0 >= 0 && v0 < MM_TUNE_VARIANTS &&
                    v1 >= 0 && v1 < MM_TUNE_VARIANTS && v2 >= 0 && v2 < MM_TUNE_VARIANTS) {
                    best[0] = v0; best[1] = v1; best[2] = v2;
                    found = true;  // the last matching line wins
                }
            }
            std::fclose(f);
        }
    }
    if (!found) {
        // time each variant of each pass on zeroed buffers (the values do
        // not matter for the time; zeros keep every intermediate finite)
        float2 *S1 = c->at<float2>(c->o_S1), *S2 = c->at<float2>(c->o_S2);
        float *mz = c->at<float>(c->o_mtmp), *H = c->at<float>(c->o_S2);
        const float *K = c->at<float>(c->o_K);
        hipStream_t st = c->stream;
        const size_t s1b = sizeof(float2) * 3 * (size_t)g.nz * g.Hx * g.ny;
        const size_t s2b = sizeof(float2) * 3 * (size_t)g.nz * g.Hx * g.Py;
        MM_TRY(hipcheck(c, hipMemsetAsync(mz, 0, sizeof(float) * 3 * (size_t)g.N, st), "clear state"));
        MM_TRY(hipcheck(c, hipMemsetAsync(S1, 0, s1b, st), "clear S1"));
        MM_TRY(hipcheck(c, hipMemsetAsync(S2, 0, s2b, st), "clear S2"));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        MM_TRY(hipcheck(c, hipEventCreate(&e0), "event"));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(c, MM_EHIP, "event");
        }
        mm_status status = MM_OK;
        auto time_it = [&](auto &&launch, float *ms_out) -> hipError_t {
            for (int r = 0; r < 2; ++r)
                if (hipError_t e = launch(); e != hipSuccess) return e;
            hipError_t e = hipEventRecord(e0, st);
            for (int r = 0; r < 10 && e == hipSuccess; ++r) e = launch();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(ms_out, e0, e1);
            return e;
        };
        const float msv = (float)c->mat.Ms;
        for (int pass = 0; pass < 3 && status == MM_OK; ++pass) {
            float best_t = 0.f;
            for (int v = 0; v < MM_TUNE_VARIANTS && status == MM_OK; ++v) {
                float t = 0.f;
                hipError_t e;
                if (pass == 0)
                    e = time_it([&] {
                        hipError_t a = mmk::launch_xfwd(g, mz, nullptr, msv, S1, st, v);
                        return a == hipSuccess ? mmk::launch_xinv(g, S1, H, st, v) : a;
                    }, &t);
                else if (pass == 1)
                    e = time_it([&] {
                        hipError_t a = mmk::launch_yfwd(g, S1, S2, st, v);
                        return a == hipSuccess ? mmk::launch_yinv(g, S2, S1, st, v) : a;
                    }, &t);
                else
                    e = time_it([&] { return mmk::launch_zconv(g, S2, K, false, st, v); }, &t);
                if (e != hipSuccess) {
                    status = hipcheck(c, e, "autotune timing");
                    break;
                }
                if (v == 0 || t < best_t) {
                    best_t = t;
                    best[pass] = v;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (status != MM_OK) return status;
        if (cache_path) {
            if (FILE *f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%s %d %d %d %d %d %d\n", arch.c_str(), g.nx, g.ny, g.nz, best[0], best[1], best[2]);
                std::fclose(f);
            } else {
                return fail(c, MM_EINVAL, "cannot append to the tuning cache %s", cache_path);
            }
        }
    }
    for (int k = 0; k < 3; ++k) c->tune[k] = best[k];
    c->drop_graphs();
    if (choice_out)
        for (int k = 0; k < 3; ++k) choice_out[k] = best[k];
    return MM_OK;
}

mm_status mm_set_fusion(mm_ctx *c, int on)
{
    if (!c) return MM_EINVAL;
    if (on < 0 || on > 2) return fail(c, MM_EINVAL, "fusion level %d outside [0, 2]", on);
    c->fusion = on;
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_set_compensated(mm_ctx *c, int on)
{
    if (!c) return MM_EINVAL;
    c->compensated = on != 0;
    c->drop_graphs();
    return MM_OK;
}

mm_status mm_forward_store(mm_ctx *c, float *m, int64_t nsteps, double dt, uint32_t flags, float *m_traj,
                           float *hd_traj)
{
    if (!c) return MM_EINVAL;
    MM_TRY(check_step_args(c, m, nsteps, dt, flags));
    if (flags & (MM_F_HEUN | MM_F_RK4))
        return fail(c, MM_EUNSUP, "the stored replay and the adjoint cover the Euler step only");
    if (c->sched) return fail(c, MM_EUNSUP, "the stored replay and the adjoint cover constant fields only");
    if (c->ms_map && c->vacuum) return fail(c, MM_EUNSUP, "the adjoint covers samples without vacuum cells");
    if (nsteps > 0 && (!m_traj || !hd_traj || !aligned16(m_traj) || !aligned16(hd_traj)))
        return fail(c, MM_EINVAL, "trajectory buffers must be 16-byte aligned device pointers");
    MM_TRY(set_device(c));
    const size_t S = 3 * (size_t)c->g.N;
    if (nsteps > 0)
        MM_TRY(hipcheck(c, hipMemcpyAsync(m_traj, m, sizeof(float) * S, hipMemcpyDeviceToDevice, c->stream),
                        "store state"));
    MM_TRY(run_steps(
        c, nsteps, dt, flags, [&](int64_t s) { return m_traj + (size_t)s * S; },
        [&](int64_t s) { return (s + 1 < nsteps) ? m_traj + (size_t)(s + 1) * S : m; },
        [&](int64_t s) { return hd_traj + (size_t)s * S; }));
    return MM_OK;
}

mm_status mm_adjoint_step(mm_ctx *c, const float *m_n, const float *hd_n, float *lam, float *g_hext, float *g_ms,
                          double dt, uint32_t flags)
{
    if (!c) return MM_EINVAL;
    MM_TRY(check_step_args(c, m_n, 1, dt, flags));
    if (flags & (MM_F_HEUN | MM_F_RK4)) return fail(c, MM_EUNSUP, "the adjoint covers the Euler step only");
    if (c->sched) return fail(c, MM_EUNSUP, "the adjoint covers constant fields only");
    if (c->ms_map && c->vacuum) return fail(c, MM_EUNSUP, "the adjoint covers samples without vacuum cells");
    if (!hd_n || !lam || !aligned16(hd_n) || !aligned16(lam))
        return fail(c, MM_EINVAL, "hd_n and lam must be 16-byte aligned device pointers");
    if ((g_hext && !aligned16(g_hext)) || (g_ms && !aligned16(g_ms)))
        return fail(c, MM_EINVAL, "gradient buffers must be 16-byte aligned");
    MM_TRY(set_device(c));
    const size_t S = 3 * (size_t)c->g.N;
    const mmk::LocalParams p = local_params(c);
    const bool comp = flags & MM_F_COMPENSATED;
    const int renorm = (flags & MM_F_NO_RENORM) ? 0 : 1;
    float *gH = c->at<float>(c->o_adj), *lam_loc = gH + S;
    MM_TRY(timed(c, MM_K_LOCAL, "adjoint local", [&] {
        return mmk::launch_adj_a(c->g, p, m_n, hd_n, ms_map_ptr(c), h_map_ptr(c), lam, (float)dt, renorm, gH, lam_loc,
                                 g_hext, g_ms, c->stream);
    }));
    float *D = nullptr;
    MM_TRY(demag(c, gH, comp, &D, nullptr, true));
    return timed(c, MM_K_LOCAL, "adjoint completion", [&] {
        return mmk::launch_adj_b(c->g, p, m_n, gH, D, ms_map_ptr(c), lam_loc, lam, g_ms, c->stream);
    });
}

mm_status mm_adjoint_segment(mm_ctx *c, const float *m_traj, const float *hd_traj, int64_t n, float *lam,
                             float *g_hext, float *g_ms, double dt, uint32_t flags)
{
    if (!c) return MM_EINVAL;
    if (n < 1) return fail(c, MM_EINVAL, "a segment has n >= 1 steps");
    if (!m_traj || !hd_traj) return fail(c, MM_EINVAL, "m_traj and hd_traj must be device pointers");
    const size_t S = 3 * (size_t)c->g.N;
    for (int64_t s = n - 1; s >= 0; --s)
        MM_TRY(mm_adjoint_step(c, m_traj + (size_t)s * S, hd_traj + (size_t)s * S, lam, g_hext, g_ms, dt, flags));
    return MM_OK;
}

mm_status mm_reduce(mm_ctx *c, const float *m, double *out)
{
    if (!c) return MM_EINVAL;
    if (!m || !out || !aligned16(m) || !aligned16(out)) return fail(c, MM_EINVAL, "m and out must be 16-byte aligned device pointers");
    MM_TRY(need_ws(c));
    if (!c->have_mat) return fail(c, MM_ESTATE, "material not set");
    if (!c->tensor) return fail(c, MM_ESTATE, "mm_build_tensor has not been called");
    MM_TRY(set_device(c));
    float *Hd = nullptr;
    MM_TRY(demag(c, m, false, &Hd));
    mmk::EnergyParams e{};
    e.A = c->mat.A;
    e.Ku = c->mat.Ku;
    e.u0 = c->mat.u[0];
    e.u1 = c->mat.u[1];
    e.u2 = c->mat.u[2];
    e.ms = c->mat.Ms;
    e.h0 = c->hext[0];
    e.h1 = c->hext[1];
    e.h2 = c->hext[2];
    e.cx = 1.0 / (c->d[0] * c->d[0]);
    e.cy = 1.0 / (c->d[1] * c->d[1]);
    e.cz = 1.0 / (c->d[2] * c->d[2]);
    e.V = c->d[0] * c->d[1] * c->d[2];
    e.mu0 = kMu0;
    e.terms = MM_T_ALL;
    e.sched = c->sched ? 1 : 0;
    e.tslot = c->tslot;
    e.clk = clock_ptr(c);
    e.t_start = c->sched_t[0];
    e.t_decay = c->sched_t[1];
    e.t_stop = c->sched_t[2];
    return hipcheck(c, mmk::launch_energy(c->g, e, m, Hd, ms_map_ptr(c), h_map_ptr(c), c->at<double>(c->o_part), out,
                                          c->stream),
                    "energy");
}

mm_status mm_reduce_loss(mm_ctx *c, const float *m, const float *target, double *out, float *grad)
{
    if (!c) return MM_EINVAL;
    if (!m || !target || !out || !aligned16(m) || !aligned16(target) || !aligned16(out))
        return fail(c, MM_EINVAL, "m, target and out must be 16-byte aligned device pointers");
    if (grad && !aligned16(grad)) return fail(c, MM_EINVAL, "grad must be 16-byte aligned");
    if (grad && (grad == m || grad == target)) return fail(c, MM_EINVAL, "grad may not alias m or target");
    MM_TRY(need_ws(c));
    MM_TRY(set_device(c));
    return hipcheck(c, mmk::launch_loss(m, target, 3 * c->g.N, grad, c->at<double>(c->o_lpart), out, c->stream),
                    "loss");
}

mm_status mm_reduce_loss_noalloc(mm_ctx *c, const float *m, const float *target, double *out, float *grad)
{
    if (!c) return MM_EINVAL;
    if (!m || !target || !out || !aligned16(m) || !aligned16(target) || !aligned16(out))
        return fail(c, MM_EINVAL, "m, target and out must be 16-byte aligned device pointers");
    if (grad && !aligned16(grad)) return fail(c, MM_EINVAL, "grad must be 16-byte aligned");
    if (grad && (grad == m || grad == target)) return fail(c, MM_EINVAL, "grad may not alias m or target");
    const long long n = 3 * c->g.N;
    if (mmk::loss_partials(n) > mmk::kScratchPartials)
        return fail(c, MM_EINVAL, "%lld cells exceed the static scratch of the no-allocation loss (at most %lld cells)",
                    (long long)c->g.N, mmk::kScratchPartials * mmk::kLossChunk / 3);
    double *sc = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_init_mu);
        sc = g_scratch[c->device];
    }
    if (!sc) return fail(c, MM_ESTATE, "device %d has no static scratch address", c->device);
    MM_TRY(set_device(c));
    return hipcheck(c, mmk::launch_loss(m, target, n, grad, sc, out, c->stream), "loss (static scratch)");
}

mm_status mm_kernel_timing(mm_ctx *c, int enable)
{
    if (!c) return MM_EINVAL;
    MM_TRY(set_device(c));
    MM_TRY(drain_timing(c));
    c->timing = enable != 0;
    if (c->timing)
        for (int k = 0; k < MM_K_COUNT; ++k) {
            c->t_ms[k] = 0.0;
            c->t_n[k] = 0;
        }
    return MM_OK;
}

mm_status mm_kernel_times(mm_ctx *c, double *ms, int64_t *launches)
{
    if (!c) return MM_EINVAL;
    if (!ms || !launches) return fail(c, MM_EINVAL, "output pointers are NULL");
    MM_TRY(set_device(c));
    MM_TRY(drain_timing(c));
    for (int k = 0; k < MM_K_COUNT; ++k) {
        ms[k] = c->t_ms[k];
        launches[k] = c->t_n[k];
    }
    return MM_OK;
}

mm_status mm_sync(mm_ctx *c)
{
    if (!c) return MM_EINVAL;
    MM_TRY(set_device(c));
    MM_TRY(hipcheck(c, hipStreamSynchronize(c->stream), "stream sync"));
    if (c->ws) {
        int flag = 0;
        MM_TRY(hipcheck(c, hipMemcpy(&flag, c->at<int>(c->o_flag), sizeof(int), hipMemcpyDeviceToHost), "read flag"));
        if (flag) {
            MM_TRY(hipcheck(c, hipMemset(c->at<int>(c->o_flag), 0, sizeof(int)), "clear flag"));
            return fail(c, MM_ENONFINITE, "a step produced a non-finite magnetisation");
        }
    }
    return MM_OK;
}

const char *mm_last_error(const mm_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

}  // extern "C"

// ===========================================================================
// Batched samples: many independent grids (each its own nx, ny, nz and
// external field, one cell size and material) advanced together.  The tensor
// spectrum depends only on the padded size and the cell size, so samples of
// one padded size share one spectrum, built as for an (Px/2, Py/2, Pz/2)
// grid: a sample with n <= P/2 never reaches the offsets beyond its own
// extent in the zero-padded convolution.
//
// Launch plan: each pass depends only on its own transform length, so the
// samples are grouped per pass by that length alone (x by Px, y by Py, z by
// Pz; the local kernel by whether nx is a multiple of 4, its vector width),
// and each group runs as one launch.  The per-sample descriptors live in the
// workspace, so a launch carries one pointer; its grid is (blocks, samples),
// as wide as the group's largest sample, rounded up to a multiple of 8 so
// that every sample keeps the XCD placement of a single-sample launch.
// (A one-dimensional grid holding exactly the samples' blocks, found through
// a block-to-sample map in device memory, was measured slower on the
// 64-film batch, 187 against 180 us per step: the map read puts a second
// dependent memory access before each block's first load, which costs more
// than the blocks beyond a smaller sample's grid, which exit after one.)
// ===========================================================================

struct mm_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    double d[3] = {0, 0, 0};
    mm_material mat{};
    bool have_mat = false, tensor = false;
    struct Sample {
        mmk::Geo g;
        size_t m_off = 0;                  // offset in the packed state (floats)
        size_t o_S1 = 0, o_S2 = 0, o_mt = 0;  // workspace byte offsets
        int group = 0;
        double h[3] = {0, 0, 0};
    };
    struct Group {
        mmk::Geo g;          // padded sizes of the group (n = P/2)
        size_t o_K = 0;      // its tensor spectrum
        std::vector<int> members;
    };
    // one launch of a pass: samples with one transform length
    struct Launch {
        int pass = 0;                   // 0 x, 1 y, 2 z, 3 local, 4 fused x-inverse + update
        int len = 0;                    // Px, Py, Pz; local: 1 if nx % 4 == 0; fused: 2 Px + (nx % 4 == 0)
        int var = 0;                    // launch-shape variant
        std::vector<int> members;
        long long width = 0;            // blocks per sample in the grid (current variant)
        size_t o_desc[3] = {0, 0, 0};   // descriptor arrays (see plan_image)
    };
    std::vector<Sample> samples;
    std::vector<Group> groups;
    std::vector<Launch> launches;       // x, then y, then z, then local, then fused
    bool fusion = false;      // Euler steps run the fused x-inverse + update launches (off: slower for thin films)
    bool all_fusable = false; // every sample has a fused form
    size_t total_state = 0;  // floats in the packed state
    size_t o_flag = 0, o_plan = 0, plan_bytes = 0, total = 0;
    char *ws = nullptr;
    const float *plan_m = nullptr;  // state pointer the uploaded descriptors were written for
    bool plan_ok = false;
    std::string err;
    std::vector<hipGraphExec_t> graph_exec;
    std::vector<std::pair<const float *, std::pair<int64_t, double>>> graph_key;
    std::vector<uint32_t> graph_flags;
    void drop_graphs()
    {
        for (auto e : graph_exec) (void)hipGraphExecDestroy(e);
        graph_exec.clear();
        graph_key.clear();
        graph_flags.clear();
    }
    ~mm_batch() { drop_graphs(); }
    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

mm_status bfail(mm_batch *b, mm_status s, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return s;
}

mm_status bhip(mm_batch *b, hipError_t e, const char *what)
{
    if (e != hipSuccess) return bfail(b, MM_EHIP, "%s: %s", what, hipGetErrorString(e));
    return MM_OK;
}

mmk::Geo make_geo(int nx, int ny, int nz, int Px, int Py, int Pz)
{
    mmk::Geo g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.Px = Px;
    g.Py = Py;
    g.Pz = Pz;
    g.Hx = Px / 2 + 1;
    g.Hy = Py == 1 ? 1 : Py / 2 + 1;
    g.Hz = Pz == 1 ? 1 : Pz / 2 + 1;
    g.N = (long long)nx * ny * nz;
    return g;
}

mmk::LocalParams batch_params(const mm_batch *b)
{
    mmk::LocalParams p{};
    const mm_material &m = b->mat;
    p.ms = (float)m.Ms;
    p.ax = (float)(2.0 * m.A / (kMu0 * b->d[0] * b->d[0]));
    p.ay = (float)(2.0 * m.A / (kMu0 * b->d[1] * b->d[1]));
    p.az = (float)(2.0 * m.A / (kMu0 * b->d[2] * b->d[2]));
    p.ku2 = (float)(2.0 * m.Ku / kMu0);
    p.u0 = (float)m.u[0];
    p.u1 = (float)m.u[1];
    p.u2 = (float)m.u[2];
    const double c1 = -m.gamma0 / (1.0 + m.alpha * m.alpha);
    p.c1 = (float)c1;
    p.c2 = (float)(m.alpha * c1);
    p.stage_kstore = -1;
    p.stage_nprev = 0;
    return p;
}

const float *spectrum_of(const mm_batch *b, int i) { return b->at<float>(b->groups[b->samples[i].group].o_K); }

// blocks of sample i's own grid in launch L with variant v, and the padded
// count that launch gives it.  A z launch with the compensated multiply runs
// variant 0 whatever its tuned variant, so its map covers the larger of the
// two grids (the kernel's bounds check retires the blocks its own grid does
// not have).
long long sample_blocks(const mm_batch *b, const mm_batch::Launch &L, int i, int v)
{
    const mmk::Geo &g = b->samples[i].g;
    if (L.pass == 4) return mmk::xe_blocks(g);
    if (L.pass == 3) return mmk::local_blocks(g, L.len != 0);
    if (L.pass == 2) return std::max(mmk::pass_blocks(2, g, v), mmk::pass_blocks(2, g, 0));
    return mmk::pass_blocks(L.pass, g, v);
}
long long launch_width(const mm_batch *b, const mm_batch::Launch &L, int v)
{
    long long n = 0;
    for (int i : L.members) n = std::max(n, sample_blocks(b, L, i, v));
    return (n + 7) & ~7LL;
}

// group the samples into launches (at creation: depends on the sizes only)
void plan_launches(mm_batch *b)
{
    b->launches.clear();
    const int ns = (int)b->samples.size();
    b->all_fusable = true;
    for (const auto &sm : b->samples) b->all_fusable = b->all_fusable && mmk::fused_xinv_euler_ok(sm.g);
    for (int pass = 0; pass < 5; ++pass) {
        if (pass == 4 && !b->all_fusable) break;
        std::vector<std::pair<int, int>> keyed;
        for (int i = 0; i < ns; ++i) {
            const mmk::Geo &g = b->samples[i].g;
            const int vec = g.nx % 4 == 0 ? 1 : 0;
            const int key = pass == 0 ? g.Px : pass == 1 ? g.Py : pass == 2 ? g.Pz : pass == 3 ? vec : 2 * g.Px + vec;
            keyed.push_back({key, i});
        }
        std::stable_sort(keyed.begin(), keyed.end(), [](const auto &u, const auto &v) { return u.first < v.first; });
        for (size_t k = 0; k < keyed.size();) {
            mm_batch::Launch L;
            L.pass = pass;
            L.len = keyed[k].first;
            while (k < keyed.size() && keyed[k].first == L.len) L.members.push_back(keyed[k++].second);
            b->launches.push_back(L);
        }
    }
    for (auto &L : b->launches) L.width = launch_width(b, L, 0);
}

// workspace bytes of the plan region, and the offsets of every array in it
size_t plan_layout(mm_batch *b, size_t base)
{
    Carve cv;
    cv.off = base;
    for (auto &L : b->launches) {
        const size_t n = L.members.size();
        switch (L.pass) {
        case 0:  // xfwd for even steps (reads m), for odd steps (reads the temporary), xinv
            L.o_desc[0] = cv.take(sizeof(mmk::XfwdDesc) * n);
            L.o_desc[1] = cv.take(sizeof(mmk::XfwdDesc) * n);
            L.o_desc[2] = cv.take(sizeof(mmk::XinvDesc) * n);
            break;
        case 1:  // forward S1 -> S2, inverse S2 -> S1
            L.o_desc[0] = cv.take(sizeof(mmk::YDesc) * n);
            L.o_desc[1] = cv.take(sizeof(mmk::YDesc) * n);
            break;
        case 2:
            L.o_desc[0] = cv.take(sizeof(mmk::ZDesc) * n);
            break;
        case 4:  // fused x-inverse + update, even and odd steps
            L.o_desc[0] = cv.take(sizeof(mmk::XeDesc) * n);
            L.o_desc[1] = cv.take(sizeof(mmk::XeDesc) * n);
            break;
        default:  // local, even and odd steps
            L.o_desc[0] = cv.take(sizeof(mmk::LocalDesc) * n);
            L.o_desc[1] = cv.take(sizeof(mmk::LocalDesc) * n);
        }
    }
    return cv.off - base;
}

// Host image of the plan region for state pointer m: every launch's
// descriptors.  Even steps read m and write the sample's temporary, odd
// steps the reverse.
std::vector<char> plan_image(const mm_batch *b, const float *m)
{
    std::vector<char> img(b->plan_bytes, 0);
    auto put = [&](size_t off, const void *src, size_t bytes) { std::memcpy(img.data() + (off - b->o_plan), src, bytes); };
    for (const auto &L : b->launches) {
        for (int par = 0; par < 2; ++par) {
            for (int k = 0; k < (int)L.members.size(); ++k) {
                const auto &sm = b->samples[L.members[k]];
                const float *src = par ? b->at<float>(sm.o_mt) : m + sm.m_off;
                float *dst = par ? const_cast<float *>(m) + sm.m_off : b->at<float>(sm.o_mt);
                if (L.pass == 0) {
                    const mmk::XfwdDesc xf{sm.g, src, nullptr, b->at<float2>(sm.o_S1), (float)b->mat.Ms};
                    put(L.o_desc[par] + sizeof(xf) * k, &xf, sizeof(xf));
                    if (par == 0) {
                        const mmk::XinvDesc xi{sm.g, b->at<float2>(sm.o_S1), b->at<float>(sm.o_S2)};
                        put(L.o_desc[2] + sizeof(xi) * k, &xi, sizeof(xi));
                    }
                } else if (L.pass == 1) {
                    const mmk::YDesc yd = par ? mmk::YDesc{sm.g, b->at<float2>(sm.o_S2), b->at<float2>(sm.o_S1)}
                                              : mmk::YDesc{sm.g, b->at<float2>(sm.o_S1), b->at<float2>(sm.o_S2)};
                    put(L.o_desc[par] + sizeof(yd) * k, &yd, sizeof(yd));
                } else if (L.pass == 2) {
                    if (par == 0) {
                        const mmk::ZDesc zd{sm.g, b->at<float2>(sm.o_S2), spectrum_of(b, L.members[k])};
                        put(L.o_desc[0] + sizeof(zd) * k, &zd, sizeof(zd));
                    }
                } else if (L.pass == 4) {
                    const mmk::XeDesc xe{sm.g,    b->at<float2>(sm.o_S1), src, nullptr, nullptr, dst, nullptr,
                                         nullptr, (float)sm.h[0], (float)sm.h[1], (float)sm.h[2], 0};
                    put(L.o_desc[par] + sizeof(xe) * k, &xe, sizeof(xe));
                } else {
                    mmk::LocalDesc ld{sm.g, src, b->at<float>(sm.o_S2), nullptr, nullptr, dst, nullptr,
                                      (float)sm.h[0], (float)sm.h[1], (float)sm.h[2]};
                    ld.perm_q = mmk::local_perm(sm.g, L.len != 0);
                    put(L.o_desc[par] + sizeof(ld) * k, &ld, sizeof(ld));
                }
            }
        }
    }
    return img;
}

// write the plan for state pointer m into the workspace (waits for the
// stream first: earlier launches may still read the old plan)
mm_status plan_upload(mm_batch *b, const float *m)
{
    if (b->plan_ok && b->plan_m == m) return MM_OK;
    const std::vector<char> img = plan_image(b, m);
    MM_TRY(bhip(b, hipStreamSynchronize(b->stream), "plan sync"));
    MM_TRY(bhip(b, hipMemcpy(b->at<char>(b->o_plan), img.data(), img.size(), hipMemcpyHostToDevice), "plan upload"));
    b->drop_graphs();
    b->plan_m = m;
    b->plan_ok = true;
    return MM_OK;
}

template <typename D>
mmk::Table<D> table_of(const mm_batch *b, const mm_batch::Launch &L, int which)
{
    return mmk::Table<D>{b->at<D>(L.o_desc[which]), L.width, (int)L.members.size()};
}

// enqueue nsteps steps of every sample (plan uploaded for m, no checks)
mm_status batch_enqueue(mm_batch *b, int64_t nsteps, double dt, uint32_t flags)
{
    const mmk::LocalParams p = batch_params(b);
    const bool comp = flags & MM_F_COMPENSATED;
    const int renorm = (flags & MM_F_NO_RENORM) ? 0 : 1;
    int *flag = b->at<int>(b->o_flag);
    hipStream_t st = b->stream;
    const bool fuse = b->fusion && b->all_fusable;
    for (int64_t s = 0; s < nsteps; ++s) {
        const int par = (int)(s & 1);
        for (const auto &L : b->launches)
            if (L.pass == 0)
                MM_TRY(bhip(b, mmk::launch_xfwd_table(table_of<mmk::XfwdDesc>(b, L, par), L.len, st, L.var), "batch xfwd"));
        for (const auto &L : b->launches)
            if (L.pass == 1)
                MM_TRY(bhip(b, mmk::launch_yfwd_table(table_of<mmk::YDesc>(b, L, 0), L.len, st, L.var), "batch yfwd"));
        for (const auto &L : b->launches)
            if (L.pass == 2)
                MM_TRY(bhip(b, mmk::launch_zconv_table(table_of<mmk::ZDesc>(b, L, 0), L.len, comp, st, L.var),
                            "batch zconv"));
        for (const auto &L : b->launches)
            if (L.pass == 1)
                MM_TRY(bhip(b, mmk::launch_yinv_table(table_of<mmk::YDesc>(b, L, 1), L.len, st, L.var), "batch yinv"));
        if (fuse) {
            for (const auto &L : b->launches)
                if (L.pass == 4)
                    MM_TRY(bhip(b, mmk::launch_xinv_euler_table(table_of<mmk::XeDesc>(b, L, par), L.len / 2,
                                                                (L.len & 1) != 0, p, (float)dt, renorm, flag, st),
                                "batch x-inverse + update"));
            continue;
        }
        for (const auto &L : b->launches)
            if (L.pass == 0)
                MM_TRY(bhip(b, mmk::launch_xinv_table(table_of<mmk::XinvDesc>(b, L, 2), L.len, st, L.var), "batch xinv"));
        for (const auto &L : b->launches)
            if (L.pass == 3)
                MM_TRY(bhip(b, mmk::launch_local_table(table_of<mmk::LocalDesc>(b, L, par), L.len != 0, false, p,
                                                       MM_T_ALL, 1, (float)dt, renorm, flag, st),
                            "batch local"));
    }
    return MM_OK;
}

mm_status batch_copy_back(mm_batch *b, float *m)
{
    for (const auto &sm : b->samples)
        MM_TRY(bhip(b, hipMemcpyAsync(m + sm.m_off, b->at<float>(sm.o_mt), sizeof(float) * 3 * sm.g.N,
                                      hipMemcpyDeviceToDevice, b->stream),
                    "copy back state"));
    return MM_OK;
}

// FNV-1a over the sample sizes: the key of a batch's tuning in the cache file
uint64_t batch_key(const mm_batch *b)
{
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ULL;
        }
    };
    mix(b->samples.size());
    for (const auto &sm : b->samples) {
        mix((uint64_t)sm.g.nx);
        mix((uint64_t)sm.g.ny);
        mix((uint64_t)sm.g.nz);
    }
    return h;
}

int tunable_launches(const mm_batch *b)
{
    int n = 0;
    for (const auto &L : b->launches) n += L.pass < 3;  // x, y and z
    return n;
}

}  // namespace

extern "C" {

mm_status mm_batch_create(mm_batch **out, int count, const int32_t *n, double dx, double dy, double dz, int device,
                          void *hip_stream)
{
    if (!out || !n || count < 1 || count > 65536) return MM_EINVAL;
    *out = nullptr;
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !std::isfinite(dx) || !std::isfinite(dy) || !std::isfinite(dz))
        return MM_EINVAL;
    for (int i = 0; i < count; ++i) {
        const int nx = n[3 * i], ny = n[3 * i + 1], nz = n[3 * i + 2];
        if (nx < 2 || nx > kMaxN || ny < 1 || ny > kMaxN || nz < 1 || nz > kMaxN) return MM_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MM_EINVAL;
    mm_batch *b = new (std::nothrow) mm_batch();
    if (!b) return MM_ENOMEM;
    b->device = device;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->d[0] = dx;
    b->d[1] = dy;
    b->d[2] = dz;
    b->samples.resize(count);
    size_t moff = 0;
    for (int i = 0; i < count; ++i) {
        auto &sm = b->samples[i];
        const int nx = n[3 * i], ny = n[3 * i + 1], nz = n[3 * i + 2];
        sm.g = make_geo(nx, ny, nz, padded(nx), padded(ny), padded(nz));
        sm.m_off = moff;
        moff += (3 * (size_t)sm.g.N + 3) & ~size_t(3);  // 16-byte aligned sample slots
        int gi = -1;
        for (size_t k = 0; k < b->groups.size(); ++k)
            if (b->groups[k].g.Px == sm.g.Px && b->groups[k].g.Py == sm.g.Py && b->groups[k].g.Pz == sm.g.Pz)
                gi = (int)k;
        if (gi < 0) {
            mm_batch::Group gr;
            gr.g = make_geo(sm.g.Px / 2, sm.g.Py > 1 ? sm.g.Py / 2 : 1, sm.g.Pz > 1 ? sm.g.Pz / 2 : 1, sm.g.Px,
                            sm.g.Py, sm.g.Pz);
            b->groups.push_back(gr);
            gi = (int)b->groups.size() - 1;
        }
        sm.group = gi;
        b->groups[gi].members.push_back(i);
    }
    b->total_state = moff;
    plan_launches(b);
    // workspace: spectra, flag, launch plan, then per-sample buffers aliased
    // with the tensor-build temporaries of the largest group
    Carve cv;
    for (auto &gr : b->groups) gr.o_K = cv.take(sizeof(float) * 6 * (size_t)gr.g.Hx * gr.g.Hy * gr.g.Hz);
    b->o_flag = cv.take(256);
    b->o_plan = cv.off;
    b->plan_bytes = plan_layout(b, b->o_plan);
    cv.off = b->o_plan;
    cv.take(b->plan_bytes);
    const size_t region = cv.off;
    Carve st;
    st.off = region;
    for (auto &sm : b->samples) {
        sm.o_S1 = st.take(sizeof(float2) * 3 * (size_t)sm.g.nz * sm.g.Hx * sm.g.ny);
        sm.o_S2 = st.take(sizeof(float2) * 3 * (size_t)sm.g.nz * sm.g.Hx * sm.g.Py);
        sm.o_mt = st.take(sizeof(float) * 3 * (size_t)sm.g.N);
    }
    size_t tmax = 0;
    for (auto &gr : b->groups) {
        const mmk::Geo &g = gr.g;
        Carve tb;
        tb.take(sizeof(double) * 6 * (size_t)g.N);
        const size_t a1 = (size_t)g.nz * g.ny * g.Hx, a2 = (size_t)g.Hz * g.Hy * g.Hx;
        tb.take(sizeof(double) * (a1 > a2 ? a1 : a2));
        tb.take(sizeof(double) * (size_t)g.nz * g.Hy * g.Hx);
        tmax = tb.off > tmax ? tb.off : tmax;
    }
    b->total = std::max(st.off, region + tmax);
    if (hipSetDevice(device) != hipSuccess) {
        delete b;
        return MM_EHIP;
    }
    {
        mm_ctx tmp;
        tmp.device = device;
        tmp.stream = b->stream;
        if (init_device(&tmp) != MM_OK) {
            delete b;
            return MM_EHIP;
        }
    }
    *out = b;
    return MM_OK;
}

mm_status mm_batch_destroy(mm_batch *b)
{
    if (!b) return MM_EINVAL;
    delete b;
    return MM_OK;
}

mm_status mm_batch_set_stream(mm_batch *b, void *hip_stream)
{
    if (!b) return MM_EINVAL;
    b->stream = static_cast<hipStream_t>(hip_stream);
    return MM_OK;
}

mm_status mm_batch_workspace_size(const mm_batch *b, size_t *bytes)
{
    if (!b || !bytes) return MM_EINVAL;
    *bytes = b->total;
    return MM_OK;
}

mm_status mm_batch_state_offsets(const mm_batch *b, int64_t *offsets)
{
    if (!b || !offsets) return MM_EINVAL;
    for (size_t i = 0; i < b->samples.size(); ++i) offsets[i] = (int64_t)b->samples[i].m_off;
    offsets[b->samples.size()] = (int64_t)b->total_state;
    return MM_OK;
}

mm_status mm_batch_set_workspace(mm_batch *b, void *dev_ptr, size_t bytes)
{
    if (!b) return MM_EINVAL;
    if (!dev_ptr) return bfail(b, MM_EINVAL, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) return bfail(b, MM_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < b->total)
        return bfail(b, MM_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", bytes, b->total);
    b->ws = static_cast<char *>(dev_ptr);
    b->tensor = false;
    b->plan_ok = false;
    b->drop_graphs();
    MM_TRY(bhip(b, hipSetDevice(b->device), "hipSetDevice"));
    return bhip(b, hipMemsetAsync(b->at<int>(b->o_flag), 0, sizeof(int), b->stream), "clear flag");
}

mm_status mm_batch_set_material(mm_batch *b, const mm_material *m)
{
    if (!b) return MM_EINVAL;
    mm_ctx tmp;
    const mm_status s = mm_set_material(&tmp, m);
    if (s != MM_OK) return bfail(b, s, "%s", tmp.err.c_str());
    b->mat = tmp.mat;
    b->have_mat = true;
    b->plan_ok = false;  // Ms is in the x-forward descriptors
    b->drop_graphs();
    return MM_OK;
}

mm_status mm_batch_set_hext(mm_batch *b, const double *h)
{
    if (!b) return MM_EINVAL;
    if (!h) return bfail(b, MM_EINVAL, "fields are NULL");
    for (size_t i = 0; i < 3 * b->samples.size(); ++i)
        if (!std::isfinite(h[i])) return bfail(b, MM_EINVAL, "fields must be finite");
    for (size_t i = 0; i < b->samples.size(); ++i)
        for (int k = 0; k < 3; ++k) b->samples[i].h[k] = h[3 * i + k];
    b->plan_ok = false;  // the fields are in the local descriptors
    b->drop_graphs();
    return MM_OK;
}

mm_status mm_batch_build_tensor(mm_batch *b)
{
    if (!b) return MM_EINVAL;
    if (!b->ws) return bfail(b, MM_ESTATE, "no workspace set");
    MM_TRY(bhip(b, hipSetDevice(b->device), "hipSetDevice"));
    const size_t region = b->o_plan + b->plan_bytes;
    for (auto &gr : b->groups) {
        const mmk::Geo &g = gr.g;
        Carve tb;
        tb.off = region;
        double *T = b->at<double>(tb.take(sizeof(double) * 6 * (size_t)g.N));
        const size_t a1 = (size_t)g.nz * g.ny * g.Hx, a2 = (size_t)g.Hz * g.Hy * g.Hx;
        double *tA = b->at<double>(tb.take(sizeof(double) * (a1 > a2 ? a1 : a2)));
        double *tB = b->at<double>(tb.take(sizeof(double) * (size_t)g.nz * g.Hy * g.Hx));
        MM_TRY(bhip(b, mmk::launch_tensor_octant(g, b->d[0], b->d[1], b->d[2], T, b->stream), "tensor octant"));
        MM_TRY(bhip(b, mmk::launch_tensor_spectrum(g, T, tA, tB, b->at<float>(gr.o_K), b->stream), "tensor spectrum"));
    }
    MM_TRY(bhip(b, hipStreamSynchronize(b->stream), "tensor build sync"));
    b->tensor = true;
    return MM_OK;
}

mm_status mm_batch_step(mm_batch *b, float *m, int64_t nsteps, double dt, uint32_t flags)
{
    if (!b) return MM_EINVAL;
    if (!m || !aligned16(m)) return bfail(b, MM_EINVAL, "m must be a 16-byte aligned device pointer");
    if (nsteps < 0) return bfail(b, MM_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0) || !std::isfinite(dt)) return bfail(b, MM_EINVAL, "dt must be finite and > 0");
    if (flags & (MM_F_HEUN | MM_F_RK4)) return bfail(b, MM_EUNSUP, "batched steps are Euler steps only");
    if (flags & ~uint32_t(MM_F_NO_RENORM | MM_F_COMPENSATED | MM_F_GRAPH))
        return bfail(b, MM_EINVAL, "unknown flag bits 0x%x", flags);
    if (!b->ws) return bfail(b, MM_ESTATE, "no workspace set");
    if (!b->have_mat) return bfail(b, MM_ESTATE, "material not set");
    if (!b->tensor) return bfail(b, MM_ESTATE, "mm_batch_build_tensor has not been called");
    MM_TRY(bhip(b, hipSetDevice(b->device), "hipSetDevice"));
    MM_TRY(plan_upload(b, m));
    const uint32_t sf = flags & ~uint32_t(MM_F_GRAPH);
    if (!(flags & MM_F_GRAPH)) {
        MM_TRY(batch_enqueue(b, nsteps, dt, sf));
        return (nsteps & 1) ? batch_copy_back(b, m) : MM_OK;
    }
    if (!b->stream) return bfail(b, MM_EINVAL, "MM_F_GRAPH needs a non-null stream");
    const int64_t chunk = nsteps >= kGraphChunk ? kGraphChunk : (nsteps & ~int64_t(1));
    int64_t done = 0;
    if (chunk >= 2) {
        hipGraphExec_t exec = nullptr;
        for (size_t k = 0; k < b->graph_exec.size(); ++k)
            if (b->graph_key[k].first == m && b->graph_key[k].second.first == chunk &&
                b->graph_key[k].second.second == dt && b->graph_flags[k] == sf)
                exec = b->graph_exec[k];
        if (!exec) {
            MM_TRY(bhip(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture"));
            const mm_status s = batch_enqueue(b, chunk, dt, sf);
            hipGraph_t graph = nullptr;
            const hipError_t e_end = hipStreamEndCapture(b->stream, &graph);
            if (s != MM_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return s;
            }
            MM_TRY(bhip(b, e_end, "end capture"));
            const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            MM_TRY(bhip(b, e_inst, "instantiate graph"));
            b->graph_exec.push_back(exec);
            b->graph_key.push_back({m, {chunk, dt}});
            b->graph_flags.push_back(sf);
        }
        for (; done + chunk <= nsteps; done += chunk) MM_TRY(bhip(b, hipGraphLaunch(exec, b->stream), "graph launch"));
    }
    MM_TRY(batch_enqueue(b, nsteps - done, dt, sf));
    return ((nsteps - done) & 1) ? batch_copy_back(b, m) : MM_OK;
}

mm_status mm_batch_set_fusion(mm_batch *b, int on)
{
    if (!b) return MM_EINVAL;
    b->fusion = on != 0;
    b->drop_graphs();
    return MM_OK;
}

mm_status mm_batch_set_tuning(mm_batch *b, const int32_t *choices, int32_t n)
{
    if (!b) return MM_EINVAL;
    if (!choices || n != tunable_launches(b))
        return bfail(b, MM_EINVAL, "expected %d choices (x, y and z launches)", tunable_launches(b));
    for (int k = 0; k < n; ++k)
        if (choices[k] < 0 || choices[k] >= MM_TUNE_VARIANTS)
            return bfail(b, MM_EINVAL, "tuning choice %d out of range [0, %d)", choices[k], MM_TUNE_VARIANTS);
    int k = 0;
    for (auto &L : b->launches) {
        if (L.pass >= 3) continue;
        const int L1 = L.pass == 0 ? L.len / 2 : L.len;
        L.var = mmk::pass_variant(L.pass, L1, choices[k++]);
        L.width = launch_width(b, L, L.var);
    }
    b->drop_graphs();
    return MM_OK;
}

mm_status mm_batch_get_tuning(const mm_batch *b, int32_t *choices, int32_t capacity, int32_t *n)
{
    if (!b || !n) return MM_EINVAL;
    *n = tunable_launches(b);
    if (choices && capacity < *n) return MM_EINVAL;
    if (choices) {
        int k = 0;
        for (const auto &L : b->launches)
            if (L.pass < 3) choices[k++] = L.var;
    }
    return MM_OK;
}

mm_status mm_batch_autotune(mm_batch *b, const char *cache_path, int32_t *choices, int32_t capacity, int32_t *n)
{
    if (!b) return MM_EINVAL;
    if (!b->ws) return bfail(b, MM_ESTATE, "no workspace set");
    if (!b->have_mat) return bfail(b, MM_ESTATE, "material not set");
    if (!b->tensor) return bfail(b, MM_ESTATE, "mm_batch_build_tensor has not been called");
    const int nl = tunable_launches(b);
    if (n) *n = nl;
    if (choices && capacity < nl) return bfail(b, MM_EINVAL, "choices holds %d entries, %d needed", capacity, nl);
    MM_TRY(bhip(b, hipSetDevice(b->device), "hipSetDevice"));
    hipDeviceProp_t prop;
    MM_TRY(bhip(b, hipGetDeviceProperties(&prop, b->device), "device properties"));
    std::string arch(prop.gcnArchName);
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    char key[32];
    std::snprintf(key, sizeof key, "batch-%016llx", (unsigned long long)batch_key(b));
    std::vector<int32_t> best(nl, 0);
    bool found = false;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char a[256], k2[64];
            int cnt = 0;
            while (std::fscanf(f, "%255s %63s %d", a, k2, &cnt) == 3) {
                std::vector<int32_t> v(cnt > 0 ? cnt : 0);
                bool ok = cnt == nl;
                for (int q = 0; q < cnt; ++q)
                    if (std::fscanf(f, "%d", &v[q]) != 1 || v[q] < 0 || v[q] >= MM_TUNE_VARIANTS) ok = false;
                if (ok && arch == a && std::string(k2) == key) {
                    best = v;
                    found = true;  // the last matching line wins
                }
            }
            std::fclose(f);
        }
    }
    if (!found) {
        // time each variant of each launch on zeroed sample buffers: x
        // launches as x-forward + x-inverse, y launches as forward + inverse,
        // z launches alone
        MM_TRY(bhip(b, hipStreamSynchronize(b->stream), "tune sync"));
        for (const auto &sm : b->samples) {
            MM_TRY(bhip(b, hipMemsetAsync(b->at<float>(sm.o_mt), 0, sizeof(float) * 3 * sm.g.N, b->stream), "clear"));
            MM_TRY(bhip(b, hipMemsetAsync(b->at<float2>(sm.o_S1), 0, sizeof(float2) * 3 * sm.g.nz * sm.g.Hx * sm.g.ny,
                                          b->stream), "clear"));
            MM_TRY(bhip(b, hipMemsetAsync(b->at<float2>(sm.o_S2), 0, sizeof(float2) * 3 * sm.g.nz * sm.g.Hx * sm.g.Py,
                                          b->stream), "clear"));
        }
        // the odd-step x-forward descriptors read the zeroed temporaries; the
        // even-step set (for a state pointer that is not given here) is not
        // launched, so any pointer serves as its base
        float *mt0 = b->at<float>(b->samples[0].o_mt);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        MM_TRY(bhip(b, hipEventCreate(&e0), "event"));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return bfail(b, MM_EHIP, "event");
        }
        mm_status status = MM_OK;
        int k = 0;
        for (auto &L : b->launches) {
            if (L.pass >= 3 || status != MM_OK) continue;
            const int L1 = L.pass == 0 ? L.len / 2 : L.len;
            float best_t = 0.f;
            for (int v = 0; v < MM_TUNE_VARIANTS && status == MM_OK; ++v) {
                if (mmk::pass_variant(L.pass, L1, v) != v) continue;
                L.var = v;
                L.width = launch_width(b, L, v);
                // the x-forward reads the temporaries through the odd-step set
                status = plan_upload(b, mt0);
                if (status != MM_OK) break;
                auto launch = [&]() -> hipError_t {
                    hipError_t e;
                    if (L.pass == 0) {
                        e = mmk::launch_xfwd_table(table_of<mmk::XfwdDesc>(b, L, 1), L.len, b->stream, v);
                        if (e == hipSuccess) e = mmk::launch_xinv_table(table_of<mmk::XinvDesc>(b, L, 2), L.len, b->stream, v);
                    } else if (L.pass == 1) {
                        e = mmk::launch_yfwd_table(table_of<mmk::YDesc>(b, L, 0), L.len, b->stream, v);
                        if (e == hipSuccess) e = mmk::launch_yinv_table(table_of<mmk::YDesc>(b, L, 1), L.len, b->stream, v);
                    } else {
                        e = mmk::launch_zconv_table(table_of<mmk::ZDesc>(b, L, 0), L.len, false, b->stream, v);
                    }
                    return e;
                };
                float t = 0.f;
                hipError_t e = hipSuccess;
                for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch();
                if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
                for (int r = 0; r < 10 && e == hipSuccess; ++r) e = launch();
                if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
                if (e != hipSuccess) {
                    status = bhip(b, e, "batch autotune timing");
                    break;
                }
                if (v == 0 || t < best_t) {
                    best_t = t;
                    best[k] = v;
                }
            }
            ++k;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->plan_ok = false;  // the descriptors were written for the temporaries
        if (status != MM_OK) return status;
        if (cache_path) {
            if (FILE *f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%s %s %d", arch.c_str(), key, nl);
                for (int q = 0; q < nl; ++q) std::fprintf(f, " %d", best[q]);
                std::fprintf(f, "\n");
                std::fclose(f);
            } else {
                return bfail(b, MM_EINVAL, "cannot append to the tuning cache %s", cache_path);
            }
        }
    }
    MM_TRY(mm_batch_set_tuning(b, best.data(), nl));
    if (choices)
        for (int q = 0; q < nl; ++q) choices[q] = best[q];
    return MM_OK;
}

mm_status mm_batch_sync(mm_batch *b)
{
    if (!b) return MM_EINVAL;
    MM_TRY(bhip(b, hipSetDevice(b->device), "hipSetDevice"));
    MM_TRY(bhip(b, hipStreamSynchronize(b->stream), "stream sync"));
    if (b->ws) {
        int flag = 0;
        MM_TRY(bhip(b, hipMemcpy(&flag, b->at<int>(b->o_flag), sizeof(int), hipMemcpyDeviceToHost), "read flag"));
        if (flag) {
            MM_TRY(bhip(b, hipMemset(b->at<int>(b->o_flag), 0, sizeof(int)), "clear flag"));
            return bfail(b, MM_ENONFINITE, "a step produced a non-finite magnetisation");
        }
    }
    return MM_OK;
}

const char *mm_batch_last_error(const mm_batch *b)
{
    if (!b) return "null batch";
    return b->err.c_str();
}

}  // extern "C"
