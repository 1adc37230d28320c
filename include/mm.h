/*
 * mm.h -- C ABI of the MI355X (gfx950) micromagnetic step library.
 *
 * The library evaluates the effective field of Zhu, "Grace: a Cross-platform
 * Micromagnetic Simulator On Graphics Processing Units" (arXiv:1411.2565),
 * Sec. 2 eq. (2):
 *     H_eff = H_exch + H_anis + H_demag + H_extern,
 * with the demagnetising field computed as the zero-padded FFT convolution of
 * the magnetisation with the cell-averaged demag tensor (Sec. 3), the exchange
 * field with the six-neighbour scheme (Sec. 3), and advances the magnetisation
 * with the explicit-Euler integration of the LLG equation, eq. (3) (Sec. 3).
 *
 * Conventions shared by every call:
 *   - Units are SI: lengths m, fields and Ms A/m, A J/m, Ku J/m^3, dt s,
 *     gamma0 = gamma*mu0 in m/(A s).  mu0 = 4 pi 1e-7 exactly.
 *   - The state is the unit magnetisation m, FP32, structure of arrays
 *     [3][nz][ny][nx] with x fastest, in device memory.  Per-cell scalar maps
 *     are [nz][ny][nx].
 *   - Every device pointer is owned by the caller, must be 16-byte aligned
 *     and must stay valid until the work enqueued on the context's stream has
 *     finished.  The library keeps no pointer to caller arrays after a call
 *     returns, except the workspace given to mm_set_workspace.
 *   - The library allocates no device memory.  All scratch lives in one
 *     caller-provided workspace (mm_workspace_size / mm_set_workspace).
 *   - Calls enqueue on the context's HIP stream and return without waiting,
 *     except mm_create, mm_build_tensor and mm_sync, which synchronise.
 *     Argument checks are synchronous and happen on the host before any
 *     work is enqueued; a rejected call enqueues nothing.
 *   - Errors are negative mm_status codes; mm_last_error returns a message
 *     for the most recent failure on that context.  No C++ exception
 *     crosses this interface.  A context is not thread-safe.
 *   - Supported sizes: 2 <= nx <= 512, 1 <= ny <= 512, 1 <= nz <= 512.
 *     Each axis with n > 1 is zero-padded to the smallest power of two
 *     P >= 2n - 1 (an axis with n = 1 is not padded); any such P gives the
 *     same linear convolution.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MM_OK = 0,
    MM_EINVAL = -1,      /* invalid argument (size, pointer, value) */
    MM_ESTATE = -2,      /* call out of order (no workspace, material or tensor) */
    MM_ENOMEM = -3,      /* workspace too small */
    MM_EHIP = -4,        /* a HIP runtime call failed */
    MM_EUNSUP = -5,      /* supported by the method but not by this library */
    MM_ENONFINITE = -6   /* a step produced a non-finite magnetisation */
} mm_status;

typedef struct mm_ctx mm_ctx;

/* Grid of nx*ny*nz rectangular cells of size dx*dy*dz (Sec. 2, and the
 * "-rectang" record of the paper's input file, Sec. 5). */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
} mm_geometry;

/* Material of Sec. 2: Ms (uniform; see mm_set_ms_map for a map), exchange
 * stiffness A, uniaxial anisotropy constant Ku along the unit axis u (the
 * paper's anisotropy field H_K corresponds to Ku = mu0 Ms H_K / 2), damping
 * alpha and gamma0 = gamma*mu0 of eq. (3). */
typedef struct {
    double Ms, A, Ku, u[3], alpha, gamma0;
} mm_material;

/* Field terms of eq. (2). */
enum { MM_T_EXCH = 1, MM_T_DEMAG = 2, MM_T_ANIS = 4, MM_T_ZEEMAN = 8, MM_T_ALL = 15 };

/* Step flags. */
enum {
    MM_F_NO_RENORM = 1,    /* skip m <- m/|m| after each Euler step */
    MM_F_COMPENSATED = 2,  /* compensated (Dot2) FP32 spectral tensor multiply */
    MM_F_GRAPH = 4,        /* mm_step_llg: replay captured chunks of 32 steps (needs a non-null stream) */
    MM_F_HEUN = 8,         /* mm_step_llg: Heun step (explicit trapezoid, order 2) instead of Euler */
    MM_F_RK4 = 16,         /* mm_step_llg: classic fourth-order Runge-Kutta step instead of Euler */
    MM_F_BS23 = 32,        /* mm_step_adaptive: Bogacki-Shampine 3(2) pair (MM_F_HEUN: Heun/Euler 2(1)) */
    MM_F_DP54 = 64         /* mm_step_adaptive: Dormand-Prince 5(4) pair */
};

/* Create a context for a geometry on HIP device `device`; work is enqueued
 * on `hip_stream` (a hipStream_t, NULL = the device's null stream).  Checks
 * the sizes, fixes the padded FFT sizes and prepares the device-side
 * constant tables (synchronous).  *out receives the context. */
mm_status mm_create(mm_ctx **out, const mm_geometry *g, int device, void *hip_stream);

/* Destroy a context (does not free the caller's workspace). */
mm_status mm_destroy(mm_ctx *c);

/* Change the stream subsequent calls enqueue on. */
mm_status mm_set_stream(mm_ctx *c, void *hip_stream);

/* Bytes of device workspace the context needs (for the tensor spectrum,
 * FFT intermediates, the second state buffer, maps and reduction partials). */
mm_status mm_workspace_size(const mm_ctx *c, size_t *bytes);

/* Hand the context a caller-owned device buffer of at least
 * mm_workspace_size bytes, 256-byte aligned.  The tensor spectrum and the
 * copied maps live in it, so replacing the workspace requires calling
 * mm_build_tensor (and the map setters) again. */
mm_status mm_set_workspace(mm_ctx *c, void *dev_ptr, size_t bytes);

/* Set the material (Sec. 2; eq. (3) for alpha and gamma0).  Requires
 * Ms > 0, A >= 0, Ku >= 0, |u| > 0 (normalised here), alpha >= 0,
 * gamma0 > 0. */
mm_status mm_set_material(mm_ctx *c, const mm_material *mat);

/* Per-cell saturation magnetisation map (N floats, device, A/m), copied into
 * the workspace; NULL returns to the uniform Ms.  Cells with Ms = 0 are
 * vacuum, which makes the geometry non-regular (named as future work in
 * Sec. 6): they are no demag source, exchange omits them as neighbours (a
 * free surface, as at the sample boundary), exchange and anisotropy fields
 * are zero there (mm_compute_heff returns the demag and applied fields),
 * their state is never changed, and mm_reduce skips them (energies, and the
 * mean magnetisation is over magnetic cells).  The state in vacuum cells
 * must still be finite.  Values must be finite and >= 0, checked here
 * (MM_EINVAL otherwise, the uniform Ms stays); the check synchronises the
 * stream.  With vacuum cells, mm_forward_store and mm_adjoint_step return
 * MM_EUNSUP. */
mm_status mm_set_ms_map(mm_ctx *c, const float *ms_dev);

/* Uniform external field (Sec. 2, H_extern), A/m. */
mm_status mm_set_hext(mm_ctx *c, const double h[3]);

/* Per-cell external field map (Sec. 2, H_extern of eq. (2) given cell by
 * cell; 3N floats [3][nz][ny][nx], device, A/m), copied into the workspace
 * on the stream; NULL returns to the uniform field. */
mm_status mm_set_hext_map(mm_ctx *c, const float *h_dev);

/* Time-dependent external field.  The paper's input file (Sec. 5) gives the
 * external field with a startTime, a decayTime and a stopTime; the profile
 * between them is not stated and is read here as
 *     s(t) = 0                              t <  t_start
 *            1                              t_start <= t <= t_decay
 *            (t_stop - t)/(t_stop - t_decay) t_decay < t < t_stop
 *            0                              t >= t_stop
 * and multiplies the whole external field (uniform or map).  sched =
 * {t_start, t_decay, t_stop} in seconds, finite, t_start <= t_decay <=
 * t_stop (MM_EINVAL otherwise); NULL returns to the constant field.  The
 * time lives on the device (mm_set_time): each Euler step of mm_step_llg
 * evaluates the field at the current time t_n and advances it by dt in FP64
 * (t_{n+1} = t_n + dt), also inside captured graphs, so replays continue the
 * clock.  mm_compute_heff and mm_reduce use the field at the current time.
 * While a schedule is set, Runge-Kutta steps (MM_F_HEUN, MM_F_RK4),
 * mm_step_adaptive, mm_forward_store and mm_adjoint_step return MM_EUNSUP. */
mm_status mm_set_field_schedule(mm_ctx *c, const double sched[3]);

/* Set the device clock of the time-dependent field to t (s), enqueued on the
 * stream; mm_set_workspace sets it to 0. */
mm_status mm_set_time(mm_ctx *c, double t);

/* Read the device clock (the time of the next step) into *t; synchronises
 * the stream. */
mm_status mm_get_time(mm_ctx *c, double *t);

/* Build the demag tensor spectrum for the geometry (Sec. 3: the convolution
 * kernel of the zero-padded FFT evaluation).  The cell-averaged tensor is
 * evaluated in FP64 on the GPU (Newell's closed form near the source, a
 * tent-weighted Gauss-Legendre quadrature of the dipole kernel far from it),
 * transformed in FP64 and stored as FP32.  Needs the workspace; overwrites
 * the FFT intermediates.  Synchronous. */
mm_status mm_build_tensor(mm_ctx *c);

/* Diagnostic: write the FP64 real-space tensor for the non-negative octant
 * of cell offsets, [6][nz][ny][nx] in the order xx, yy, zz, xy, xz, yz,
 * into tab_dev (6N doubles, device).  Synchronous. */
mm_status mm_tensor_table(mm_ctx *c, double *tab_dev);

/* Diagnostic of the spectral multiply's arithmetic (each component of
 * H(k) = K(k) M(k), Sec. 3, is a dot product of three terms): for the n
 * triples (k0, x0, k1, x1, k2, x2) at in_dev[6 i] (6n floats, device),
 * writes out_dev[2 i] = k0 x0 + k1 x1 + k2 x2 as the plain multiply
 * computes it and out_dev[2 i + 1] as the compensated one (MM_F_COMPENSATED,
 * Dot2 of Ogita, Rump and Oishi) does, with the same device functions as
 * the z passes (2n floats, device).  0 <= n <= 2^31 (MM_EINVAL otherwise);
 * n = 0 does nothing.  Needs no workspace; synchronous. */
mm_status mm_diag_dot3(mm_ctx *c, const float *in_dev, float *out_dev, int64_t n);

/* Effective field of eq. (2) restricted to the terms in `terms`
 * (MM_T_* mask) for the state m_dev, written to h_dev (3N floats, A/m,
 * may not alias m_dev).  MM_T_DEMAG requires mm_build_tensor. */
mm_status mm_compute_heff(mm_ctx *c, const float *m_dev, float *h_dev, uint32_t terms);

/* Advance m_dev in place by nsteps explicit-Euler steps of eq. (3) with all
 * four field terms:
 *     m <- m + dt * (-gamma0/(1+alpha^2)) [m x H + alpha m x (m x H)],
 * followed by m <- m/|m| unless MM_F_NO_RENORM.  dt > 0, nsteps >= 0.
 * With MM_F_GRAPH the steps are enqueued as replays of a HIP graph holding a
 * chunk of 32 steps (or the largest even count below nsteps), captured on
 * the first such call for this (m_dev, dt, flags, stream) and kept until a
 * setter changes what the kernels read; results are identical to the eager
 * path.  The capture requires a non-null stream.
 * MM_F_HEUN or MM_F_RK4 (not both) replaces each Euler step by an explicit
 * Runge-Kutta step of the same right-hand side f (fixed-step counterparts
 * of the adaptive steps below, Sec. 6): stages k_i = f(m_i) with
 * m_1 = m and m_{i+1} = P(m + dt a_i k_i), result P(m + dt sum_i b_i k_i),
 * P the renormalisation (identity under MM_F_NO_RENORM).  Heun: a = (1),
 * b = (1/2, 1/2), two field evaluations per step; classic RK4:
 * a = (1/2, 1/2, 1), b = (1/6, 1/3, 1/3, 1/6), four.  Not accepted by
 * mm_forward_store, mm_adjoint_step or the batch calls (MM_EUNSUP): the
 * adjoint is that of the Euler step. */
mm_status mm_step_llg(mm_ctx *c, float *m_dev, int64_t nsteps, double dt, uint32_t flags);

/* FP64 reductions of the energy of eq. (1) summed over cells and of the
 * mean magnetisation, written to out_dev (8 doubles, device):
 *     E_exch, E_demag, E_anis, E_zeeman, E_total, <mx>, <my>, <mz>  (J, -).
 * Terms follow the paper's energy density with the cell volume V:
 *     E_exch  = A V sum over neighbour pairs |m_j - m_i|^2 / d^2
 *     E_demag = -(mu0 V / 2) sum Ms m . H_demag
 *     E_anis  = Ku V sum (1 - (m . u)^2)
 *     E_zeeman = -mu0 V sum Ms m . h_ext */
mm_status mm_reduce(mm_ctx *c, const float *m_dev, double *out_dev);

/* FP64 loss of a state against a target, the L2 mismatch
 *     L = 1/2 sum over all 3N components (m - t)^2
 * that the gradient of an Euler rollout (mm_adjoint_step) is taken for,
 * written to out_dev (1 double, device).  When grad_dev is not NULL it
 * receives dL/dm = m - t (3N floats, FP32; may not alias m or t).  Each
 * block of the reduction adds a fixed run of 2048 consecutive values and the
 * block sums are added in a fixed order, so the result is deterministic.
 * Needs the workspace (its partial sums); the material and tensor are not
 * used. */
mm_status mm_reduce_loss(mm_ctx *c, const float *m_dev, const float *target_dev, double *out_dev,
                         float *grad_dev);

/* The same loss for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * identical arguments and results as mm_reduce_loss, bit for bit (the same
 * kernels), but the partial sums live in a static array of the library
 * (4096 FP64 values, 32 KiB, held on every GPU the library runs on until the
 * process ends) instead of the workspace.  Needs no workspace; allocates
 * nothing and calls no allocating routine.  Contexts of more than
 * 2 796 202 cells (N with 3N > 4096 * 2048) return MM_EINVAL.  Every call on
 * one GPU shares that array: calls that may overlap on one GPU (several
 * streams or threads) race and must be serialised by the caller. */
mm_status mm_reduce_loss_noalloc(mm_ctx *c, const float *m_dev, const float *target_dev, double *out_dev,
                                 float *grad_dev);

/* Fusion level of the Euler steps of mm_step_llg and mm_forward_store.
 * on = 0: the x-inverse transform and the local terms + update run as two
 * passes (H_demag through device memory).  on = 1 (the default): as one
 * pass, so H_demag never goes to device memory (mm_forward_store has that
 * pass also store it for its trajectory).  on = 2: with a uniform Ms, that
 * pass also runs the next step's x-forward transform of the state it
 * writes, for every step of a call but the last, so the next step skips its
 * own x-forward (m is not read twice; on the 256x256x32 block it took as
 * long as level 1: 44.9 us against 27.1 + 16.4 us for the two passes it
 * replaces).  The fused pass applies to samples with a padded x length Px
 * with 8 <= Px <= 512 (nx >= 3), with or without an Ms map; other samples
 * always take two passes.  All levels give the same result bit for bit
 * (the same transform and update arithmetic).  MM_EINVAL for a level
 * outside [0, 2].  Sec. 3: the demag field, the local terms and the Euler
 * step of eq. (3) per step. */
mm_status mm_set_fusion(mm_ctx *c, int on);

/* Use (on != 0) or stop using the compensated FP32 spectral multiply in every
 * demag evaluation of this context (mm_compute_heff, mm_reduce, steps and
 * adjoint steps), in addition to per-call MM_F_COMPENSATED. */
mm_status mm_set_compensated(mm_ctx *c, int on);

/* Launch-shape tuning of the FFT passes (the paper leaves FFT performance to
 * its FFT library, Sec. 3).  Each of the x passes, the y
 * passes and the z pass has MM_TUNE_VARIANTS launch shapes: x = lines per
 * block (16, 8, 32), y = lines per thread group (1, 2, 4), z = points per
 * thread and columns per block (default; the other of 4/8 points; half the
 * columns).  A variant applies to single-sample launches whose line has 64
 * points or more.  The x and y variants give results identical bit for bit
 * to the default; the z variants differ in rounding only (another radix
 * split).  The choice is kept by the context (graphs are re-captured). */
#define MM_TUNE_VARIANTS 3
/* Set the choice {x, y, z}, each in [0, MM_TUNE_VARIANTS). */
mm_status mm_set_tuning(mm_ctx *c, const int32_t choice[3]);
mm_status mm_get_tuning(const mm_ctx *c, int32_t choice[3]);
/* Choose the fastest variant of each pass for this geometry and GPU.  If
 * cache_path names a text file holding a line "<gfx arch> nx ny nz x y z"
 * for this device and geometry, that choice is taken without timing;
 * otherwise every variant runs 2 + 10 times on zeroed workspace buffers,
 * timed with HIP events on the context's stream (synchronous), and the
 * winners are appended to the file when cache_path is not NULL (MM_EINVAL
 * if it cannot be written).  Needs the workspace; overwrites the FFT
 * intermediates and the second state buffer, not the tensor, maps or any
 * caller buffer.  choice_out (may be NULL) receives {x, y, z}. */
mm_status mm_autotune(mm_ctx *c, const char *cache_path, int32_t choice_out[3]);

/* Adaptive time steps (named as future work in Sec. 6): advance m_dev in
 * place from t = 0 to t_end (s) with an embedded explicit Runge-Kutta pair
 * of the right-hand side of eq. (3), selected by exactly one of
 *   MM_F_HEUN  Heun with embedded Euler, order 2(1): b = (1/2, 1/2),
 *              bh = (1, 0);
 *   MM_F_BS23  Bogacki-Shampine 3(2): a = (1/2, 3/4), b = (2/9, 1/3, 4/9),
 *              a fourth stage at the new state, bh = (7/24, 1/4, 1/3, 1/8);
 *   MM_F_DP54  Dormand-Prince 5(4), the published seven-stage tableau, the
 *              seventh stage at the new state (q = 4);
 * plus optionally MM_F_NO_RENORM and MM_F_COMPENSATED.  Stage states and the
 * result are renormalised as in mm_step_llg.  Each attempt with step h
 * estimates err = max over cells |h sum_i (b_i - bh_i) k_i| (FP32, reduced
 * on the GPU) and is accepted when err <= tol (tol dimensionless, in units
 * of |m|).  Either way the next step is
 *   h * min(5, max(0.2, 0.9 (tol/err)^(1/(q+1))))   (q = 1, 2 or 4; 5 if err = 0)
 * and a step that would pass t_end is shortened to end there.  *dt_io gives
 * the first step and receives the last proposed one; *accepted / *rejected
 * (may be NULL) count the attempts.  The host waits for the GPU after every
 * attempt (the decision needs the error), so this call is synchronous and is
 * not for graph capture.  Errors: MM_EINVAL for bad arguments or flags;
 * MM_ESTATE after max_steps attempts without reaching t_end, and
 * MM_ENONFINITE for a non-finite estimate; in both cases m_dev holds the last
 * accepted state. */
mm_status mm_step_adaptive(mm_ctx *c, float *m_dev, double t_end, double *dt_io, double tol, uint32_t flags,
                           int64_t max_steps, int64_t *accepted, int64_t *rejected);

/* Forward rollout that keeps what the adjoint needs (the explicit Euler
 * integration of eq. (3), Sec. 3, run as the first half of the gradient
 * computation of mm_adjoint_step): advances m_dev in place
 * by nsteps Euler steps exactly as mm_step_llg does, and stores the state
 * entering step s in m_traj[s] and its demagnetising field in hd_traj[s]
 * (each nsteps * 3N floats, device, [s][3][nz][ny][nx]). */
mm_status mm_forward_store(mm_ctx *c, float *m_dev, int64_t nsteps, double dt, uint32_t flags,
                           float *m_traj, float *hd_traj);

/* Adjoint of one Euler step, the exact transpose of the discrete step
 * (eq. (3) with the field of eq. (2)), for a loss L of the later states.
 * Inputs: the state m_n entering the step and its demagnetising field hd_n
 * (from mm_forward_store), lam = dL/dm_{n+1} (3N floats, device).  Output:
 * lam is overwritten with dL/dm_n.  g_hext (3N floats) and g_ms (N floats),
 * when non-NULL, are accumulated with this step's contribution to dL/dh_ext
 * and dL/dMs (per-cell maps; add up over steps).  The demag transpose is the
 * same FFT convolution, the tensor being symmetric and even. */
mm_status mm_adjoint_step(mm_ctx *c, const float *m_n, const float *hd_n, float *lam, float *g_hext,
                          float *g_ms, double dt, uint32_t flags);

/* The adjoint of a stored segment of n >= 1 Euler steps (the same transpose
 * as mm_adjoint_step, eq. (3) with the field of eq. (2)): m_traj and hd_traj
 * as written by mm_forward_store for those n steps ([s][3][nz][ny][nx]),
 * steps n-1 down to 0.  lam holds dL/dm_n on entry and dL/dm_0 on return;
 * g_hext and g_ms accumulate as in mm_adjoint_step.  The same kernels in the
 * same order as n calls of mm_adjoint_step, so the same results bit for bit,
 * enqueued by one call. */
mm_status mm_adjoint_segment(mm_ctx *c, const float *m_traj, const float *hd_traj, int64_t n, float *lam,
                             float *g_hext, float *g_ms, double dt, uint32_t flags);

/* Kernel identifiers for mm_kernel_times. */
enum {
    MM_K_XFWD = 0,   /* x-forward real FFT (transposed write) */
    MM_K_YFWD = 1,   /* y-forward FFT */
    MM_K_ZCONV = 2,  /* z FFT + tensor multiply + inverse z FFT */
    MM_K_YINV = 3,   /* y-inverse FFT */
    MM_K_XINV = 4,   /* x-inverse real FFT -> H_demag */
    MM_K_LOCAL = 5,  /* local field terms (+ Euler LLG update in mm_step_llg) */
    MM_K_XINV_LOCAL = 6,  /* x-inverse + local terms + Euler update in one pass (mm_step_llg) */
    MM_K_XINV_LOCAL_XFWD = 7,  /* the same, followed by the next step's x-forward (fusion level 2) */
    MM_K_COUNT = 8
};

/* Diagnostic timing: while enabled, every kernel launched by mm_step_llg and
 * mm_compute_heff records a start and a stop HIP event on the context's
 * stream as part of its own dispatch, and its duration is accumulated per
 * kernel identifier.  Enabling clears the totals.  Events serialise nothing
 * that the single stream does not already serialise; the host waits for the
 * stream only when 16384 event pairs are pending (and in mm_kernel_times). */
mm_status mm_kernel_timing(mm_ctx *c, int enable);

/* Synchronise the stream, fold pending event pairs into the totals and
 * return, per MM_K_* identifier, the accumulated milliseconds (ms[MM_K_COUNT])
 * and number of launches (launches[MM_K_COUNT]); host pointers. */
mm_status mm_kernel_times(mm_ctx *c, double *ms, int64_t *launches);

/* ---- Batched samples --------------------------------------------------
 * Many independent grids of rectangular cells (one cell size and material,
 * each its own nx, ny, nz and uniform external field) advanced together by
 * the same step as mm_step_llg (Sec. 3, applied to each sample).  Samples
 * with equal padded sizes share one tensor spectrum.  Each pass runs as one
 * launch per transform length (x by Px, y by Py, z by Pz; the local update
 * by whether nx is a multiple of 4) over all samples of that length; the
 * per-sample descriptors of every launch live in the workspace and are
 * written (synchronously) by the first mm_batch_step for a state pointer
 * and after a setter.
 * The state of all samples is one packed FP32 device array: sample b's
 * [3][nz][ny][nx] block starts at float offset offsets[b]
 * (mm_batch_state_offsets), each block 16-byte aligned. */
typedef struct mm_batch mm_batch;

/* count samples (1..65536), n = count triples (nx, ny, nz) on the host, each
 * within the single-sample limits; cell size dx, dy, dz (m). */
mm_status mm_batch_create(mm_batch **out, int count, const int32_t *n, double dx, double dy, double dz,
                          int device, void *hip_stream);
mm_status mm_batch_destroy(mm_batch *b);
mm_status mm_batch_set_stream(mm_batch *b, void *hip_stream);
/* Float offsets of each sample in the packed state; offsets[count] is the
 * packed length (count + 1 int64 on the host). */
mm_status mm_batch_state_offsets(const mm_batch *b, int64_t *offsets);
mm_status mm_batch_workspace_size(const mm_batch *b, size_t *bytes);
mm_status mm_batch_set_workspace(mm_batch *b, void *dev_ptr, size_t bytes);
/* shared material (same checks as mm_set_material) */
mm_status mm_batch_set_material(mm_batch *b, const mm_material *mat);
/* per-sample uniform external fields: 3*count doubles on the host, A/m */
mm_status mm_batch_set_hext(mm_batch *b, const double *h);
/* one FP64-built spectrum per padded size; synchronous */
mm_status mm_batch_build_tensor(mm_batch *b);
/* nsteps Euler steps of every sample, in place in the packed state; flags
 * as mm_step_llg (MM_F_GRAPH captures chunks of 32 steps of the whole batch) */
mm_status mm_batch_step(mm_batch *b, float *m_packed, int64_t nsteps, double dt, uint32_t flags);
/* As mm_set_fusion, for the batch's Euler steps: with on != 0 and every
 * sample having a fused form (8 <= Px <= 512), each group of samples with
 * one padded x length and one update width (nx % 4 == 0 or not) runs the
 * x-inverse, the local terms and the update as one launch; else (on = 0,
 * the default) the x-inverse and update launches.  Same results bit for
 * bit.  Off by default: batches of thin films give the fused launch too few
 * blocks per sample to overlap its phases (64 films of 1-2 layers: 192 us
 * per step fused against 176 us).  Drops the batch's captured graphs.
 * Sec. 3, applied to every sample. */
mm_status mm_batch_set_fusion(mm_batch *b, int on);
/* Launch-shape tuning of the batch's launches (the paper leaves FFT
 * performance to its FFT library, Sec. 3): one choice in
 * [0, MM_TUNE_VARIANTS) per x, y and z launch, in that order and, within a
 * pass, by increasing transform length; *n receives their number.  The
 * variants are those of mm_set_tuning (x and y regroup lines: results equal
 * the default bit for bit; z changes the radix split: rounding only) and
 * apply to launches whose lines have 64 points or more (others keep 0).
 * mm_batch_autotune times every variant of every launch (2 + 10 runs on
 * zeroed sample buffers, HIP events on the batch's stream, synchronous),
 * keeps the fastest and appends it to cache_path (if not NULL) under the
 * GPU's arch name and a hash of the sample sizes; a matching line already in
 * the file is taken without timing.  choices (capacity entries, may be NULL)
 * receives the result.  Needs the workspace, material and tensor; overwrites
 * the samples' FFT buffers and temporaries, not the caller's state. */
mm_status mm_batch_autotune(mm_batch *b, const char *cache_path, int32_t *choices, int32_t capacity, int32_t *n);
mm_status mm_batch_set_tuning(mm_batch *b, const int32_t *choices, int32_t n);
mm_status mm_batch_get_tuning(const mm_batch *b, int32_t *choices, int32_t capacity, int32_t *n);
mm_status mm_batch_sync(mm_batch *b);
const char *mm_batch_last_error(const mm_batch *b);

/* Wait for the context's stream; report a HIP error or a non-finite state
 * flagged by an earlier step (MM_ENONFINITE, flag cleared on report). */
mm_status mm_sync(mm_ctx *c);

/* Message for the last failure on this context ("" if none).  The pointer
 * stays valid until the next call on the context. */
const char *mm_last_error(const mm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
