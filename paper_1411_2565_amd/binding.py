"""Python binding of the C ABI in ``include/mm.h`` (argument marshalling only).

Each ``mm_*`` function here has the name and meaning of the C entry point it
wraps; device memory is passed as torch CUDA (HIP) tensors, and work is
enqueued on torch's current stream.  Every computation runs in the HIP
kernels of ``libmm.so``; if the library is missing this module raises instead
of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

MM_OK, MM_EINVAL, MM_ESTATE, MM_ENOMEM, MM_EHIP, MM_EUNSUP, MM_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
MM_T_EXCH, MM_T_DEMAG, MM_T_ANIS, MM_T_ZEEMAN, MM_T_ALL = 1, 2, 4, 8, 15
MM_F_NO_RENORM, MM_F_COMPENSATED, MM_F_GRAPH, MM_F_HEUN, MM_F_RK4, MM_F_BS23, MM_F_DP54 = 1, 2, 4, 8, 16, 32, 64

_NAMES = {0: "MM_OK", -1: "MM_EINVAL", -2: "MM_ESTATE", -3: "MM_ENOMEM", -4: "MM_EHIP",
          -5: "MM_EUNSUP", -6: "MM_ENONFINITE"}


class mm_geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class mm_material(ctypes.Structure):
    _fields_ = [("Ms", ctypes.c_double), ("A", ctypes.c_double), ("Ku", ctypes.c_double),
                ("u", ctypes.c_double * 3), ("alpha", ctypes.c_double), ("gamma0", ctypes.c_double)]


class MMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = ctypes.c_void_p


def load():
    """Load libmm.so from the package directory (built by ``build.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
    L = ctypes.CDLL(path)
    st = ctypes.c_int
    sig = {
        "mm_create": [ctypes.POINTER(_P), ctypes.POINTER(mm_geometry), ctypes.c_int, _P],
        "mm_destroy": [_P],
        "mm_set_stream": [_P, _P],
        "mm_workspace_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
        "mm_set_workspace": [_P, _P, ctypes.c_size_t],
        "mm_set_material": [_P, ctypes.POINTER(mm_material)],
        "mm_set_ms_map": [_P, _P],
        "mm_set_hext": [_P, ctypes.POINTER(ctypes.c_double)],
        "mm_set_hext_map": [_P, _P],
        "mm_build_tensor": [_P],
        "mm_tensor_table": [_P, _P],
        "mm_diag_dot3": [_P, _P, _P, ctypes.c_int64],
        "mm_compute_heff": [_P, _P, _P, ctypes.c_uint32],
        "mm_step_llg": [_P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32],
        "mm_reduce": [_P, _P, _P],
        "mm_sync": [_P],
        "mm_kernel_timing": [_P, ctypes.c_int],
        "mm_set_compensated": [_P, ctypes.c_int],
        "mm_set_fusion": [_P, ctypes.c_int],
        "mm_batch_set_fusion": [_P, ctypes.c_int],
        "mm_set_tuning": [_P, ctypes.POINTER(ctypes.c_int32)],
        "mm_get_tuning": [_P, ctypes.POINTER(ctypes.c_int32)],
        "mm_autotune": [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)],
        "mm_step_adaptive": [_P, _P, ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                             ctypes.c_uint32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_int64)],
        "mm_forward_store": [_P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32, _P, _P],
        "mm_adjoint_step": [_P, _P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_uint32],
        "mm_adjoint_segment": [_P, _P, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_double, ctypes.c_uint32],
        "mm_kernel_times": [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
        "mm_set_field_schedule": [_P, ctypes.POINTER(ctypes.c_double)],
        "mm_set_time": [_P, ctypes.c_double],
        "mm_get_time": [_P, ctypes.POINTER(ctypes.c_double)],
        "mm_reduce_loss": [_P, _P, _P, _P, _P],
        "mm_reduce_loss_noalloc": [_P, _P, _P, _P, _P],
    }
    sig.update({
        "mm_batch_create": [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_double,
                            ctypes.c_double, ctypes.c_double, ctypes.c_int, _P],
        "mm_batch_destroy": [_P],
        "mm_batch_set_stream": [_P, _P],
        "mm_batch_state_offsets": [_P, ctypes.POINTER(ctypes.c_int64)],
        "mm_batch_workspace_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
        "mm_batch_set_workspace": [_P, _P, ctypes.c_size_t],
        "mm_batch_set_material": [_P, ctypes.POINTER(mm_material)],
        "mm_batch_set_hext": [_P, ctypes.POINTER(ctypes.c_double)],
        "mm_batch_build_tensor": [_P],
        "mm_batch_step": [_P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32],
        "mm_batch_sync": [_P],
        "mm_batch_autotune": [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32)],
        "mm_batch_set_tuning": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
        "mm_batch_get_tuning": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    })
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.mm_last_error.argtypes = [_P]
    L.mm_last_error.restype = ctypes.c_char_p
    L.mm_batch_last_error.argtypes = [_P]
    L.mm_batch_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def mm_last_error(ctx) -> str:
    return load().mm_last_error(ctx).decode()


def _check(ctx, status, what):
    if status != MM_OK:
        msg = mm_last_error(ctx) if ctx else ""
        raise MMError(status, f"{what}: {msg}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C names

def mm_create(n, d, device=0, stream=None):
    g = mm_geometry(int(n[0]), int(n[1]), int(n[2]), float(d[0]), float(d[1]), float(d[2]))
    ctx = _P()
    s = stream if stream is not None else _stream()
    _check(None, load().mm_create(ctypes.byref(ctx), ctypes.byref(g), int(device), s), "mm_create")
    return ctx


def mm_destroy(ctx):
    _check(None, load().mm_destroy(ctx), "mm_destroy")


def mm_set_stream(ctx, stream=None):
    _check(ctx, load().mm_set_stream(ctx, stream if stream is not None else _stream()), "mm_set_stream")


def mm_workspace_size(ctx) -> int:
    b = ctypes.c_size_t()
    _check(ctx, load().mm_workspace_size(ctx, ctypes.byref(b)), "mm_workspace_size")
    return b.value


def mm_set_workspace(ctx, ws):
    _check(ctx, load().mm_set_workspace(ctx, ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()),
           "mm_set_workspace")


def mm_set_material(ctx, Ms, A, Ku=0.0, u=(1.0, 0.0, 0.0), alpha=0.5, gamma0=2.211e5):
    m = mm_material(float(Ms), float(A), float(Ku), (ctypes.c_double * 3)(*map(float, u)),
                    float(alpha), float(gamma0))
    _check(ctx, load().mm_set_material(ctx, ctypes.byref(m)), "mm_set_material")


def mm_set_ms_map(ctx, ms, N=None):
    import torch
    p = None if ms is None else _dev(ms, torch.float32, N if N is not None else ms.numel(), "ms map")
    _check(ctx, load().mm_set_ms_map(ctx, p), "mm_set_ms_map")


def mm_set_hext(ctx, h):
    arr = (ctypes.c_double * 3)(*map(float, h))
    _check(ctx, load().mm_set_hext(ctx, arr), "mm_set_hext")


def mm_set_hext_map(ctx, h, N=None):
    import torch
    p = None if h is None else _dev(h, torch.float32, 3 * N if N is not None else h.numel(), "field map")
    _check(ctx, load().mm_set_hext_map(ctx, p), "mm_set_hext_map")


def mm_build_tensor(ctx):
    _check(ctx, load().mm_build_tensor(ctx), "mm_build_tensor")


def mm_tensor_table(ctx, out, N):
    import torch
    _check(ctx, load().mm_tensor_table(ctx, _dev(out, torch.float64, 6 * N, "table")), "mm_tensor_table")


def mm_diag_dot3(ctx, inp, out, n):
    """Plain and compensated three-term dot products of n triples (6n floats
    in, 2n floats out), as the spectral multiply computes them."""
    import torch
    n = int(n)
    _check(ctx, load().mm_diag_dot3(ctx, _dev(inp, torch.float32, 6 * n, "in") if n else None,
                                    _dev(out, torch.float32, 2 * n, "out") if n else None, n), "mm_diag_dot3")


def mm_compute_heff(ctx, m, h, terms, N):
    import torch
    _check(ctx, load().mm_compute_heff(ctx, _dev(m, torch.float32, 3 * N, "m"),
                                       _dev(h, torch.float32, 3 * N, "h"), int(terms)), "mm_compute_heff")


def mm_step_llg(ctx, m, nsteps, dt, flags, N):
    import torch
    _check(ctx, load().mm_step_llg(ctx, _dev(m, torch.float32, 3 * N, "m"), int(nsteps), float(dt), int(flags)),
           "mm_step_llg")


def mm_reduce(ctx, m, out, N):
    import torch
    _check(ctx, load().mm_reduce(ctx, _dev(m, torch.float32, 3 * N, "m"), _dev(out, torch.float64, 8, "out")),
           "mm_reduce")


def mm_reduce_loss(ctx, m, target, out, grad, N):
    import torch
    g = None if grad is None else _dev(grad, torch.float32, 3 * N, "grad")
    _check(ctx, load().mm_reduce_loss(ctx, _dev(m, torch.float32, 3 * N, "m"),
                                      _dev(target, torch.float32, 3 * N, "target"),
                                      _dev(out, torch.float64, 1, "out"), g), "mm_reduce_loss")


def mm_reduce_loss_noalloc(ctx, m, target, out, grad, N):
    import torch
    g = None if grad is None else _dev(grad, torch.float32, 3 * N, "grad")
    _check(ctx, load().mm_reduce_loss_noalloc(ctx, _dev(m, torch.float32, 3 * N, "m"),
                                              _dev(target, torch.float32, 3 * N, "target"),
                                              _dev(out, torch.float64, 1, "out"), g), "mm_reduce_loss_noalloc")


def mm_set_field_schedule(ctx, sched):
    arr = None if sched is None else (ctypes.c_double * 3)(*map(float, sched))
    _check(ctx, load().mm_set_field_schedule(ctx, arr), "mm_set_field_schedule")


def mm_set_time(ctx, t):
    _check(ctx, load().mm_set_time(ctx, float(t)), "mm_set_time")


def mm_get_time(ctx):
    t = ctypes.c_double()
    _check(ctx, load().mm_get_time(ctx, ctypes.byref(t)), "mm_get_time")
    return t.value


def mm_sync(ctx):
    _check(ctx, load().mm_sync(ctx), "mm_sync")


def mm_set_fusion(ctx, level):
    """0: two kernels; 1: x-inverse + update fused; 2: also the next x-forward."""
    _check(ctx, load().mm_set_fusion(ctx, int(level)), "mm_set_fusion")


def mm_set_compensated(ctx, on):
    _check(ctx, load().mm_set_compensated(ctx, int(bool(on))), "mm_set_compensated")


MM_TUNE_VARIANTS = 3


def mm_set_tuning(ctx, choice):
    arr = (ctypes.c_int32 * 3)(*[int(v) for v in choice])
    _check(ctx, load().mm_set_tuning(ctx, arr), "mm_set_tuning")


def mm_get_tuning(ctx):
    arr = (ctypes.c_int32 * 3)()
    _check(ctx, load().mm_get_tuning(ctx, arr), "mm_get_tuning")
    return tuple(arr)


def mm_autotune(ctx, cache_path=None):
    """Fastest launch-shape variant per pass for this geometry (x, y, z)."""
    arr = (ctypes.c_int32 * 3)()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(ctx, load().mm_autotune(ctx, path, arr), "mm_autotune")
    return tuple(arr)


def mm_step_adaptive(ctx, m, t_end, dt, tol, flags, max_steps, N):
    """Returns (last proposed dt, accepted attempts, rejected attempts)."""
    import torch
    d = ctypes.c_double(float(dt))
    a, r = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(ctx, load().mm_step_adaptive(ctx, _dev(m, torch.float32, 3 * N, "m"), float(t_end), ctypes.byref(d),
                                        float(tol), int(flags), int(max_steps), ctypes.byref(a), ctypes.byref(r)),
           "mm_step_adaptive")
    return d.value, a.value, r.value


def mm_forward_store(ctx, m, nsteps, dt, flags, m_traj, hd_traj, N):
    import torch
    n = int(nsteps)
    _check(ctx, load().mm_forward_store(ctx, _dev(m, torch.float32, 3 * N, "m"), n, float(dt), int(flags),
                                        _dev(m_traj, torch.float32, 3 * N * n, "m_traj") if n else None,
                                        _dev(hd_traj, torch.float32, 3 * N * n, "hd_traj") if n else None),
           "mm_forward_store")


def mm_adjoint_step(ctx, m_n, hd_n, lam, g_hext, g_ms, dt, flags, N):
    import torch
    gh = None if g_hext is None else _dev(g_hext, torch.float32, 3 * N, "g_hext")
    gm = None if g_ms is None else _dev(g_ms, torch.float32, N, "g_ms")
    _check(ctx, load().mm_adjoint_step(ctx, _dev(m_n, torch.float32, 3 * N, "m_n"),
                                       _dev(hd_n, torch.float32, 3 * N, "hd_n"),
                                       _dev(lam, torch.float32, 3 * N, "lam"), gh, gm, float(dt), int(flags)),
           "mm_adjoint_step")


def mm_adjoint_segment(ctx, m_traj, hd_traj, n, lam, g_hext, g_ms, dt, flags, N):
    """n adjoint steps (n-1 down to 0) of a stored segment in one call."""
    import torch
    n = int(n)
    gh = None if g_hext is None else _dev(g_hext, torch.float32, 3 * N, "g_hext")
    gm = None if g_ms is None else _dev(g_ms, torch.float32, N, "g_ms")
    _check(ctx, load().mm_adjoint_segment(ctx, _dev(m_traj, torch.float32, 3 * N * n, "m_traj"),
                                          _dev(hd_traj, torch.float32, 3 * N * n, "hd_traj"), n,
                                          _dev(lam, torch.float32, 3 * N, "lam"), gh, gm, float(dt), int(flags)),
           "mm_adjoint_segment")


MM_K_NAMES = ["xfwd", "yfwd", "zconv", "yinv", "xinv", "local", "xinv_local", "xinv_local_xfwd"]


def mm_kernel_timing(ctx, enable):
    _check(ctx, load().mm_kernel_timing(ctx, int(bool(enable))), "mm_kernel_timing")


def mm_kernel_times(ctx):
    """{kernel name: (total ms, launches)} accumulated since timing was enabled."""
    n = len(MM_K_NAMES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(ctx, load().mm_kernel_times(ctx, ms, cnt), "mm_kernel_times")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(MM_K_NAMES)}


def _bcheck(b, status, what):
    if status != MM_OK:
        msg = load().mm_batch_last_error(b).decode() if b else ""
        raise MMError(status, f"{what}: {msg}")


def mm_batch_create(sizes, d, device=0, stream=None):
    arr = (ctypes.c_int32 * (3 * len(sizes)))(*[int(v) for s in sizes for v in s])
    b = _P()
    s = stream if stream is not None else _stream()
    _bcheck(None, load().mm_batch_create(ctypes.byref(b), len(sizes), arr, float(d[0]), float(d[1]), float(d[2]),
                                         int(device), s), "mm_batch_create")
    return b


def mm_batch_destroy(b):
    _bcheck(None, load().mm_batch_destroy(b), "mm_batch_destroy")


def mm_batch_set_stream(b, stream=None):
    _bcheck(b, load().mm_batch_set_stream(b, stream if stream is not None else _stream()), "mm_batch_set_stream")


def mm_batch_state_offsets(b, count):
    off = (ctypes.c_int64 * (count + 1))()
    _bcheck(b, load().mm_batch_state_offsets(b, off), "mm_batch_state_offsets")
    return list(off)


def mm_batch_workspace_size(b):
    v = ctypes.c_size_t()
    _bcheck(b, load().mm_batch_workspace_size(b, ctypes.byref(v)), "mm_batch_workspace_size")
    return v.value


def mm_batch_set_workspace(b, ws):
    _bcheck(b, load().mm_batch_set_workspace(b, ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()),
            "mm_batch_set_workspace")


def mm_batch_set_material(b, Ms, A, Ku=0.0, u=(1.0, 0.0, 0.0), alpha=0.5, gamma0=2.211e5):
    m = mm_material(float(Ms), float(A), float(Ku), (ctypes.c_double * 3)(*map(float, u)), float(alpha), float(gamma0))
    _bcheck(b, load().mm_batch_set_material(b, ctypes.byref(m)), "mm_batch_set_material")


def mm_batch_set_hext(b, h):
    flat = [float(v) for row in h for v in row]
    _bcheck(b, load().mm_batch_set_hext(b, (ctypes.c_double * len(flat))(*flat)), "mm_batch_set_hext")


def mm_batch_build_tensor(b):
    _bcheck(b, load().mm_batch_build_tensor(b), "mm_batch_build_tensor")


def mm_batch_step(b, m, nsteps, dt, flags, total):
    import torch
    _bcheck(b, load().mm_batch_step(b, _dev(m, torch.float32, total, "packed state"), int(nsteps), float(dt),
                                    int(flags)), "mm_batch_step")


def mm_batch_sync(b):
    _bcheck(b, load().mm_batch_sync(b), "mm_batch_sync")


def mm_batch_get_tuning(b):
    n = ctypes.c_int32()
    _bcheck(b, load().mm_batch_get_tuning(b, None, 0, ctypes.byref(n)), "mm_batch_get_tuning")
    arr = (ctypes.c_int32 * max(n.value, 1))()
    _bcheck(b, load().mm_batch_get_tuning(b, arr, n.value, ctypes.byref(n)), "mm_batch_get_tuning")
    return tuple(arr[:n.value])


def mm_batch_set_fusion(b, on):
    _bcheck(b, load().mm_batch_set_fusion(b, int(bool(on))), "mm_batch_set_fusion")


def mm_batch_set_tuning(b, choices):
    arr = (ctypes.c_int32 * max(len(choices), 1))(*[int(v) for v in choices])
    _bcheck(b, load().mm_batch_set_tuning(b, arr, len(choices)), "mm_batch_set_tuning")


def mm_batch_autotune(b, cache_path=None):
    """Fastest launch-shape variant of each x, y and z launch of the batch."""
    n = len(mm_batch_get_tuning(b))
    arr = (ctypes.c_int32 * max(n, 1))()
    cnt = ctypes.c_int32()
    path = None if cache_path is None else os.fsencode(cache_path)
    _bcheck(b, load().mm_batch_autotune(b, path, arr, n, ctypes.byref(cnt)), "mm_batch_autotune")
    return tuple(arr[:cnt.value])


class Batch:
    """Many independent samples (own sizes and uniform fields, one cell size
    and material) on one GPU; the state is one packed tensor."""

    def __init__(self, sizes, d, Ms, A, Ku=0.0, u=(1.0, 0.0, 0.0), alpha=0.5, gamma0=2.211e5, hext=None, device=0):
        import torch
        self.sizes = [tuple(int(v) for v in s) for s in sizes]
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            self.b = mm_batch_create(self.sizes, d, device)
            self.offsets = mm_batch_state_offsets(self.b, len(self.sizes))
            nbytes = mm_batch_workspace_size(self.b)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            mm_batch_set_workspace(self.b, self.ws[off:off + nbytes])
            mm_batch_set_material(self.b, Ms, A, Ku, u, alpha, gamma0)
            mm_batch_set_hext(self.b, hext if hext is not None else [(0.0, 0.0, 0.0)] * len(self.sizes))
            mm_batch_build_tensor(self.b)

    @property
    def total(self):
        return self.offsets[-1]

    def pack(self, states):
        """Packed device state from a list of [3][nz][ny][nx] arrays."""
        import torch
        out = torch.zeros(self.total, dtype=torch.float32, device=self.device)
        for s, o in zip(states, self.offsets):
            t = torch.as_tensor(s, dtype=torch.float32).reshape(-1)
            out[o:o + t.numel()] = t.to(self.device)
        return out

    def unpack(self, packed, i):
        nx, ny, nz = self.sizes[i]
        o = self.offsets[i]
        return packed[o:o + 3 * nx * ny * nz].reshape(3, nz, ny, nx)

    def step(self, m, nsteps, dt, flags=0):
        mm_batch_set_stream(self.b)
        mm_batch_step(self.b, m, nsteps, dt, flags, self.total)
        return m

    def autotune(self, cache_path=None):
        mm_batch_set_stream(self.b)
        return mm_batch_autotune(self.b, cache_path)

    def set_tuning(self, choices):
        mm_batch_set_tuning(self.b, choices)

    def set_fusion(self, on):
        mm_batch_set_fusion(self.b, on)

    def tuning(self):
        return mm_batch_get_tuning(self.b)

    def sync(self):
        mm_batch_sync(self.b)

    def close(self):
        if getattr(self, "b", None):
            mm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -------------------------------------------------------------- convenience

class Sim:
    """One sample on one GPU: owns the context and a torch workspace tensor.

    ``Sim(n, d, Ms=..., A=..., ...)`` creates the context, sets the material,
    hands over the workspace and builds the tensor spectrum.  Methods enqueue
    on torch's current stream."""

    def __init__(self, n, d, Ms, A, Ku=0.0, u=(1.0, 0.0, 0.0), alpha=0.5, gamma0=2.211e5,
                 hext=(0.0, 0.0, 0.0), device=0, build_tensor=True):
        import torch
        self.n, self.d = tuple(int(v) for v in n), tuple(float(v) for v in d)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            self.ctx = mm_create(self.n, self.d, device)
            nbytes = mm_workspace_size(self.ctx)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self._ws_view = self.ws[off:off + nbytes]
            mm_set_workspace(self.ctx, self._ws_view)
            mm_set_material(self.ctx, Ms, A, Ku, u, alpha, gamma0)
            mm_set_hext(self.ctx, hext)
            if build_tensor:
                mm_build_tensor(self.ctx)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (3, nz, ny, nx)

    def _s(self):
        mm_set_stream(self.ctx)

    def heff(self, m, terms=MM_T_ALL):
        import torch
        self._s()
        h = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        mm_compute_heff(self.ctx, m, h, terms, self.N)
        return h

    def step(self, m, nsteps, dt, flags=0):
        self._s()
        mm_step_llg(self.ctx, m, nsteps, dt, flags, self.N)
        return m

    def run_adaptive(self, m, t_end, dt0, tol, flags=MM_F_HEUN, max_steps=10**7):
        """Adaptive steps of m (in place) up to t_end: (dt, accepted, rejected)."""
        self._s()
        return mm_step_adaptive(self.ctx, m, t_end, dt0, tol, flags, max_steps, self.N)

    def autotune(self, cache_path=None):
        self._s()
        return mm_autotune(self.ctx, cache_path)

    def set_tuning(self, choice):
        mm_set_tuning(self.ctx, choice)

    def reduce(self, m):
        import torch
        self._s()
        out = torch.empty(8, dtype=torch.float64, device=self.device)
        mm_reduce(self.ctx, m, out, self.N)
        return out

    def loss(self, m, target, grad=False):
        """FP64 loss 1/2 sum (m - target)^2 on the GPU: a 1-element float64
        tensor, and with grad=True also dL/dm = m - target (FP32)."""
        import torch
        self._s()
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty(self.shape, dtype=torch.float32, device=self.device) if grad else None
        mm_reduce_loss(self.ctx, m, target, out, g, self.N)
        return (out, g) if grad else out

    def set_field_schedule(self, sched):
        """(t_start, t_decay, t_stop) in s, or None for a constant field."""
        mm_set_field_schedule(self.ctx, sched)

    def set_time(self, t):
        self._s()
        mm_set_time(self.ctx, t)

    def time(self):
        self._s()
        return mm_get_time(self.ctx)

    def tensor_table(self):
        import torch
        self._s()
        out = torch.empty((6,) + self.shape[1:], dtype=torch.float64, device=self.device)
        mm_tensor_table(self.ctx, out, self.N)
        return out

    def set_ms_map(self, ms):
        self._s()
        mm_set_ms_map(self.ctx, ms, self.N)

    def set_hext_map(self, h):
        self._s()
        mm_set_hext_map(self.ctx, h, self.N)

    def set_hext(self, h):
        mm_set_hext(self.ctx, h)

    def sync(self):
        mm_sync(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            mm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
