"""FP64 CPU oracle for the micromagnetic step (test infrastructure only).

This package is the reference the GPU library is checked against.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg import it;
the product library never does.  It shares no code with the GPU path: the
arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP), and this module only
marshals numpy arrays into it.

Paper: R. Zhu, "Grace: a Cross-platform Micromagnetic Simulator On Graphics
Processing Units", arXiv:1411.2565.  Sec. 2 (eqs. 1-3) defines the energy,
effective field and LLG equation; Sec. 3 the demag convolution, six-neighbour
exchange and explicit Euler integration.  Every function below is pinned by
the ``-m "not gpu"`` tests (closed forms, invariants, brute force).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import _build

MU0 = 4.0e-7 * np.pi
T_EXCH, T_DEMAG, T_ANIS, T_ZEEMAN = 1, 2, 4, 8
T_ALL = 15

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("A", ctypes.c_double), ("Ku", ctypes.c_double), ("u", ctypes.c_double * 3),
        ("alpha", ctypes.c_double), ("gamma0", ctypes.c_double),
        ("Ms", _D), ("hext", _D), ("tab", _D),
        ("terms", ctypes.c_int), ("renorm", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.library_path()
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_tensor_at.argtypes = [ctypes.c_double] * 6 + [ctypes.c_int, ctypes.c_int, _D]
        L.orc_tensor_table.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [_D]
        L.orc_conv.argtypes = [ctypes.c_int] * 3 + [_D, _D, _D]
        L.orc_laplacian.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [_D, _D]
        P = ctypes.POINTER(_Problem)
        L.orc_demag.argtypes = [P, _D, _D]
        L.orc_demag_observers.argtypes = [P, _D, _I64, ctypes.c_int64, _D]
        L.orc_heff.argtypes = [P, _D, ctypes.c_int, _D]
        L.orc_llg_rhs.argtypes = [P, _D, _D, _D]
        L.orc_step.argtypes = [P, _D, ctypes.c_double, _D]
        L.orc_run.argtypes = [P, _D, ctypes.c_int64, ctypes.c_double, _D]
        L.orc_run_rk.argtypes = [P, _D, ctypes.c_int64, ctypes.c_double, ctypes.c_int]
        L.orc_run_rk.restype = ctypes.c_int
        L.orc_run_adaptive.argtypes = [P, _D, ctypes.c_double, _D, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int64, _I64, _I64]
        L.orc_run_adaptive.restype = ctypes.c_int
        L.orc_energy.argtypes = [P, _D, _D]
        L.orc_adjoint.argtypes = [P, _D, ctypes.c_int64, ctypes.c_double, _D, _D, _D, _D]
        L.orc_adjoint.restype = ctypes.c_double
        L.orc_step_cells.argtypes = [P, _D, _I64, ctypes.c_int64, ctypes.c_double, _D]
        L.orc_threads.restype = ctypes.c_int
        L.orc_field_scale.argtypes = [ctypes.c_double] * 4
        L.orc_field_scale.restype = ctypes.c_double
        L.orc_run_scheduled.argtypes = [P, _D, ctypes.c_int64] + [ctypes.c_double] * 5
        L.orc_run_scheduled.restype = ctypes.c_double
        L.orc_loss.argtypes = [_D, _D, ctypes.c_int64]
        L.orc_loss.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def tensor_at(X, Y, Z, dx, dy, dz, method=0, nodes=0):
    """Six tensor components (xx, yy, zz, xy, xz, yz) between two cells whose
    centres are (X, Y, Z) metres apart.  method 0 = the oracle's near/far
    split, 1 = Newell only, 2 = tent quadrature only (``nodes`` per half-axis)."""
    out = np.zeros(6)
    lib().orc_tensor_at(X, Y, Z, dx, dy, dz, method, nodes, _p(out))
    return out


def tensor_table(n, d):
    """Octant table [6][nz][ny][nx] of N at offsets 0 <= o < n."""
    nx, ny, nz = n
    tab = np.zeros((6, nz, ny, nx))
    lib().orc_tensor_table(nx, ny, nz, d[0], d[1], d[2], _p(tab))
    return tab


@dataclass
class Problem:
    """One micromagnetic problem in SI units (Sec. 2).  ``Ms`` and ``hext``
    may be scalars / 3-vectors (uniform) or per-cell maps."""

    n: tuple
    d: tuple
    Ms: object = 8.0e5
    A: float = 1.3e-11
    Ku: float = 0.0
    u: tuple = (1.0, 0.0, 0.0)
    alpha: float = 0.5
    gamma0: float = 2.211e5
    hext: object = (0.0, 0.0, 0.0)
    terms: int = T_ALL
    renorm: bool = True
    tab: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        nx, ny, nz = self.n
        N = nx * ny * nz
        Ms = np.asarray(self.Ms, dtype=np.float64)
        self._Ms = _f64(np.broadcast_to(Ms, (nz, ny, nx)) if Ms.ndim == 0 else Ms, (N,))
        if not (np.all(np.isfinite(self._Ms)) and np.all(self._Ms >= 0)):
            raise ValueError("Ms must be finite and >= 0 (0 marks a vacuum cell)")
        h = np.asarray(self.hext, dtype=np.float64)
        if h.shape == (3,):
            h = np.broadcast_to(h[:, None], (3, N))
        self._hext = _f64(h, (3, N))
        if self.tab is None:
            self.tab = tensor_table(self.n, self.d)
        self._tab = _f64(self.tab)
        self._st = _Problem(nx, ny, nz, self.d[0], self.d[1], self.d[2], self.A, self.Ku,
                            (ctypes.c_double * 3)(*self.u), self.alpha, self.gamma0,
                            _p(self._Ms), _p(self._hext), _p(self._tab),
                            int(self.terms), int(bool(self.renorm)))

    @property
    def N(self):
        return self.n[0] * self.n[1] * self.n[2]

    def _shape(self):
        nx, ny, nz = self.n
        return (3, nz, ny, nx)

    def _struct(self, terms=None):
        st = _Problem.from_buffer_copy(self._st)
        if terms is not None:
            st.terms = int(terms)
        return st

    def demag(self, m):
        m = _f64(m, self._shape())
        H = np.zeros_like(m)
        st = self._struct()
        lib().orc_demag(ctypes.byref(st), _p(m), _p(H))
        return H

    def demag_observers(self, m, obs):
        m = _f64(m, self._shape())
        obs = np.ascontiguousarray(obs, dtype=np.int64)
        out = np.zeros((3, obs.size))
        st = self._struct()
        lib().orc_demag_observers(ctypes.byref(st), _p(m), obs.ctypes.data_as(_I64),
                                  obs.size, _p(out))
        return out

    def heff(self, m, terms=None):
        m = _f64(m, self._shape())
        H = np.zeros_like(m)
        st = self._struct()
        lib().orc_heff(ctypes.byref(st), _p(m), int(self.terms if terms is None else terms), _p(H))
        return H

    def llg_rhs(self, m, H):
        m = _f64(m, self._shape())
        H = _f64(H, self._shape())
        f = np.zeros_like(m)
        st = self._struct()
        lib().orc_llg_rhs(ctypes.byref(st), _p(m), _p(H), _p(f))
        return f

    METHODS = {"euler": 0, "heun": 1, "rk4": 2}

    def run(self, m0, nsteps, dt, traj=False, method="euler"):
        """nsteps steps from m0: explicit Euler (Sec. 3), or Heun / classic
        fourth-order Runge-Kutta with renormalised stage states."""
        if method != "euler":
            if traj:
                raise ValueError("trajectories are stored for the Euler method only")
            m = _f64(m0, self._shape()).copy()
            st = self._struct()
            if lib().orc_run_rk(ctypes.byref(st), _p(m), int(nsteps), float(dt), self.METHODS[method]):
                raise ValueError(f"unknown method {method}")
            return m
        m = _f64(m0, self._shape()).copy()
        st = self._struct()
        tr = np.zeros((nsteps + 1,) + self._shape()) if traj else None
        lib().orc_run(ctypes.byref(st), _p(m), int(nsteps), float(dt),
                      _p(tr) if traj else ctypes.cast(None, _D))
        return (m, tr) if traj else m

    def run_scheduled(self, m0, nsteps, dt, schedule, t0=0.0):
        """nsteps Euler steps with the external field switched by ``schedule``
        = (t_start, t_decay, t_stop) in seconds (off, full, linear decay, off;
        see ``field_scale``), the first step at time t0.  Returns (m, t_end)."""
        m = _f64(m0, self._shape()).copy()
        st = self._struct()
        ts, td, tp = (float(v) for v in schedule)
        t = lib().orc_run_scheduled(ctypes.byref(st), _p(m), int(nsteps), float(dt), float(t0), ts, td, tp)
        return m, t

    PAIRS = {"heun_euler": 1, "bs23": 2, "dp54": 3}

    def run_adaptive(self, m0, t_end, dt0, tol, pair="heun_euler", max_steps=10**6):
        """Adaptive steps with an embedded pair up to time t_end: returns
        (m, last proposed dt, accepted steps, rejected steps)."""
        m = _f64(m0, self._shape()).copy()
        st = self._struct()
        dt = ctypes.c_double(float(dt0))
        acc, rej = ctypes.c_int64(0), ctypes.c_int64(0)
        rc = lib().orc_run_adaptive(ctypes.byref(st), _p(m), float(t_end), ctypes.byref(dt), float(tol),
                                    self.PAIRS[pair], int(max_steps), ctypes.byref(acc), ctypes.byref(rej))
        if rc:
            raise RuntimeError(f"orc_run_adaptive failed ({rc})")
        return m, dt.value, acc.value, rej.value

    def step_cells(self, m, cells, dt):
        """One Euler step evaluated only at the given linear cell indices
        (all sources enter the demag sum): updated m there, [3][ncells]."""
        m = _f64(m, self._shape())
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((3, cells.size))
        st = self._struct()
        lib().orc_step_cells(ctypes.byref(st), _p(m), cells.ctypes.data_as(_I64), cells.size,
                             float(dt), _p(out))
        return out

    def energy(self, m):
        m = _f64(m, self._shape())
        out = np.zeros(5)
        st = self._struct()
        lib().orc_energy(ctypes.byref(st), _p(m), _p(out))
        return out

    def adjoint(self, m0, nsteps, dt, target):
        """Loss 1/2 sum |m_T - t|^2 and its exact gradients w.r.t. m0, the
        external-field map and the Ms map (every cell magnetic)."""
        if np.any(self._Ms == 0):
            raise ValueError("the adjoint covers samples without vacuum cells")
        m0 = _f64(m0, self._shape())
        t = _f64(target, self._shape())
        gm = np.zeros(self._shape())
        gh = np.zeros(self._shape())
        gms = np.zeros(self._shape()[1:])
        st = self._struct()
        loss = lib().orc_adjoint(ctypes.byref(st), _p(m0), int(nsteps), float(dt), _p(t),
                                 _p(gm), _p(gh), _p(gms))
        return loss, gm, gh, gms


def field_scale(t, schedule):
    """Profile of the time-dependent external field at time t for
    schedule = (t_start, t_decay, t_stop): 0 before t_start, 1 up to
    t_decay, linear to 0 at t_stop, 0 after."""
    return lib().orc_field_scale(float(t), *(float(v) for v in schedule))


def loss(m, t):
    """1/2 sum (m - t)^2 over all components, FP64."""
    m = _f64(m).ravel()
    t = _f64(t).ravel()
    if m.size != t.size:
        raise ValueError("m and t differ in size")
    return lib().orc_loss(_p(m), _p(t), m.size)


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return lib().orc_threads()


def conv(n, tab, v):
    """sum_j N(r_i - r_j) v_j for an arbitrary field v [3][nz][ny][nx]."""
    nx, ny, nz = n
    v = _f64(v, (3, nz, ny, nx))
    out = np.zeros_like(v)
    tab = _f64(tab)
    lib().orc_conv(nx, ny, nz, _p(tab), _p(v), _p(out))
    return out


def laplacian(n, d, v):
    nx, ny, nz = n
    v = _f64(v, (3, nz, ny, nx))
    out = np.zeros_like(v)
    lib().orc_laplacian(nx, ny, nz, d[0], d[1], d[2], _p(v), _p(out))
    return out
