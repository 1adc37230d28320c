"""Seeded synthetic inputs for the micromagnetic workloads.

This module draws random numbers and fixes parameters; it holds none of the
method's arithmetic (no fields, no tensor, no integrator).  Both the GPU
library's tests/benchmarks and the CPU oracle's tests take their inputs from
here, so the two sides see identical data.

All random draws are FP64 from ``numpy.random.default_rng(seed)`` (PCG64), in
the order written below.  Material values follow the paper's workloads: the
mu-MAG standard problem #4 material (Ms = 8.0e5 A/m, A = 1.3e-11 J/m,
alpha = 0.02, Sec. 4) for the films, and cubic 5 nm cells for the blocks.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

MU0 = 4.0e-7 * np.pi
GAMMA0 = 2.211e5  # gamma * mu0, m/(A s)


@dataclass(frozen=True)
class Workload:
    name: str
    n: tuple                    # (nx, ny, nz) cells
    d: tuple                    # cell size (dx, dy, dz), m
    Ms: float
    A: float
    alpha: float
    dt: float
    nsteps: int
    Ku: float = 0.0
    u: tuple = (1.0, 0.0, 0.0)
    gamma0: float = GAMMA0
    init: str = "sphere"        # "sphere" | "near_uniform"
    seed: int = 0
    field_mT: float = 0.0       # uniform in-plane field magnitude drawn after m0
    extra: dict = field(default_factory=dict, compare=False)

    @property
    def N(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (3, nz, ny, nx)


def unit(v, axis=0):
    return v / np.linalg.norm(v, axis=axis, keepdims=True)


def sphere(rng, shape):
    """Unit vectors uniform on the sphere (normalised Gaussian triples)."""
    return unit(rng.standard_normal(shape))


def near_uniform(rng, shape, base=(1.0, 0.1, 0.0), sigma=0.05):
    """(1, 0.1, 0) plus N(0, sigma) per cell and component, renormalised."""
    b = np.asarray(base, dtype=np.float64).reshape((3,) + (1,) * (len(shape) - 1))
    return unit(b + sigma * rng.standard_normal(shape))


# --------------------------------------------------------------- workloads --

BLOCK_16x16x2 = Workload("block 16x16x2, 5 nm cubes", (16, 16, 2), (5e-9,) * 3,
                         Ms=8.0e5, A=1.3e-11, alpha=0.5, dt=1e-13, nsteps=100)

FILM_256x64x1 = Workload("film 256x64x1, 4x4x3 nm cells", (256, 64, 1), (4e-9, 4e-9, 3e-9),
                         Ms=8.0e5, A=1.3e-11, alpha=0.02, dt=5e-14, nsteps=20000,
                         Ku=5e2, u=(1.0, 0.0, 0.0), init="near_uniform", field_mT=25.0)

BLOCK_256x256x32 = Workload("block 256x256x32, 5 nm cubes", (256, 256, 32), (5e-9,) * 3,
                            Ms=8.6e5, A=1.3e-11, alpha=0.1, dt=1e-13, nsteps=1000)

# standalone trajectory sample with the large block's material (seed 1)
BLOCK_64x64x8 = replace(BLOCK_256x256x32, name="block 64x64x8, 5 nm cubes", n=(64, 64, 8),
                        seed=1, nsteps=100)

FILM_128x128x4 = Workload("film 128x128x4, 5 nm cubes (adjoint)", (128, 128, 4), (5e-9,) * 3,
                          Ms=8.0e5, A=1.3e-11, alpha=0.05, dt=1e-13, nsteps=2000,
                          init="near_uniform", field_mT=20.0)


# Table 1's benchmark: N x N x N cubes, A = 1e-11 J/m, Ms = 1e6 A/m and an
# anisotropy field 2 Ku / (mu0 Ms) = 1e5 A/m (Sec. 4).  The paper states no
# cell size, axis, damping or time step: 5 nm cubes, easy axis x, alpha = 0.5
# (the sample relaxes) and dt = 1e-13 s (stable for these cells) are used.
TABLE1_SIZES = (8, 16, 32, 64, 128, 256)


def table1_cube(N: int) -> Workload:
    Ms, HK = 1.0e6, 1.0e5
    return Workload(f"cube {N}x{N}x{N}, 5 nm cells", (N, N, N), (5e-9,) * 3,
                    Ms=Ms, A=1.0e-11, alpha=0.5, dt=1e-13, nsteps=1000,
                    Ku=0.5 * MU0 * Ms * HK, u=(1.0, 0.0, 0.0))


# Standard problem #4 as the paper runs it (Sec. 4): 500 x 125 x 3 cells of
# 1 nm, A = 1.3e-11 J/m, Ms = 8.0e5 A/m, no anisotropy; relaxed at large
# damping, then reversed at alpha = 0.02 under field 1 or field 2 (mT, as
# B = mu0 H).  The paper's input file uses dt = 1e-13 s, far above the
# explicit Euler limit for 1 nm cells at alpha = 0.02 (about 6e-16 s): that dt
# serves for timing only; trajectories are compared at SP4_STABLE_DT.
SP4_FIELD1_mT = (-24.6, 4.3, 0.0)
SP4_FIELD2_mT = (-35.5, -6.3, 0.0)
SP4_STABLE_DT = 2e-16
SP4_500x125x3 = Workload("film 500x125x3, 1 nm cells (standard problem #4)", (500, 125, 3), (1e-9,) * 3,
                         Ms=8.0e5, A=1.3e-11, alpha=0.02, dt=1e-13, nsteps=10000,
                         init="near_uniform")


def disk_ms_map(n, Ms, fill=1.0):
    """Ms map of the elliptic cylinder inscribed in the grid's x-y extent
    (a disk on a square grid), through all z layers: Ms at cells whose
    centre lies inside (semi-axes fill * nx/2, fill * ny/2), 0 (vacuum)
    elsewhere.  Shape [nz][ny][nx]."""
    nx, ny, nz = n
    x = (np.arange(nx) + 0.5) / nx * 2.0 - 1.0
    y = (np.arange(ny) + 0.5) / ny * 2.0 - 1.0
    X, Y = np.meshgrid(x, y)
    inside = X * X + Y * Y < fill * fill
    return np.broadcast_to(np.where(inside, float(Ms), 0.0), (nz, ny, nx)).copy()


# Non-regular geometry (Sec. 6): a film disk of 256 nm diameter, 4x4x3 nm
# cells on a 64x64x2 grid, the SP4 material at alpha = 0.1, a 20 mT field
# at a seeded in-plane angle, dt = 5e-14 s.
DISK_64x64x2 = Workload("disk film on 64x64x2 cells, 4x4x3 nm (vacuum outside the disk)", (64, 64, 2),
                        (4e-9, 4e-9, 3e-9), Ms=8.0e5, A=1.3e-11, alpha=0.1, dt=5e-14, nsteps=100,
                        init="near_uniform", field_mT=20.0)


def field_mT(b_mT):
    """A field given as B = mu0 H in mT, returned as H in A/m."""
    return np.asarray(b_mT, dtype=np.float64) * (1e-3 / MU0)


def initial_m(w: Workload):
    """m0 for a workload, and the rng positioned after the m0 draw."""
    rng = np.random.default_rng(w.seed)
    if w.init == "sphere":
        m = sphere(rng, w.shape)
    else:
        m = near_uniform(rng, w.shape)
    return m, rng


def uniform_field(w: Workload, rng):
    """In-plane field of |B| = field_mT at an angle drawn after m0, in A/m."""
    th = rng.uniform(0.0, 2.0 * np.pi)
    return np.array([np.cos(th), np.sin(th), 0.0]) * (w.field_mT * 1e-3 / MU0)


def inputs(w: Workload):
    """(m0, h_ext uniform 3-vector in A/m) for a single-sample workload."""
    m, rng = initial_m(w)
    h = uniform_field(w, rng) if w.field_mT else np.zeros(3)
    return m, h


def adjoint_inputs(w: Workload = FILM_128x128x4):
    """m0, per-cell Ms map, per-cell h_ext map and the smooth target pattern
    for the gradient workload.  Draw order: m0, field angle, (a, b)."""
    m, rng = initial_m(w)
    nx, ny, nz = w.n
    h = uniform_field(w, rng)
    hmap = np.broadcast_to(h.reshape(3, 1, 1, 1), w.shape).copy()
    msmap = np.full(w.shape[1:], w.Ms)
    a, b = rng.uniform(0.0, 2.0 * np.pi, 2)
    Lx, Ly = nx * w.d[0], ny * w.d[1]
    x = (np.arange(nx) + 0.5) * w.d[0]
    y = (np.arange(ny) + 0.5) * w.d[1]
    X, Y = np.meshgrid(x, y)  # [ny][nx]
    phi = np.pi / 4 + 0.5 * np.sin(2 * np.pi * X / Lx + a) * np.cos(2 * np.pi * Y / Ly + b)
    t = np.stack([np.cos(phi), np.sin(phi), 0.2 * np.sin(2 * np.pi * (X / Lx + Y / Ly))])
    t = unit(t)
    target = np.broadcast_to(t[:, None], w.shape).copy()
    return m, msmap, hmap, target


def batch_films(count=64, seed=0):
    """Ragged batch of thin films: sizes nx in [64, 256], ny in [64, 128],
    nz in {1, 2}; field magnitude uniform in [0, 50] mT along a direction
    uniform on the sphere; m0 near-uniform.  Draw order per sample: nx, ny,
    nz, |B|, direction, m0."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        nx = int(rng.integers(64, 257))
        ny = int(rng.integers(64, 129))
        nz = int(rng.integers(1, 3))
        B = rng.uniform(0.0, 50.0)
        direction = unit(rng.standard_normal(3))
        w = Workload(f"film {nx}x{ny}x{nz} #{b}", (nx, ny, nz), (4e-9, 4e-9, 3e-9),
                     Ms=8.0e5, A=1.3e-11, alpha=0.02, dt=5e-14, nsteps=5000,
                     init="near_uniform")
        m = near_uniform(rng, w.shape)
        h = direction * (B * 1e-3 / MU0)
        out.append((w, m, h))
    return out
