"""The local kernel's block order on grids whose z-planes span 8q blocks.

The field/update kernel permutes its blocks so that each XCD takes the same
eighth of every z-plane (q blocks per plane each).  A wrong permutation would
leave cells unvisited or visit them twice.  Both show up as O(1) errors here:
- the local field terms (exchange, anisotropy, Zeeman) on the whole grid
  against the FP64 oracle;
- one Euler step against the oracle's LLG right-hand side, evaluated at the
  GPU's own full field (so the test needs no O(N^2) demag on the CPU).

Grids: 96x256x4 (24 blocks of 1024 cells per plane, q = 3) and 192x256x3
(48 per plane, q = 6).  With one cell per thread (nx % 4 != 0) a plane of 8q
blocks would need ny >= 1024, beyond the largest grid, so that form always
keeps the launch order.
"""
import numpy as np
import pytest

import oracle
from paper_1411_2565_amd import workloads

pytestmark = pytest.mark.gpu

LOCAL = 1 | 4 | 8  # exchange, anisotropy, Zeeman
KW = dict(Ms=8e5, A=1.3e-11, Ku=4e4, u=(0.0, 0.6, 0.8), alpha=0.3)
HEXT = (2e4, -1e4, 5e3)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.mark.parametrize("n", [(96, 256, 4), (192, 256, 3)])
def test_local_terms_and_step_on_permuted_grid(gpu_lib, n):
    import torch
    d = (4e-9, 4e-9, 3e-9)
    rng = np.random.default_rng(sum(n))
    m0 = workloads.sphere(rng, (3,) + n[::-1]).astype(np.float32).astype(np.float64)
    P = oracle.Problem(n, d, hext=HEXT, **KW)
    sim = gpu_lib.Sim(n, d, hext=HEXT, **KW)
    m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")

    h_loc = sim.heff(m, LOCAL).double().cpu().numpy()
    e_loc = rel(h_loc, P.heff(m0, LOCAL))
    print(f"{n}: local terms rel L2 vs oracle {e_loc:.2e}")
    assert e_loc < 1e-5

    h_all = sim.heff(m, gpu_lib.MM_T_ALL).double().cpu().numpy()
    dt = 1e-13
    sim.step(m, 1, dt)
    sim.sync()
    m1 = m.double().cpu().numpy()
    ref = m0 + dt * P.llg_rhs(m0, h_all)
    ref /= np.linalg.norm(ref, axis=0, keepdims=True)
    err = np.abs(m1 - ref).max()
    print(f"{n}: one Euler step, max |m1 - ref| {err:.2e}")
    assert err < 1e-5
    sim.close()
