"""Non-regular geometry on the GPU (named as future work in Sec. 6): cells
with Ms = 0 in the Ms map are vacuum.  They are no demag source; exchange
omits them as neighbours; exchange and anisotropy fields vanish there; their
state never changes; energies and the mean magnetisation skip them.

Checks against the FP64 oracle (same rules): H_eff within 1e-5, 100 Euler
steps within 1e-4, RK4 and adaptive runs, energies within 1e-6; vacuum
padding leaves a sample's fields unchanged on the GPU too; a staircase
sphere (cubic symmetry) has an average demag field of exactly -M/3; invalid
maps are rejected.
"""
import numpy as np
import pytest

import oracle
from paper_1411_2565_amd import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda:0")


def host(t):
    return t.detach().cpu().double().numpy()


def disk_case(gpu_lib, Ku=0.0):
    w = workloads.DISK_64x64x2
    m0, h = workloads.inputs(w)
    ms = workloads.disk_ms_map(w.n, w.Ms)
    kw = dict(A=w.A, Ku=Ku, u=(0.6, 0.8, 0.0), alpha=w.alpha)
    sim = gpu_lib.Sim(w.n, w.d, Ms=w.Ms, hext=tuple(h), **kw)
    sim.set_ms_map(gpu(ms))
    m = gpu(m0)
    P = oracle.Problem(w.n, w.d, Ms=host(gpu(ms)), hext=h, **kw)
    return w, sim, P, m, ms > 0


def test_disk_heff_energy_and_trajectory(gpu_lib):
    w, sim, P, m, mag = disk_case(gpu_lib, Ku=2e4)
    mf = host(m)
    H = host(sim.heff(m))
    Ho = P.heff(mf)
    e_h = rel(H, Ho)
    assert np.all(host(sim.heff(m, gpu_lib.MM_T_EXCH | gpu_lib.MM_T_ANIS))[:, ~mag] == 0)
    E = host(sim.reduce(m))
    Eo = P.energy(mf)
    mean_o = mf[:, mag].mean(axis=1)
    sim.step(m, 100, w.dt)
    sim.sync()
    mo = P.run(mf, 100, w.dt)
    e_t = rel(host(m), mo)
    print(f"disk 64x64x2 ({mag.sum()} of {mag.size} cells magnetic): H_eff rel L2 {e_h:.2e}, "
          f"100 steps rel L2 {e_t:.2e}, energy {E[4]:.6e} vs {Eo[4]:.6e}")
    assert e_h < 1e-5
    assert e_t < 1e-4
    np.testing.assert_allclose(E[:5], Eo, rtol=1e-6, atol=1e-6 * abs(Eo[4]))
    np.testing.assert_allclose(E[5:], mean_o, rtol=0, atol=1e-6)
    assert np.array_equal(host(m)[:, ~mag], mf[:, ~mag])  # vacuum state untouched
    sim.close()


@pytest.mark.parametrize("mode", ["rk4", "adaptive", "adaptive_dp54"])
def test_disk_runge_kutta(gpu_lib, mode):
    w, sim, P, m, mag = disk_case(gpu_lib)
    mf = host(m)
    if mode == "rk4":
        sim.step(m, 40, w.dt, gpu_lib.MM_F_RK4)
        mo = P.run(mf, 40, w.dt, method="rk4")
    else:
        dp = mode == "adaptive_dp54"
        dt, acc, rej = sim.run_adaptive(m, 2e-12, w.dt, 1e-5, gpu_lib.MM_F_DP54 if dp else gpu_lib.MM_F_BS23)
        mo, dto, acco, rejo = P.run_adaptive(mf, 2e-12, w.dt, 1e-5, "dp54" if dp else "bs23")
        print(f"adaptive: GPU {acc}/{rej}, oracle {acco}/{rejo}")
        assert abs(acc - acco) <= max(2, 0.05 * acco)
    sim.sync()
    e = rel(host(m), mo)
    print(f"disk {mode}: rel L2 {e:.2e}")
    assert e < 1e-4
    assert np.array_equal(host(m)[:, ~mag], mf[:, ~mag])
    sim.close()


def test_vacuum_padding_is_invisible_on_gpu(gpu_lib):
    """The 13x11x3 sample alone and embedded in a 21x17x5 grid of vacuum give
    the same H_eff on its cells (FP32 rounding of different FFT sizes)."""
    rng = np.random.default_rng(9)
    n0, n1, off, d = (13, 11, 3), (21, 17, 5), (4, 3, 1), (4e-9, 5e-9, 3e-9)
    sl = (slice(None), slice(off[2], off[2] + n0[2]), slice(off[1], off[1] + n0[1]), slice(off[0], off[0] + n0[0]))
    m0 = workloads.sphere(rng, (3, n0[2], n0[1], n0[0]))
    ms0 = 8e5 * (0.8 + 0.4 * rng.random((n0[2], n0[1], n0[0])))
    m1 = workloads.sphere(rng, (3, n1[2], n1[1], n1[0]))
    m1[sl] = m0
    ms1 = np.zeros((n1[2], n1[1], n1[0]))
    ms1[sl[1:]] = ms0
    kw = dict(Ms=8e5, A=1.3e-11, Ku=3e4, u=(0.0, 0.6, 0.8), alpha=0.3, hext=(1e4, 2e4, -5e3))
    s0 = gpu_lib.Sim(n0, d, **kw)
    s0.set_ms_map(gpu(ms0))
    s1 = gpu_lib.Sim(n1, d, **kw)
    s1.set_ms_map(gpu(ms1))
    H0 = host(s0.heff(gpu(m0)))
    H1 = host(s1.heff(gpu(m1)))[sl]
    e = rel(H1, H0)
    print(f"padded vs bare H_eff: rel L2 {e:.2e}")
    assert e < 1e-6
    s0.close()
    s1.close()


def test_staircase_sphere_average_field(gpu_lib):
    R, N = 16, 34
    c = np.arange(N) + 0.5 - N / 2
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = x * x + y * y + z * z < R * R
    m = np.zeros((3, N, N, N))
    m[0] = 1.0
    sim = gpu_lib.Sim((N, N, N), (5e-9,) * 3, Ms=8e5, A=1.3e-11)
    sim.set_ms_map(gpu(np.where(inside, 8e5, 0.0)))
    Hd = host(sim.heff(gpu(m), gpu_lib.MM_T_DEMAG))
    avg = Hd[:, inside].mean(axis=1) / 8e5
    print(f"sphere R=16 ({inside.sum()} cells): average H/Ms = {avg}")
    np.testing.assert_allclose(avg[0], -1.0 / 3.0, rtol=1e-5)
    assert np.abs(avg[1:]).max() < 1e-6
    sim.close()


def test_invalid_maps_and_unsupported_calls(gpu_lib):
    import torch
    b = gpu_lib
    w, sim, P, m, mag = disk_case(gpu_lib)
    for bad in (-1.0, float("nan"), float("inf")):
        ms = workloads.disk_ms_map(w.n, w.Ms)
        ms[0, 5, 7] = bad
        with pytest.raises(b.MMError) as ei:
            sim.set_ms_map(gpu(ms))
        assert ei.value.code == b.MM_EINVAL
    sim.set_ms_map(gpu(workloads.disk_ms_map(w.n, w.Ms)))
    traj = torch.empty((2,) + tuple(m.shape), device="cuda:0")
    with pytest.raises(b.MMError) as ei:
        b.mm_forward_store(sim.ctx, m, 2, w.dt, 0, traj, torch.empty_like(traj), sim.N)
    assert ei.value.code == b.MM_EUNSUP
    sim.set_ms_map(gpu(np.full((w.n[2], w.n[1], w.n[0]), w.Ms)))  # no vacuum: allowed again
    b.mm_forward_store(sim.ctx, m, 2, w.dt, 0, traj, torch.empty_like(traj), sim.N)
    sim.sync()
    sim.close()
