"""GPU FP64 loss reduction and time-dependent external field against the
FP64 oracle, through the C ABI.

Loss: 1/2 sum (m - t)^2 reduced in FP64 on the GPU from FP32 inputs; the
oracle gets the same FP32 values, so the two agree to FP64 rounding (bar
1e-12 relative), and the gradient m - t equals the FP32 difference bit for
bit.  Field schedule (the field record of Sec. 5 with its start, decay and
stop times): trajectories across the whole profile within the trajectory
bar (1e-4 relative L2, 1e-3 of max |m| per cell), graph replays and split
calls equal to one eager call bit for bit, the device clock equal to the
FP64 sum of the steps.

Paper: Zhu, arXiv:1411.2565, eqs. (1)-(3), Sec. 3 (Euler), Sec. 5 (field
record).
"""
import numpy as np
import pytest

import oracle
from paper_1411_2565_amd import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def cellmax(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / np.abs(b).max()


def gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda:0")


def host(t):
    return t.detach().cpu().double().numpy()


@pytest.mark.parametrize("n", [(2, 1, 1), (13, 7, 3), (64, 64, 1), (128, 128, 4)])
def test_loss_matches_oracle(gpu_lib, n):
    """Ragged sizes: 6 values (less than one block), 819 (one partial
    block), 12288 (6 blocks), 196608 (96 blocks)."""
    import torch
    rng = np.random.default_rng(31)
    shape = (3, n[2], n[1], n[0])
    m = workloads.sphere(rng, shape)
    t = workloads.sphere(rng, shape)
    sim = gpu_lib.Sim(n, (5e-9,) * 3, Ms=8e5, A=1.3e-11, build_tensor=False)
    mg, tg = gpu(m), gpu(t)
    out, g = sim.loss(mg, tg, grad=True)
    L = float(out.cpu()[0])
    Lo = oracle.loss(host(mg), host(tg))
    print(f"loss {n}: GPU {L:.17e} oracle {Lo:.17e} rel {abs(L - Lo) / Lo:.1e}")
    assert abs(L - Lo) <= 1e-12 * Lo
    assert torch.equal(g, mg - tg)
    out2 = sim.loss(mg, tg)
    assert float(out2.cpu()[0]) == L  # fixed reduction order
    sim.close()


def test_loss_autograd(gpu_lib):
    import torch
    from paper_1411_2565_amd.rollout import l2_loss
    rng = np.random.default_rng(5)
    n = (24, 16, 3)
    m = gpu(workloads.sphere(rng, (3, 3, 16, 24))).requires_grad_(True)
    t = gpu(workloads.sphere(rng, (3, 3, 16, 24)))
    sim = gpu_lib.Sim(n, (5e-9,) * 3, Ms=8e5, A=1.3e-11, build_tensor=False)
    L = l2_loss(m, t, sim)
    assert L.dtype == torch.float64
    (2.0 * L).backward()
    assert torch.equal(m.grad, 2.0 * (m.detach() - t))
    sim.close()


SCHED = (3.05e-12, 6.05e-12, 9.05e-12)   # on at step 31, decaying from step 61, off from step 91


def _sched_problem():
    w = workloads.BLOCK_16x16x2
    m0, _ = workloads.inputs(w)
    args = dict(Ms=w.Ms, A=w.A, alpha=w.alpha, Ku=2e4, u=(0.0, 0.6, 0.8), hext=(4e4, -2e4, 6e4))
    return w, m0, args


def test_field_schedule_trajectory_matches_oracle(gpu_lib):
    """120 Euler steps through off, full, decay and off again, from t = 0."""
    w, m0, args = _sched_problem()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    sim.set_field_schedule(SCHED)
    sim.set_time(0.0)
    m = gpu(m0)
    sim.step(m, 120, w.dt)
    sim.sync()
    P = oracle.Problem(w.n, w.d, **args)
    mo, t_end = P.run_scheduled(host(gpu(m0)), 120, w.dt, SCHED, t0=0.0)
    e, c = rel(host(m), mo), cellmax(host(m), mo)
    print(f"scheduled field, 120 steps: rel L2 {e:.2e}, cell max {c:.2e}")
    assert e < 1e-4 and c < 1e-3
    assert sim.time() == t_end
    # the schedule matters: the constant field gives another state
    mc = P.run(host(gpu(m0)), 120, w.dt)
    assert rel(mc, mo) > 100 * e
    sim.close()


def test_field_schedule_graph_and_split_calls_equal_eager(gpu_lib):
    """Graph replays (chunks of 32 steps plus an eager remainder) and a run
    split over calls advance the device clock exactly as one eager call."""
    import torch
    w, m0, args = _sched_problem()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sim = gpu_lib.Sim(w.n, w.d, **args)
        sim.set_field_schedule(SCHED)
        ref = gpu(m0)
        sim.set_time(0.0)
        sim.step(ref, 120, w.dt)
        t_ref = sim.time()
        for rep in range(2):
            g = gpu(m0)
            sim.set_time(0.0)
            sim.step(g, 120, w.dt, gpu_lib.MM_F_GRAPH)
            junk = torch.randn(1000, device="cuda:0").sum()
            s.synchronize()
            assert torch.equal(g, ref), rep
            assert sim.time() == t_ref
            assert torch.isfinite(junk)
        sp = gpu(m0)
        sim.set_time(0.0)
        sim.step(sp, 45, w.dt)
        sim.step(sp, 33, w.dt, gpu_lib.MM_F_GRAPH)
        sim.step(sp, 42, w.dt)
        s.synchronize()
        assert torch.equal(sp, ref)
        sim.sync()
        sim.close()


def test_field_schedule_heff_and_energy_at_clock_time(gpu_lib):
    """mm_compute_heff and mm_reduce see the field at the device clock's
    time: inside the decay, before the start and after the stop."""
    w, m0, args = _sched_problem()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    sim.set_field_schedule(SCHED)
    P = oracle.Problem(w.n, w.d, **args)
    mf = host(gpu(m0))
    h = np.asarray(args["hext"])
    for t in (1e-12, 4e-12, 7.3e-12, 9.05e-12, 2e-11):
        sim.set_time(t)
        s = oracle.field_scale(t, SCHED)
        Hz = host(sim.heff(gpu(m0), gpu_lib.MM_T_ZEEMAN))
        ref = np.broadcast_to((s * h).reshape(3, 1, 1, 1), Hz.shape)
        assert np.abs(Hz - ref).max() <= 1e-6 * np.abs(h).max(), t
        E = sim.reduce(gpu(m0)).cpu().numpy()
        Q = oracle.Problem(w.n, w.d, **dict(args, hext=tuple(s * h)))
        Eo = Q.energy(mf)
        assert abs(E[3] - Eo[3]) <= 1e-6 * abs(P.energy(mf)[3]), (t, E[3], Eo[3])
    sim.close()


def test_field_schedule_rejections(gpu_lib):
    import torch
    b = gpu_lib
    w, m0, args = _sched_problem()
    sim = b.Sim(w.n, w.d, **args)
    with pytest.raises(b.MMError) as ei:
        sim.set_field_schedule((2e-12, 1e-12, 3e-12))
    assert ei.value.code == b.MM_EINVAL
    sim.set_field_schedule(SCHED)
    m = gpu(m0)
    for call in (lambda: sim.step(m, 2, w.dt, b.MM_F_RK4),
                 lambda: sim.run_adaptive(m, 1e-12, 1e-14, 1e-5, b.MM_F_BS23)):
        with pytest.raises(b.MMError) as ei:
            call()
        assert ei.value.code == b.MM_EUNSUP
    traj = torch.empty((2, 3 * w.N), dtype=torch.float32, device="cuda:0")
    with pytest.raises(b.MMError) as ei:
        b.mm_forward_store(sim.ctx, m, 2, w.dt, 0, traj, traj.clone(), w.N)
    assert ei.value.code == b.MM_EUNSUP
    sim.set_field_schedule(None)
    sim.step(m, 2, w.dt, b.MM_F_RK4)  # constant field again: accepted
    sim.sync()
    sim.close()
