"""The fused x-inverse + update pass against the two-kernel step, through the
C ABI.

Euler steps run the x-inverse transform, the local terms and the update as
one pass (fusion level 1: H_demag stays on chip), and by default (level 2)
that pass also runs the next step's x-forward transform of the state it
writes, so the next step skips its own; at level 0 they run as the
x-inverse kernel (H_demag to device memory) and the update kernel.  All
levels evaluate the same transforms and the same update arithmetic, so
every state after n steps must agree bit for bit: ragged y tiles, z-planes
whose tile count is odd, every x transform length up to 256, nx a multiple
of 4 (4 cells per thread) or not (odd and even nx, one cell at a time),
anisotropy, a uniform and a mapped external field, the time-dependent field,
graph replays, and batches (every group of samples with one padded x length
and update width as one launch).  Samples the fused pass does not cover
(padded x length below 8) take the two kernels either way.

Paper: Zhu, arXiv:1411.2565, Sec. 3 (demag field, local terms, Euler step
of eq. (3)).
"""
import numpy as np
import pytest

from paper_1411_2565_amd import workloads

pytestmark = pytest.mark.gpu


def gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda:0")


def run(gpu_lib, n, steps, level, hmap=None, sched=None, flags=0, seed=5, timed_steps=1):
    rng = np.random.default_rng(seed)
    sim = gpu_lib.Sim(n, (4e-9, 5e-9, 3e-9), Ms=8.0e5, A=1.3e-11, Ku=5e4, u=(0.6, 0.0, 0.8), alpha=0.3,
                      hext=(2e4, -1e4, 3e4))
    gpu_lib.mm_set_fusion(sim.ctx, level)
    hm = None  # the context keeps the map's pointer: hold the tensor until the end
    if hmap is not None:
        hm = gpu(hmap)
        gpu_lib.mm_set_hext_map(sim.ctx, hm, sim.N)
    if sched is not None:
        sim.set_field_schedule(sched)
        sim.set_time(0.0)
    m = gpu(workloads.sphere(rng, (3, n[2], n[1], n[0])))
    sim.step(m, steps, 2e-14, flags)
    sim.sync()
    t = sim.time() if sched is not None else None
    times = None
    gpu_lib.mm_kernel_timing(sim.ctx, True)
    sim.step(m, timed_steps, 2e-14, flags)
    times = gpu_lib.mm_kernel_times(sim.ctx)
    gpu_lib.mm_kernel_timing(sim.ctx, False)
    sim.sync()
    sim.close()
    del hm
    return m, t, times


# (nx, ny, nz): x transform lengths 4..256, ragged y tiles (ny % 8 != 0),
# odd tile counts and z-plane counts that break the paired block order; nx
# not a multiple of 4, odd or even; single-cell y and z axes
SIZES = [(4, 3, 2), (8, 8, 1), (16, 16, 2), (20, 12, 3), (32, 32, 4), (64, 24, 5), (100, 9, 2),
         (128, 128, 4), (256, 40, 3), (256, 256, 32), (3, 4, 2), (7, 5, 3), (18, 10, 2), (13, 9, 2),
         (66, 17, 3), (255, 20, 2), (6, 12, 140), (16, 1, 4), (9, 1, 1), (40, 7, 1)]


@pytest.mark.parametrize("n", SIZES, ids=lambda n: "x".join(map(str, n)))
def test_fused_step_equals_two_kernel_step(gpu_lib, n):
    import torch
    steps = 3 if n == (256, 256, 32) else 7
    c, _, tc = run(gpu_lib, n, steps, 2, timed_steps=3)
    a, _, ta = run(gpu_lib, n, steps, 1, timed_steps=3)
    b, _, tb = run(gpu_lib, n, steps, 0, timed_steps=3)
    assert torch.isfinite(a).all()
    assert torch.equal(a, b), f"{n}: level 1 vs 0 max |diff| {(a - b).abs().max().item():.3e}"
    assert torch.equal(c, b), f"{n}: level 2 vs 0 max |diff| {(c - b).abs().max().item():.3e}"
    # which passes ran over a 3-step call: level 2 chains the x-forward of
    # steps 2 and 3 into the fused passes of steps 1 and 2
    assert tc["xfwd"][1] == 1 and tc["xinv_local_xfwd"][1] == 2 and tc["xinv_local"][1] == 1
    assert tc["xinv"][1] == 0 and tc["local"][1] == 0
    assert ta["xfwd"][1] == 3 and ta["xinv_local"][1] == 3 and ta["xinv_local_xfwd"][1] == 0
    assert ta["xinv"][1] == 0 and ta["local"][1] == 0
    assert tb["xinv_local"][1] == 0 and tb["xinv_local_xfwd"][1] == 0 and tb["xinv"][1] == 3
    assert tb["local"][1] == 3


def test_fusion_level_is_checked(gpu_lib):
    sim = gpu_lib.Sim((8, 8, 2), (5e-9,) * 3, Ms=8e5, A=1.3e-11)
    for bad in (-1, 3):
        with pytest.raises(gpu_lib.MMError):
            gpu_lib.mm_set_fusion(sim.ctx, bad)
    sim.close()


def test_unfusable_sample_takes_two_kernels(gpu_lib):
    import torch
    n = (2, 6, 3)  # padded x length 4
    a, _, ta = run(gpu_lib, n, 5, 2)
    b, _, _ = run(gpu_lib, n, 5, 0)
    assert torch.equal(a, b)
    assert ta["xinv_local"][1] == 0 and ta["xinv"][1] == 1 and ta["local"][1] == 1


@pytest.mark.parametrize("n", [(32, 20, 3), (128, 64, 4)], ids=lambda n: "x".join(map(str, n)))
def test_fused_step_with_field_map_and_schedule(gpu_lib, n):
    import torch
    rng = np.random.default_rng(8)
    hmap = 4e4 * rng.standard_normal((3, n[2], n[1], n[0]))
    sched = (3e-14, 9e-14, 1.5e-13)  # on after 2 steps, decays from step 5, off after step 8
    a, ta, _ = run(gpu_lib, n, 10, 2, hmap=hmap, sched=sched)
    b, tb, _ = run(gpu_lib, n, 10, 0, hmap=hmap, sched=sched)
    assert torch.equal(a, b)
    assert ta == tb and abs(ta - 10 * 2e-14) < 1e-25


@pytest.mark.parametrize("level", [1, 2])
def test_fused_graph_replays_equal_eager_two_kernel_steps(gpu_lib, level):
    """Graph replays (capture needs a stream of its own) of fused steps,
    three replays with eager work and a synchronisation between them, each
    equal to the eager two-kernel steps."""
    import torch
    n = (64, 48, 4)
    rng = np.random.default_rng(9)
    m0 = workloads.sphere(rng, (3, n[2], n[1], n[0]))
    s = torch.cuda.Stream()
    kw = dict(Ms=8.0e5, A=1.3e-11, Ku=5e4, alpha=0.3, hext=(2e4, 0.0, 1e4))
    with torch.cuda.stream(s):
        fused = gpu_lib.Sim(n, (5e-9,) * 3, **kw)    # fused steps in one captured graph
        split = gpu_lib.Sim(n, (5e-9,) * 3, **kw)    # eager two-kernel steps
        gpu_lib.mm_set_fusion(fused.ctx, level)
        gpu_lib.mm_set_fusion(split.ctx, 0)
        graph, eager = gpu(m0), gpu(m0)
        for rep in range(3):
            fused.step(graph, 20, 2e-14, gpu_lib.MM_F_GRAPH)
            split.step(eager, 20, 2e-14)
            fused.sync()
            split.sync()
            assert torch.equal(graph, eager), rep
        fused.close()
        split.close()


def test_batch_fused_equals_two_kernel_steps(gpu_lib):
    """The 64 films (groups by padded x length 256 / 512 and nx % 4): 20
    steps with the fused launches, eager and replaying 32-step graphs on a
    stream of its own, against 20 eager two-kernel steps, bit for bit."""
    import torch
    films = workloads.batch_films(count=64, seed=0)
    w0 = films[0][0]
    hs = [tuple(h) for (_, _, h) in films]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B = gpu_lib.Batch([w.n for (w, _, _) in films], w0.d, Ms=w0.Ms, A=w0.A, alpha=w0.alpha, hext=hs)
        a = B.pack([m0 for (_, m0, _) in films])
        b, c = a.clone(), a.clone()
        B.set_fusion(True)
        B.step(a, 20, w0.dt)
        B.step(c, 64, w0.dt, gpu_lib.MM_F_GRAPH)
        B.set_fusion(False)
        B.step(b, 20, w0.dt)
        d = b.clone()
        B.step(d, 44, w0.dt)
        B.sync()
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)
        assert torch.equal(c, d)
        B.close()


@pytest.mark.parametrize("vacuum", [False, True], ids=["ms-map", "vacuum"])
@pytest.mark.parametrize("n", [(32, 20, 3), (30, 17, 2)], ids=lambda n: "x".join(map(str, n)))
def test_fused_step_with_ms_map(gpu_lib, n, vacuum):
    """An Ms map (with vacuum cells: a disk) takes the mapped fused pass:
    equal bit for bit to the two-kernel step at every fusion level."""
    import torch
    rng = np.random.default_rng(12)
    nx, ny, nz = n
    ms = 8e5 * (1.0 + 0.2 * rng.random((nz, ny, nx)))
    if vacuum:
        yy, xx = np.mgrid[0:ny, 0:nx]
        ms[:, (xx - nx / 2 + 0.5) ** 2 + (yy - ny / 2 + 0.5) ** 2 > (0.45 * min(nx, ny)) ** 2] = 0.0
    m0 = workloads.sphere(rng, (3, nz, ny, nx))
    out = []
    for level in (0, 1, 2):
        sim = gpu_lib.Sim(n, (4e-9, 4e-9, 3e-9), Ms=8e5, A=1.3e-11, Ku=2e4, u=(0.0, 0.0, 1.0), alpha=0.2,
                          hext=(1e4, 2e4, -1e4))
        msg = gpu(ms)
        gpu_lib.mm_set_ms_map(sim.ctx, msg, sim.N)
        gpu_lib.mm_set_fusion(sim.ctx, level)
        m = gpu(m0)
        gpu_lib.mm_kernel_timing(sim.ctx, True)
        sim.step(m, 6, 2e-14)
        t = gpu_lib.mm_kernel_times(sim.ctx)
        gpu_lib.mm_kernel_timing(sim.ctx, False)
        sim.sync()
        out.append((m, t))
        sim.close()
        del msg
    assert torch.isfinite(out[0][0]).all()
    assert torch.equal(out[1][0], out[0][0]) and torch.equal(out[2][0], out[0][0])
    # with a map, level 2 runs as level 1 (the chained x-forward needs a uniform Ms)
    assert out[1][1]["xinv_local"][1] == 6 and out[2][1]["xinv_local"][1] == 6
    assert out[2][1]["xinv_local_xfwd"][1] == 0 and out[0][1]["local"][1] == 6


def test_fused_forward_store_and_adjoint(gpu_lib):
    """mm_forward_store (states and H_demag of every step) and the adjoint
    segment with the fused x-inverse passes equal the two-kernel forms bit
    for bit, with Ms and field maps."""
    import torch
    n = (24, 20, 4)
    rng = np.random.default_rng(13)
    N = n[0] * n[1] * n[2]
    ms = 8e5 * (1.0 + 0.1 * rng.random((n[2], n[1], n[0])))
    hm = 2e4 * rng.standard_normal((3, n[2], n[1], n[0]))
    m0 = workloads.sphere(rng, (3, n[2], n[1], n[0]))
    lam0 = rng.standard_normal((3, N))
    res = []
    for level in (0, 1):
        sim = gpu_lib.Sim(n, (5e-9,) * 3, Ms=8e5, A=1.3e-11, alpha=0.1)
        msg, hmg = gpu(ms), gpu(hm)
        gpu_lib.mm_set_ms_map(sim.ctx, msg, N)
        gpu_lib.mm_set_hext_map(sim.ctx, hmg, N)
        gpu_lib.mm_set_fusion(sim.ctx, level)
        m = gpu(m0)
        mt = torch.empty((7, 3 * N), dtype=torch.float32, device="cuda:0")
        ht = torch.empty_like(mt)
        gpu_lib.mm_forward_store(sim.ctx, m, 7, 2e-14, 0, mt, ht, N)
        lam = gpu(lam0)
        g_h = torch.zeros_like(hmg)
        g_ms = torch.zeros_like(msg)
        gpu_lib.mm_adjoint_segment(sim.ctx, mt, ht, 7, lam, g_h, g_ms, 2e-14, 0, N)
        sim.sync()
        res.append((m, mt, ht, lam, g_h, g_ms))
        sim.close()
        del msg, hmg
    for a, b in zip(*res):
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)
