"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: H_eff (and each term alone) within 1e-5 relative L2, the state
after 100 Euler steps within 1e-4 relative L2; beside each L2 bar, the
largest per-cell error relative to the largest value (1e-4 for fields,
1e-3 for states), so that a few wrong cells cannot hide in the norm; FP64
reductions within 1e-6 relative (FP32 inputs, FP64 accumulation); the GPU's
FP64 tensor table within 1e-10 of max|N| of the oracle's independently built
table.

Paper: Zhu, arXiv:1411.2565, Sec. 2 eqs. (1)-(3), Sec. 3 (FFT demag with
zero padding, six-neighbour exchange, Euler).
"""
import numpy as np
import pytest

import oracle
from paper_1411_2565_amd import workloads
from tests.closed_forms import aharoni

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def cellmax(a, b):
    """largest per-cell error over the largest reference value"""
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / np.abs(b).max()


FIELD_L2, FIELD_CELL = 1e-5, 1e-4
STATE_L2, STATE_CELL = 1e-4, 1e-3


def check_field(label, H, ref):
    e, c = rel(H, ref), cellmax(H, ref)
    print(f"{label}: rel L2 {e:.2e}, cell max {c:.2e}")
    assert e < FIELD_L2 and c < FIELD_CELL, (e, c)


def check_state(label, m, ref):
    e, c = rel(m, ref), cellmax(m, ref)
    print(f"{label}: rel L2 {e:.2e}, cell max {c:.2e}")
    assert e < STATE_L2 and c < STATE_CELL, (e, c)


def gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda:0")


def host(t):
    return t.detach().cpu().double().numpy()


def sphere(shape, seed):
    rng = np.random.default_rng(seed)
    return workloads.sphere(rng, shape)


GEOMS = [
    ((16, 16, 2), (5e-9,) * 3),            # block 16x16x2
    ((13, 7, 3), (5e-9,) * 3),             # ragged, non power of two
    ((33, 17, 1), (4e-9, 4e-9, 3e-9)),     # thin film, odd sizes
    ((8, 1, 5), (5e-9, 3e-9, 2e-9)),       # single-cell y axis
    ((2, 3, 4), (5e-9,) * 3),              # smallest x
    ((64, 20, 2), (4e-9, 4e-9, 3e-9)),     # several FFT tiles along x
    ((40, 24, 6), (3e-9, 4e-9, 5e-9)),     # anisotropic cells
    ((2, 512, 2), (5e-9, 2e-9, 5e-9)),     # longest y transform (1024 points)
    ((3, 2, 512), (5e-9, 5e-9, 1e-9)),     # longest z transform (1024 points)
    # 64-point z transforms (the digit-split z pass): a column tile wider
    # than Py, a ragged nz < Pz/2, and nz = Pz/2 exactly
    ((5, 3, 20), (5e-9, 4e-9, 3e-9)),      # Py = 8: half the tile's columns beyond Py
    ((6, 40, 17), (4e-9,) * 3),            # Py = 128, nz = 17
    ((2, 9, 32), (3e-9, 5e-9, 2e-9)),      # Py = 32, nz = 32
]


@pytest.mark.parametrize("n,d", GEOMS[:1] + GEOMS[5:])
def test_tensor_table_matches_oracle(gpu_lib, n, d):
    sim = gpu_lib.Sim(n, d, Ms=8e5, A=1.3e-11, build_tensor=False)
    tab = sim.tensor_table().cpu().numpy()
    ref = oracle.tensor_table(n, d)
    err = np.abs(tab - ref).max() / np.abs(ref).max()
    print(f"tensor table {n}: max err / max|N| = {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("n,d", GEOMS)
def test_demag_matches_direct_sum(gpu_lib, n, d):
    shape = (3, n[2], n[1], n[0])
    m = sphere(shape, 0)
    sim = gpu_lib.Sim(n, d, Ms=8e5, A=1.3e-11)
    H = host(sim.heff(gpu(m), gpu_lib.MM_T_DEMAG))
    Ho = oracle.Problem(n, d, Ms=8e5).heff(host(gpu(m)), oracle.T_DEMAG)
    check_field(f"demag {n}", H, Ho)


def test_demag_with_ms_map(gpu_lib):
    n, d = (24, 12, 3), (4e-9, 4e-9, 3e-9)
    shape = (3, 3, 12, 24)
    m = sphere(shape, 2)
    rng = np.random.default_rng(3)
    Ms = 8e5 * (0.5 + rng.random(shape[1:]))
    sim = gpu_lib.Sim(n, d, Ms=8e5, A=1.3e-11)
    sim.set_ms_map(gpu(Ms))
    H = host(sim.heff(gpu(m), gpu_lib.MM_T_DEMAG | gpu_lib.MM_T_EXCH))
    Ho = oracle.Problem(n, d, Ms=host(gpu(Ms))).heff(host(gpu(m)), oracle.T_DEMAG | oracle.T_EXCH)
    check_field("demag + exchange with an Ms map", H, Ho)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_uniform_body_average_is_aharoni(gpu_lib, axis):
    """Whole-sample pin through the GPU path: the mean demag field of a
    uniformly magnetised block is -D_body Ms (Aharoni's prism factors)."""
    n, d = (16, 16, 2), (5e-9,) * 3
    m = np.zeros((3, 2, 16, 16))
    m[axis] = 1.0
    sim = gpu_lib.Sim(n, d, Ms=8e5, A=1.3e-11)
    H = host(sim.heff(gpu(m), gpu_lib.MM_T_DEMAG)).mean(axis=(1, 2, 3))
    D = aharoni(80e-9, 80e-9, 10e-9)[axis]
    assert abs(H[axis] + D * 8e5) < 2e-6 * 8e5
    assert np.abs(np.delete(H, axis)).max() < 2e-6 * 8e5


def _block16(**kw):
    w = workloads.BLOCK_16x16x2
    m0, h = workloads.inputs(w)
    args = dict(Ms=w.Ms, A=w.A, alpha=w.alpha)
    args.update(kw)
    return w, m0, args


@pytest.mark.parametrize("terms", [1, 2, 4, 8, 15])
def test_heff_terms_block16(gpu_lib, terms):
    w, m0, args = _block16(Ku=3e4, u=(0.48, 0.6, 0.64), hext=(1e4, -2e4, 5e3))
    sim = gpu_lib.Sim(w.n, w.d, **args)
    mf = host(gpu(m0))
    H = host(sim.heff(gpu(m0), terms))
    P = oracle.Problem(w.n, w.d, **args)
    Ho = P.heff(mf, terms)
    check_field(f"H_eff terms={terms}", H, Ho)


def test_trajectory_block16_100_steps(gpu_lib):
    import torch
    w, m0, args = _block16()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    m = gpu(m0)
    sim.step(m, w.nsteps, w.dt)
    sim.sync()
    mo = oracle.Problem(w.n, w.d, **args).run(host(gpu(m0)), w.nsteps, w.dt)
    check_state("trajectory 16x16x2, 100 steps", host(m), mo)
    assert torch.isfinite(m).all()


def test_trajectory_block64x64x8_100_steps(gpu_lib):
    """Standalone 64x64x8 sample with the large block's material (seed 1):
    100 steps against the oracle's full direct-sum trajectory."""
    w = workloads.BLOCK_64x64x8
    m0, _ = workloads.inputs(w)
    sim = gpu_lib.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    m = gpu(m0)
    mf = host(m)
    sim.step(m, w.nsteps, w.dt)
    sim.sync()
    mo = oracle.Problem(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha).run(mf, w.nsteps, w.dt)
    check_state("trajectory 64x64x8, 100 steps", host(m), mo)
    sim.close()


def test_trajectory_split_calls_equal_one_call(gpu_lib):
    """Odd/even step counts go through the internal double buffer: 37 steps
    in one call must equal 20 + 17 steps bit for bit."""
    import torch
    w, m0, args = _block16()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    a, b = gpu(m0), gpu(m0)
    sim.step(a, 37, w.dt)
    sim.step(b, 20, w.dt)
    sim.step(b, 17, w.dt)
    sim.sync()
    assert torch.equal(a, b)
    c = gpu(m0)
    sim.step(c, 0, w.dt)
    sim.sync()
    assert torch.equal(c, gpu(m0))


def test_block_steps_are_deterministic(gpu_lib):
    """The 256x256x32 block, 50 steps from the same state twice: equal bit
    for bit.  The x passes and the y-inverse order their FFT exchanges
    within each wavefront instead of by block barriers; a missing ordering
    would show up as run-to-run differences here, at the full grid."""
    import torch
    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    sim = gpu_lib.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    a, b = gpu(m0), gpu(m0)
    sim.step(a, 50, w.dt)
    sim.step(b, 50, w.dt)
    h1 = sim.heff(a)
    h2 = sim.heff(a)
    sim.sync()
    assert torch.equal(a, b)
    assert torch.equal(h1, h2)
    sim.close()


def test_norm_identity_without_renorm(gpu_lib):
    w, m0, args = _block16()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    m = gpu(m0)
    H = host(sim.heff(m))
    mf = host(m)
    f = oracle.Problem(w.n, w.d, **args).llg_rhs(mf, H)
    sim.step(m, 1, w.dt, gpu_lib.MM_F_NO_RENORM)
    sim.sync()
    n2 = np.sum(host(m) ** 2, axis=0)
    expect = np.sum(mf ** 2, axis=0) + w.dt ** 2 * np.sum(f ** 2, axis=0)
    assert np.abs(n2 - expect).max() < 5e-6
    assert np.abs(n2 - 1).max() > 1e-3


def test_reduce_energy_block16(gpu_lib):
    w, m0, args = _block16(Ku=3e4, u=(0.0, 0.6, 0.8), hext=(1e4, -2e4, 5e3))
    sim = gpu_lib.Sim(w.n, w.d, **args)
    m = gpu(m0)
    out = sim.reduce(m).cpu().numpy()
    mf = host(m)
    E = oracle.Problem(w.n, w.d, **args).energy(mf)
    for q in range(5):
        assert abs(out[q] - E[q]) < 1e-6 * abs(E[q]) + 1e-30, (q, out[q], E[q])
    np.testing.assert_allclose(out[5:], mf.mean(axis=(1, 2, 3)), rtol=1e-9, atol=1e-12)


def test_reduce_block_256x256x32_local_terms(gpu_lib):
    """FP64 reductions at the headline size: the exchange, anisotropy and
    Zeeman energies and <m> of the 256x256x32 block (after 10 steps, with an
    anisotropy axis and a field added) against the oracle.  Both sides add
    the same FP32 inputs in FP64, in different orders.  (The demag energy
    needs the O(N^2) direct sum and is checked at 16x16x2 above.)"""
    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    args = dict(Ms=w.Ms, A=w.A, alpha=w.alpha, Ku=5e3, u=(0.0, 0.6, 0.8), hext=(1e4, -2e4, 5e3))
    sim = gpu_lib.Sim(w.n, w.d, **args)
    m = gpu(m0)
    sim.step(m, 10, w.dt)
    out = sim.reduce(m).cpu().numpy()
    mf = host(m)
    P = oracle.Problem(w.n, w.d, terms=oracle.T_EXCH | oracle.T_ANIS | oracle.T_ZEEMAN, **args)
    E = P.energy(mf)
    for q in (0, 2, 3):
        print(f"block 256x256x32 energy term {q}: GPU {out[q]:.15e} oracle {E[q]:.15e}")
        assert abs(out[q] - E[q]) <= 1e-10 * abs(E[q]), q
    np.testing.assert_allclose(out[5:], mf.mean(axis=(1, 2, 3)), rtol=1e-10, atol=1e-13)
    sim.close()


def test_energy_decreases_on_gpu(gpu_lib):
    w, m0, args = _block16()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    m = gpu(m0)
    E = [sim.reduce(m).cpu().numpy()[4]]
    for _ in range(20):
        sim.step(m, 1, 2e-14)
        E.append(sim.reduce(m).cpu().numpy()[4])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-6 * np.abs(E[:-1]))
    assert E[-1] < E[0]


def test_film_256x64_heff_and_short_trajectory(gpu_lib):
    w = workloads.FILM_256x64x1
    m0, h = workloads.inputs(w)
    args = dict(Ms=w.Ms, A=w.A, Ku=w.Ku, u=w.u, alpha=w.alpha, hext=tuple(h))
    sim = gpu_lib.Sim(w.n, w.d, **args)
    mf = host(gpu(m0))
    P = oracle.Problem(w.n, w.d, **args)
    for t in (2, 15):
        check_field(f"film 256x64x1 terms={t}", host(sim.heff(gpu(m0), t)), P.heff(mf, t))
    m = gpu(m0)
    sim.step(m, 100, w.dt)
    sim.sync()
    check_state("film 256x64x1 100 steps", host(m), P.run(mf, 100, w.dt))


def test_block_256x256x32_sampled_observers(gpu_lib):
    """Full-size block in the benchmark's launch configuration: H_demag and
    H_eff at 1024 sampled cells against the oracle's direct sum over all
    2.1M sources."""
    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    sim = gpu_lib.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    m = gpu(m0)
    Hd = host(sim.heff(m, gpu_lib.MM_T_DEMAG)).reshape(3, -1)
    rng = np.random.default_rng(123)
    N = w.N
    obs = np.concatenate([[0, N - 1, 255, N - 256], rng.choice(N, 1020, replace=False)])
    mf = host(m)
    P = oracle.Problem(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    Ho = P.demag_observers(mf, obs)
    check_field("block 256x256x32 sampled demag", Hd[:, obs], Ho)


def test_block_256x256x32_sampled_step(gpu_lib):
    """The benchmark's launch configuration (one eager mm_step_llg of the
    256x256x32 block): the step increment m1 - m0 at 512 sampled cells
    against the oracle's full Euler step there (direct-sum demag over all
    sources, exchange, LLG, renormalisation)."""
    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    sim = gpu_lib.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    m = gpu(m0)
    mf = host(m)
    sim.step(m, 1, w.dt)
    sim.sync()
    rng = np.random.default_rng(321)
    N = w.N
    obs = np.unique(np.concatenate([[0, 255, N - 256, N - 1], rng.choice(N, 512, replace=False)]))
    P = oracle.Problem(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    m1o = P.step_cells(mf, obs, w.dt)
    m0s = mf.reshape(3, -1)[:, obs]
    check_field(f"block 256x256x32 one step at {obs.size} cells (increment)",
                host(m).reshape(3, -1)[:, obs] - m0s, m1o - m0s)
    sim.close()


def test_invalid_arguments(gpu_lib):
    import torch
    b = gpu_lib
    with pytest.raises(b.MMError) as ei:
        b.mm_create((1, 4, 4), (5e-9,) * 3)
    assert ei.value.code == b.MM_EINVAL
    ctx = b.mm_create((8, 8, 2), (5e-9,) * 3)
    m = torch.zeros((3, 2, 8, 8), device="cuda:0")
    with pytest.raises(b.MMError) as ei:
        b.mm_step_llg(ctx, m, 1, 1e-13, 0, 128)
    assert ei.value.code == b.MM_ESTATE
    ws = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(b.MMError) as ei:
        b.mm_set_workspace(ctx, ws)
    assert ei.value.code in (b.MM_ENOMEM, b.MM_EINVAL)
    b.mm_destroy(ctx)
    sim = b.Sim((8, 8, 2), (5e-9,) * 3, Ms=8e5, A=1.3e-11)
    with pytest.raises(b.MMError) as ei:
        b.mm_step_llg(sim.ctx, m, 1, -1e-13, 0, 128)
    assert ei.value.code == b.MM_EINVAL
    with pytest.raises(b.MMError) as ei:
        b.mm_set_material(sim.ctx, Ms=-1, A=1e-11)
    assert ei.value.code == b.MM_EINVAL


def test_zero_and_odd_step_counts(gpu_lib):
    """nsteps = 0 leaves the state as it is, eager and with MM_F_GRAPH;
    nsteps < 0 is rejected; odd counts with MM_F_GRAPH (a captured even chunk
    and an eager tail, or no chunk at all) equal eager stepping bit for bit."""
    import torch
    w, m0, args = _block16()
    s = torch.cuda.Stream()  # graph capture needs a stream of its own
    with torch.cuda.stream(s):
        sim = gpu_lib.Sim(w.n, w.d, **args)
        m = gpu(m0)
        ref = m.clone()
        for flags in (0, gpu_lib.MM_F_GRAPH):
            sim.step(m, 0, w.dt, flags)
            sim.sync()
            assert torch.equal(m, ref)
        with pytest.raises(gpu_lib.MMError) as ei:
            gpu_lib.mm_step_llg(sim.ctx, m, -1, w.dt, 0, sim.N)
        assert ei.value.code == gpu_lib.MM_EINVAL
        for n in (1, 3, 35):
            a, b = gpu(m0), gpu(m0)
            sim.step(a, n, w.dt)
            sim.step(b, n, w.dt, gpu_lib.MM_F_GRAPH)
            sim.sync()
            assert torch.equal(a, b), n
        sim.close()


def test_nonfinite_state_is_reported(gpu_lib):
    import torch
    b = gpu_lib
    sim = b.Sim((8, 8, 2), (5e-9,) * 3, Ms=8e5, A=1.3e-11)
    m = gpu(sphere((3, 2, 8, 8), 4))
    m[0, 1, 3, 3] = float("nan")
    sim.step(m, 2, 1e-13)
    with pytest.raises(b.MMError) as ei:
        sim.sync()
    assert ei.value.code == b.MM_ENONFINITE
    sim.sync()  # flag cleared once reported


def test_graph_replay_matches_eager(gpu_lib):
    """Steps replayed from captured HIP graphs equal the eager steps bit for
    bit, over several replays with other eager work and synchronisations in
    between (the state pointer is the same buffer each time)."""
    import torch
    w, m0, args = _block16(hext=(2e4, 0.0, 1e4))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sim = gpu_lib.Sim(w.n, w.d, **args)
        eager = gpu(m0)
        graph = gpu(m0)
        for rep in range(3):
            sim.step(eager, 70, w.dt)
            sim.step(graph, 70, w.dt, gpu_lib.MM_F_GRAPH)
            junk = torch.randn(1000, device="cuda:0").sum()  # unrelated eager work
            s.synchronize()
            assert torch.equal(eager, graph), rep
            assert torch.isfinite(junk)
        sim.sync()


@pytest.mark.parametrize("n,d,seed", [((16, 16, 2), (5e-9,) * 3, 0), ((64, 64, 8), (5e-9,) * 3, 1)])
def test_compensated_multiply_error_vs_oracle(gpu_lib, n, d, seed):
    """Precision form: FP32 FFTs with a compensated (Dot2) spectral multiply.
    Reports the FP64-oracle error of H_demag and H_eff for plain and
    compensated evaluation; both meet the 1e-5 bar and the compensated one
    is not worse than plain by more than rounding noise."""
    import torch
    shape = (3, n[2], n[1], n[0])
    m = host(gpu(sphere(shape, seed)))
    sim = gpu_lib.Sim(n, d, Ms=8.6e5, A=1.3e-11, alpha=0.1)
    P = oracle.Problem(n, d, Ms=8.6e5, A=1.3e-11, alpha=0.1)
    refs = {t: P.heff(m, t) for t in (2, 15)}
    errs = {}
    for comp in (0, 1):
        gpu_lib.mm_set_compensated(sim.ctx, comp)
        for t in (2, 15):
            errs[(comp, t)] = rel(host(sim.heff(gpu(m), t)), refs[t])
    gpu_lib.mm_set_compensated(sim.ctx, 0)
    print(f"precision {n}: H_demag plain {errs[(0, 2)]:.3e} compensated {errs[(1, 2)]:.3e}; "
          f"H_eff plain {errs[(0, 15)]:.3e} compensated {errs[(1, 15)]:.3e}")
    for v in errs.values():
        assert v < 1e-5
    assert errs[(1, 2)] < 1.5 * errs[(0, 2)]


def test_compensated_dot_is_twice_the_working_precision(gpu_lib):
    """The compensated multiply's three-term dot product (Dot2, Ogita, Rump
    and Oishi 2005) against the exact rational value of the same float
    inputs: within its published bound |res - s| <= u |s| + gamma_3^2
    sum |k_i x_i| (u = 2^-24, gamma_3 = 3u / (1 - 3u)) on every triple, as if
    evaluated in twice the working precision and rounded once; the plain
    form's error grows with the condition number (median above 30 u where it
    exceeds 1e4).  An fma contracted into the two-sum would count each
    product's rounding twice and break the bound.  Inputs with heavy
    cancellation, since the full field pipeline cannot show the multiply's
    own error (the FP32 transforms and tensor spectrum carry errors of the
    same size)."""
    import torch
    from tests.dot2_check import U, cancelling_triples, against_bound
    n = 4096 + 77  # a ragged last block
    trip = cancelling_triples(n, 3)
    sim = gpu_lib.Sim((8, 8, 2), (5e-9,) * 3, Ms=8.6e5, A=1.3e-11, alpha=0.1)
    lib = gpu_lib.load()
    assert lib.mm_diag_dot3(sim.ctx, None, None, -1) == gpu_lib.MM_EINVAL
    assert lib.mm_diag_dot3(sim.ctx, None, None, 0) == gpu_lib.MM_OK
    inp = torch.tensor(trip.reshape(-1), dtype=torch.float32, device="cuda:0")
    out = torch.empty(2 * n, dtype=torch.float32, device="cuda:0")
    gpu_lib.mm_diag_dot3(sim.ctx, inp, out, n)
    res = out.cpu().numpy().reshape(n, 2).astype(np.float64)
    worst, conds, plain_rel = against_bound(trip, res[:, 1], res[:, 0])
    u = U
    hi = conds > 1e4
    print(f"Dot2 diagnostic: {n} triples, condition numbers {conds.min():.1e} .. {conds.max():.1e}; "
          f"compensated error / bound max {worst:.3f}; plain relative error median {np.median(plain_rel[hi]):.2e} "
          f"(max {plain_rel.max():.2e}) over {hi.sum()} triples with condition > 1e4")
    assert worst <= 1.0
    assert hi.sum() > n // 4
    assert np.median(plain_rel[hi]) > 30 * u
    sim.close()


def test_compensated_trajectory_block16(gpu_lib):
    import torch
    w, m0, args = _block16()
    sim = gpu_lib.Sim(w.n, w.d, **args)
    mo = oracle.Problem(w.n, w.d, **args).run(host(gpu(m0)), w.nsteps, w.dt)
    out = {}
    for flags in (0, gpu_lib.MM_F_COMPENSATED):
        m = gpu(m0)
        sim.step(m, w.nsteps, w.dt, flags)
        sim.sync()
        out[flags] = rel(host(m), mo)
    print(f"trajectory 16x16x2 100 steps: plain {out[0]:.3e} compensated {out[gpu_lib.MM_F_COMPENSATED]:.3e}")
    assert max(out.values()) < 1e-4
