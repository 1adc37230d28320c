#!/usr/bin/env python3
"""Throughput of the micromagnetic step on one MI355X.

One step = the whole hot path once: demagnetising field by zero-padded FFT
convolution (x-forward real FFT, y-forward FFT, z FFT + tensor multiply +
inverse z FFT, y-inverse FFT, x-inverse real FFT), exchange + anisotropy +
Zeeman field, and one explicit Euler LLG update with renormalisation
(Zhu, arXiv:1411.2565, Secs. 2-3), on the 256x256x32 block of 5 nm cubes
(Ms = 8.6e5 A/m, A = 1.3e-11 J/m, alpha = 0.1, dt = 1e-13 s, random initial
state on the unit sphere, seed 0), FP32 with an FP64-built tensor spectrum.

Prints one JSON line: cell-steps/s over the timed steps (state resident in
HBM before timing starts), the roofline position of the dominant kernel
(algorithmic bytes per launch / average launch duration from HIP events on
the launch stream), and the FP64 CPU oracle timed on a bounded sample of the
same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# (each scaled by what the same counter reads for a plain copy of known
# size), keyed by kernel; valid only for the kernel code whose hash
# (kernel_source_sha) is recorded with them.  The summaries and commands are in profiles/.
MEASURED_TRAFFIC = {
    # k_zconv64<false, false>: FETCH_SIZE 76 697.4 KiB x 2.0 + WRITE_SIZE 98 688.0 KiB
    "zconv": {"bytes_per_launch": 258132736,
              "source_sha": "8f130732107ed39672f024651b8380b26c65f6e1a486dc707f7be6fcae7987ea"},
}

def kernel_source_sha():
    """SHA-256 of the kernel sources' code: kernels.hip, fft.hpp and
    launch.hpp with comments, trailing blanks and empty lines removed, so
    that a change of comments keeps a measured traffic valid and any change
    of code voids it."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft.hpp", "launch.hpp"):
        with open(os.path.join(ROOT, "paper_1411_2565_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec and rec["source_sha"] == kernel_source_sha():
        return rec["bytes_per_launch"]
    return None


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Achieved read+write GB/s of a plain device copy (the practical HBM
    ceiling on this GPU), timed with events on the current stream."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def calibration_copy(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the PMC byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()


def kernel_bytes(n, P):
    """HBM bytes per launch of each kernel as implemented (FP32 data,
    complex64 spectra, each array read or written once; the tensor spectrum
    is the real octant, 6 floats per stored frequency).  Unfused, the
    x-inverse writes H_demag and the local kernel reads it back; the fused
    x-inverse + update reads S1 and m and writes m; chained with the next
    step's x-forward it also writes S1 (and that step's x-forward, which
    reads m, does not run)."""
    nx, ny, nz = n
    Px, Py, Pz = P
    Hx = Px // 2 + 1
    Hy = Py // 2 + 1 if Py > 1 else 1
    Hz = Pz // 2 + 1 if Pz > 1 else 1
    N = nx * ny * nz
    m = 4 * 3 * N
    s1 = 8 * 3 * nz * Hx * ny
    s2 = 8 * 3 * nz * Hx * Py
    k = 4 * 6 * Hx * Hy * Hz
    return {"xfwd": m + s1, "yfwd": s1 + s2, "zconv": 2 * s2 + k, "yinv": s2 + s1,
            "xinv": s1 + m, "local": 3 * m, "xinv_local": s1 + 2 * m, "xinv_local_xfwd": 2 * s1 + 2 * m}


def model_bytes(n, P):
    """Algorithmic HBM bytes of one step: the same passes with the x-inverse
    and the local update counted as one pass (S1 read, m read, m written),
    i.e. without the H_demag round trip -- 734.15 MB at 256x256x32."""
    kb = kernel_bytes(n, P)
    return kb["xfwd"] + kb["yfwd"] + kb["zconv"] + kb["yinv"] + kb["xinv_local"]


def unfused_leg(binding, sim, m, w, flags, args):
    """The same steps with the x-inverse and the update as two kernels
    (H_demag written and read back): settle, time, then per-kernel events."""
    import torch
    binding.mm_set_fusion(sim.ctx, 0)
    sim.step(m, args.settle_steps + args.warmup, w.dt, flags)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(m, args.steps, w.dt, flags)
    torch.cuda.synchronize()
    us = 1e6 * (time.perf_counter() - t0) / max(args.steps, 1)
    binding.mm_kernel_timing(sim.ctx, True)
    sim.step(m, args.profile_steps, w.dt, flags)
    times = binding.mm_kernel_times(sim.ctx)
    binding.mm_kernel_timing(sim.ctx, False)
    binding.mm_set_fusion(sim.ctx, 0 if args.no_fusion else args.fusion_level)
    sim.sync()
    return {"us_per_step": round(us, 2),
            "kernels_us": {k: round(1e3 * tot / cnt, 2) for k, (tot, cnt) in times.items() if cnt}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def padded(n):
    if n == 1:
        return 1
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return p


def cpu_baseline(w, m0, target_s=12.0):
    """FP64 oracle, one Euler step at sampled cells of the same workload."""
    import numpy as np
    import oracle
    t = time.perf_counter()
    P = oracle.Problem(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    t_tab = time.perf_counter() - t
    rng = np.random.default_rng(7)
    cal = rng.choice(w.N, 64, replace=False)
    t = time.perf_counter()
    P.step_cells(m0, cal, w.dt)
    t64 = time.perf_counter() - t
    ncell = int(max(64, min(16384, 64 * target_s / max(t64, 1e-6))))
    cells = rng.choice(w.N, ncell, replace=False)
    t = time.perf_counter()
    P.step_cells(m0, cells, w.dt)
    el = time.perf_counter() - t
    return {"value": ncell / el, "unit": "cell-steps/s", "cores": oracle.threads(), "kind": "oracle",
            "cpu": cpu_model(),
            # a full step of the block at this rate (every cell a direct sum
            # over all sources): an extrapolation, not run
            "full_step_s_extrapolated_not_run": round(w.N * el / ncell, 1),
            "sample": (f"one FP64 Euler step (direct-sum Newell demag over all {w.N} source cells + "
                       f"exchange/anisotropy/Zeeman + LLG) at {ncell} randomly sampled cells of the "
                       f"{w.n[0]}x{w.n[1]}x{w.n[2]} block; {el:.1f} s; tensor table build "
                       f"{t_tab:.1f} s not counted")}


def cpu_full_steps():
    """The FP64 oracle's full Euler step (direct sum over all sources) on
    the three workloads small enough for it: seconds per step and
    cell-steps/s, timed on the host threads."""
    import oracle
    from paper_1411_2565_amd import workloads
    rows = []
    for w in (workloads.BLOCK_16x16x2, workloads.BLOCK_64x64x8, workloads.FILM_128x128x4):
        m0, h = workloads.inputs(w)
        P = oracle.Problem(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, hext=h)
        reps = 20 if w.N <= 1024 else 1
        t = time.perf_counter()
        P.run(m0, reps, w.dt)
        el = (time.perf_counter() - t) / reps
        rows.append({"workload": w.name, "cells": w.N, "s_per_step": float(f"{el:.4g}"),
                     "cell_steps_per_s": w.N / el})
    return {"kind": "oracle", "cores": oracle.threads(), "cpu": cpu_model(), "rows": rows}


def adjoint_ratio(binding, T=2000):
    """Backward (segment replay + hand-written adjoint) over forward wall time
    of a T-step rollout on the 128x128x4 film, per-cell field and Ms maps,
    L2 loss to the target pattern, sqrt(T) checkpoints; then the same with
    the whole trajectory stored by the forward (no replay; 2 T 3N floats of
    device memory), reported beside it."""
    import torch
    from paper_1411_2565_amd import workloads
    from paper_1411_2565_amd.rollout import l2_loss, rollout
    w = workloads.FILM_128x128x4
    m0, ms, h, t = workloads.adjoint_inputs(w)
    dev = torch.device("cuda", 0)
    f32 = dict(dtype=torch.float32, device=dev)
    sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, device=0)
    tgt = torch.tensor(t, **f32)

    def once(store="checkpoint"):
        m0g = torch.tensor(m0, **f32).requires_grad_(True)
        hg = torch.tensor(h, **f32).requires_grad_(True)
        msg = torch.tensor(ms, **f32).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mT = rollout(m0g, hg, msg, sim, T, w.dt, 0, None, store)
        loss = l2_loss(mT, tgt, sim)  # FP64 reduction on the GPU
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    once()  # warm-up
    fwd, bwd = once()
    once("all")
    fwd_a, bwd_a = once("all")
    sim.close()
    return {"workload": "film 128x128x4, 5 nm cubes, T=2000, dt=1e-13, maps of h_ext and Ms, "
                        "checkpoint every 45 steps",
            "forward_s": round(fwd, 4), "backward_s": round(bwd, 4), "ratio": round(bwd / fwd, 3),
            "stored": {"forward_s": round(fwd_a, 4), "backward_s": round(bwd_a, 4),
                       "ratio": round(bwd_a / fwd_a, 3), "bytes": 2 * T * 3 * w.N * 4}}


def batch_rate(binding, steps=5000, single_steps=200):
    """Aggregate cell-steps/s of the 64-film batch (one launch per pass and
    transform length, 32-step hipGraph chunks), then with the launch shapes
    the batch autotuner picks, against the same films stepped one by one
    (eager launches, and each film replaying its own graphs), on the same
    GPU."""
    import torch
    from paper_1411_2565_amd import workloads
    films = workloads.batch_films(count=64, seed=0)
    w0 = films[0][0]
    cells = sum(w.N for (w, _, _) in films)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B = binding.Batch([w.n for (w, _, _) in films], w0.d, Ms=w0.Ms, A=w0.A, alpha=w0.alpha,
                          hext=[tuple(h) for (_, _, h) in films])
        m = B.pack([m0 for (_, m0, _) in films])
        B.step(m, 64, w0.dt, binding.MM_F_GRAPH)
        B.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.step(m, steps, w0.dt, binding.MM_F_GRAPH)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        # the same batch with launch shapes chosen by the batch autotuner
        choice = B.autotune(None)
        B.step(m, 64, w0.dt, binding.MM_F_GRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.step(m, steps, w0.dt, binding.MM_F_GRAPH)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        launches = len(choice)
        B.sync()
        B.close()
        sims = []
        states = []
        for (w, m0, h) in films:
            sims.append(binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, hext=tuple(h)))
            states.append(torch.tensor(m0, dtype=torch.float32, device="cuda:0"))
        for sim, st in zip(sims, states):
            sim.step(st, 4, w0.dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sim, st in zip(sims, states):
            sim.step(st, single_steps, w0.dt)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        # the same films one by one, each replaying its own captured graphs
        for sim, st in zip(sims, states):
            sim.step(st, 64, w0.dt, binding.MM_F_GRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sim, st in zip(sims, states):
            sim.step(st, single_steps, w0.dt, binding.MM_F_GRAPH)
        torch.cuda.synchronize()
        tsg = time.perf_counter() - t0
        for sim in sims:
            sim.close()
    return {"workload": f"64 films, {cells} cells in all, 4x4x3 nm, dt=5e-14",
            "batched_cell_steps_per_s": cells * steps / tb, "batched_us_per_step": round(1e6 * tb / steps, 1),
            "tuned_us_per_step": round(1e6 * tt / steps, 1), "tuned_choice_xyz_launches": list(choice),
            "tunable_launches": launches,
            "one_by_one_cell_steps_per_s": cells * single_steps / ts,
            "one_by_one_us_per_step": round(1e6 * ts / single_steps, 1),
            "one_by_one_graph_us_per_step": round(1e6 * tsg / single_steps, 1),
            "speedup": round((cells * steps / tb) / (cells * single_steps / ts), 2),
            "speedup_vs_graph_one_by_one": round((cells * steps / tb) / (cells * single_steps / tsg), 2)}


def compensated_leg(binding, w, m0, steps=1000, timed_steps_n=300, crop_stride=8):
    """Plain against compensated (Dot2) spectral multiply on the benchmark
    block: microseconds per step of each, and the error of H_demag against
    the FP64 oracle's direct sum on a subsample of the centred 64x64x8
    crop of observers (x, y in [96, 160), z in [12, 20); every
    crop_stride-th cell) at step 0 and after `steps` steps of each form."""
    import numpy as np
    import torch
    import oracle
    nx, ny, nz = w.n
    z, y, x = np.meshgrid(np.arange(12, 20), np.arange(96, 160), np.arange(96, 160), indexing="ij")
    obs = ((z * ny + y) * nx + x).ravel()[::crop_stride]
    P = oracle.Problem(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha)
    sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, device=0)
    out = {"workload": f"block {nx}x{ny}x{nz}, dt={w.dt}", "observers": int(obs.size),
           "crop": "x,y in [96,160), z in [12,20), every %d-th cell" % crop_stride, "steps": steps}

    def err(m):
        Hd = sim.heff(m, binding.MM_T_DEMAG).cpu().double().numpy().reshape(3, -1)[:, obs]
        ref = P.demag_observers(m.cpu().double().numpy(), obs)
        return {"rel_l2": float(np.linalg.norm(Hd - ref) / np.linalg.norm(ref)),
                "cell_max": float(np.abs(Hd - ref).max() / np.abs(ref).max())}

    for name, comp in (("plain", 0), ("compensated", 1)):
        binding.mm_set_compensated(sim.ctx, comp)
        m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
        e0 = err(m)
        sim.step(m, steps, w.dt)
        sim.sync()
        e1 = err(m)
        sim.step(m, 20, w.dt)
        t = timed_steps(sim, m, timed_steps_n, w.dt, 0)
        out[name] = {"us_per_step": round(1e6 * t / timed_steps_n, 1), "h_demag_error_step0": e0,
                     f"h_demag_error_step{steps}": e1}
    sim.sync()
    sim.close()
    return out


# Table 1 of the paper: ms per Euler step on an AMD Radeon HD 7970 GHz
# Edition (C++ AMP), N x N x N cubes.  Context only: other hardware.
PAPER_TABLE1_MS = {8: 1.95, 16: 2.723, 32: 3.151, 64: 6.558, 128: 26.34}


def timed_steps(sim, m, steps, dt, flags):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(m, steps, dt, flags)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def small_configs(binding):
    """The two latency-bound workloads at their configured step counts: the
    16x16x2 parity block (100 steps of 1e-13 s, repeated 20 times) and the
    256x64x1 thin film (20 000 steps of 5e-14 s, its field applied): eager
    launches and 32-step hipGraph chunks."""
    import torch
    from paper_1411_2565_amd import workloads
    rows = []
    s = torch.cuda.Stream()  # graph capture needs a non-default stream
    for w, steps in ((workloads.BLOCK_16x16x2, 2000), (workloads.FILM_256x64x1, 20000)):
        m0, h = workloads.inputs(w)
        with torch.cuda.stream(s):
            sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, Ku=w.Ku, u=w.u, alpha=w.alpha, hext=tuple(h), device=0)
            m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
            sim.step(m, 64, w.dt, binding.MM_F_GRAPH)
            sim.step(m, 64, w.dt)
            te = timed_steps(sim, m, steps, w.dt, 0)
            tg = timed_steps(sim, m, steps, w.dt, binding.MM_F_GRAPH)
            sim.sync()
            sim.close()
        rows.append({"workload": w.name, "cells": w.N, "steps": steps, "dt": w.dt,
                     "us_per_step": round(1e6 * te / steps, 2), "us_per_step_graph": round(1e6 * tg / steps, 2),
                     "cell_steps_per_s": w.N * steps / min(te, tg)})
    return rows


def sweep_row(binding, w, graphs=True):
    import torch
    from paper_1411_2565_amd import workloads
    m0, _ = workloads.inputs(w)
    t = time.perf_counter()
    sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, Ku=w.Ku, u=w.u, alpha=w.alpha, device=0)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
    steps = 32 * max(4, min(64, int(6e7 / w.N)))
    if graphs:
        sim.step(m, 64, w.dt, binding.MM_F_GRAPH)
    sim.step(m, 32, w.dt)
    te = timed_steps(sim, m, steps, w.dt, 0)
    tg = timed_steps(sim, m, steps, w.dt, binding.MM_F_GRAPH) if graphs else None
    binding.mm_kernel_timing(sim.ctx, True)
    sim.step(m, 20, w.dt)
    kt = binding.mm_kernel_times(sim.ctx)
    binding.mm_kernel_timing(sim.ctx, False)
    sim.sync()
    sim.close()
    N = w.n[0]
    return {"n": N, "cells": w.N, "padded": [padded(v) for v in w.n], "steps": steps,
            "us_per_step": round(1e6 * te / steps, 2),
            "us_per_step_graph": round(1e6 * tg / steps, 2) if graphs else None,
            "cell_steps_per_s": w.N * steps / (min(te, tg) if graphs else te), "tensor_build_s": round(t_build, 3),
            "kernels_us": {k: round(1e3 * t / c, 2) for k, (t, c) in kt.items() if c},
            "paper_ms_per_step": PAPER_TABLE1_MS.get(N)}


def size_sweep(binding, sizes=None, graphs=True):
    """Per-step time on Table 1's N^3 cubes (A = 1e-11 J/m, Ms = 1e6 A/m,
    anisotropy field 1e5 A/m along x, 5 nm cells, alpha = 0.5, dt = 1e-13 s,
    random initial state): eager launches and 32-step hipGraph chunks."""
    import torch
    from paper_1411_2565_amd import workloads
    rows = []
    s = torch.cuda.Stream()  # graph capture needs a non-default stream
    for N in sizes or workloads.TABLE1_SIZES:
        with torch.cuda.stream(s):
            rows.append(sweep_row(binding, workloads.table1_cube(N), graphs))
        torch.cuda.empty_cache()
    return {"workload": "N^3 cubes, 5 nm cells, A=1e-11, Ms=1e6, H_K=1e5 A/m along x, alpha=0.5, dt=1e-13",
            "paper_hardware": "AMD Radeon HD 7970 GHz Edition (Table 1)", "rows": rows}


def sp4_rate(binding, steps=2048):
    """Standard problem #4 film as the paper runs it (500 x 125 x 3 cells of
    1 nm, padded 1024 x 256 x 8, alpha = 0.02, field 1, dt = 1e-13 s as in the
    paper's input file): per-step time, eager and hipGraph."""
    import torch
    from paper_1411_2565_amd import workloads
    w = workloads.SP4_500x125x3
    m0, _ = workloads.inputs(w)
    h = workloads.field_mT(workloads.SP4_FIELD1_mT)
    s = torch.cuda.Stream()  # graph capture needs a non-default stream
    with torch.cuda.stream(s):
        sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, hext=tuple(h), device=0)
        m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
        sim.step(m, 64, w.dt, binding.MM_F_GRAPH)
        sim.step(m, 32, w.dt)
        te = timed_steps(sim, m, steps, w.dt, 0)
        tg = timed_steps(sim, m, steps, w.dt, binding.MM_F_GRAPH)
        sim.sync()
        sim.close()
    return {"workload": "film 500x125x3, 1 nm cells, padded 1024x256x8, alpha=0.02, field 1, dt=1e-13",
            "steps": steps, "us_per_step": round(1e6 * te / steps, 2), "us_per_step_graph": round(1e6 * tg / steps, 2),
            "cell_steps_per_s": w.N * steps / min(te, tg)}


def integrator_rates(binding, steps=200):
    """Per-step time of the Euler, Heun and classic RK4 steps on the
    256x256x32 block (1, 2 and 4 field evaluations per step), eager, and of
    adaptive Bogacki-Shampine 3(2) and Dormand-Prince 5(4) attempts (4 and
    7 evaluations, an error reduction and a host round trip each)."""
    import torch
    from paper_1411_2565_amd import workloads
    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, device=0)
    out = {"workload": "block 256x256x32, 5 nm cubes, dt=1e-13", "steps": steps}
    for name, fl in (("euler", 0), ("heun", binding.MM_F_HEUN), ("rk4", binding.MM_F_RK4)):
        m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
        sim.step(m, 10, w.dt, fl)
        t = timed_steps(sim, m, steps, w.dt, fl)
        out[name + "_us_per_step"] = round(1e6 * t / steps, 1)
    m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
    sim.step(m, 20, w.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dt, acc, rej = sim.run_adaptive(m, 2e-12, 1e-14, 1e-5, binding.MM_F_BS23)
    el = time.perf_counter() - t0
    out["bs23_adaptive"] = {"t_end": 2e-12, "tol": 1e-5, "accepted": acc, "rejected": rej,
                            "last_dt": dt, "us_per_attempt": round(1e6 * el / max(acc + rej, 1), 1)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dt, acc, rej = sim.run_adaptive(m, 2e-12, 1e-14, 1e-5, binding.MM_F_DP54)
    el = time.perf_counter() - t0
    out["dp54_adaptive"] = {"t_end": 2e-12, "tol": 1e-5, "accepted": acc, "rejected": rej,
                            "last_dt": dt, "us_per_attempt": round(1e6 * el / max(acc + rej, 1), 1)}
    sim.sync()
    sim.close()
    return out


def geometry_rate(binding, steps=500):
    """Step time on the 256x256x32 grid with the inscribed elliptic cylinder
    as magnetic body (vacuum outside, Ms map), against the full block: the
    cost of non-regular geometry on the same FFT grid."""
    import torch
    from paper_1411_2565_amd import workloads
    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    ms = workloads.disk_ms_map(w.n, w.Ms)
    out = {"workload": "256x256x32 grid, 5 nm cubes, disk of 1.28 um diameter through all 32 layers "
                       "(vacuum outside), dt=1e-13", "magnetic_cells": int((ms > 0).sum()), "steps": steps}
    for name, use_map in (("full_block", False), ("disk", True)):
        sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, device=0)
        if use_map:
            sim.set_ms_map(torch.tensor(ms, dtype=torch.float32, device="cuda:0"))
        m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
        sim.step(m, 20, w.dt)
        t = timed_steps(sim, m, steps, w.dt, 0)
        sim.sync()
        sim.close()
        out[name + "_us_per_step"] = round(1e6 * t / steps, 1)
    return out


def tuning_rates(binding, steps=300):
    """Autotuned launch shapes against the defaults: per-step time on the
    256x256x32 block and on the 128^3 and 256^3 cubes of the sweep."""
    import torch
    from paper_1411_2565_amd import workloads
    rows = []
    for w in (workloads.BLOCK_256x256x32, workloads.table1_cube(128), workloads.table1_cube(256)):
        m0, _ = workloads.inputs(w)
        sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, Ku=w.Ku, u=w.u, alpha=w.alpha, device=0)
        m = torch.tensor(m0, dtype=torch.float32, device="cuda:0")
        n = steps if w.N <= 2097152 else max(20, steps // 8)
        sim.step(m, 20, w.dt)
        t_def = timed_steps(sim, m, n, w.dt, 0)
        choice = sim.autotune(None)
        sim.step(m, 20, w.dt)
        t_tun = timed_steps(sim, m, n, w.dt, 0)
        sim.sync()
        sim.close()
        del m
        torch.cuda.empty_cache()
        rows.append({"workload": w.name, "choice_xyz": list(choice), "steps": n,
                     "default_us_per_step": round(1e6 * t_def / n, 1), "tuned_us_per_step": round(1e6 * t_tun / n, 1)})
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps right before the timed region")
    ap.add_argument("--settle-steps", type=int, default=300,
                    help="untimed steps before the warm-up: the GPU ramps its clocks over the first "
                         "~100-300 steps of a burst")
    ap.add_argument("--profile-steps", type=int, default=200,
                    help="steps of the per-kernel event-timed region that follows the timed region")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--compensated", action="store_true",
                    help="run the headline timing with the compensated spectral multiply")
    ap.add_argument("--no-fusion", action="store_true",
                    help="run the headline timing with the x-inverse and the update as two kernels")
    ap.add_argument("--fusion-level", type=int, default=1, choices=(1, 2),
                    help="1: x-inverse + update fused; 2: also the next step's x-forward")
    ap.add_argument("--no-unfused-leg", action="store_true",
                    help="skip the timing of the two-kernel (unfused) step")
    ap.add_argument("--no-compensated-leg", action="store_true",
                    help="skip the plain-vs-compensated timing and crop errors")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-films throughput")
    ap.add_argument("--no-graphs", action="store_true",
                    help="with --sweep: time the cubes with eager launches only (for rocprofv3 --pmc runs)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the latency-bound workloads (they replay hipGraphs, which rocprofv3 --pmc "
                         "runs of this ROCm have not survived)")
    ap.add_argument("--sweep", action="store_true",
                    help="also time the N^3 cube size sweep and the standard problem #4 film")
    ap.add_argument("--sweep-sizes", type=int, nargs="+", default=None,
                    help="with --sweep: only these cube sizes N, and no standard problem #4 film")
    ap.add_argument("--integrators", action="store_true",
                    help="also time the Heun, RK4 and adaptive steps on the block")
    ap.add_argument("--geometry", action="store_true",
                    help="also time a disk (vacuum outside) on the block's grid")
    ap.add_argument("--tune", action="store_true",
                    help="also autotune the launch shapes and time them against the defaults")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (3 times) for PMC counter calibration")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the single-GPU throughput is the --gpus 1 line)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_2565_amd import binding, workloads

    w = workloads.BLOCK_256x256x32
    m0, _ = workloads.inputs(w)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    flags = binding.MM_F_COMPENSATED if args.compensated else 0

    t = time.perf_counter()
    sim = binding.Sim(w.n, w.d, Ms=w.Ms, A=w.A, alpha=w.alpha, device=0)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    m = torch.tensor(m0, dtype=torch.float32, device=dev)
    binding.mm_set_fusion(sim.ctx, 0 if args.no_fusion else args.fusion_level)

    print(f"bench: {args.settle_steps} settle + {args.warmup} warm-up steps", file=sys.stderr, flush=True)
    sim.step(m, args.settle_steps, w.dt, flags)
    sim.step(m, args.warmup, w.dt, flags)
    sim.sync()

    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(m, args.steps, w.dt, flags)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.sync()
    ms_step = 1e3 * el / max(args.steps, 1)
    value = w.N * args.steps / el

    # per-kernel durations: right after the timed region, the same steps
    # again with every kernel's dispatch recording its own start and stop
    # events on the launch stream.  (Recording them inside the timed region
    # itself was measured to add about 15 us of gaps per step.)
    print(f"bench: per-kernel event timing over {args.profile_steps} steps", file=sys.stderr, flush=True)
    binding.mm_kernel_timing(sim.ctx, True)
    sim.step(m, args.profile_steps, w.dt, flags)
    times = binding.mm_kernel_times(sim.ctx)
    binding.mm_kernel_timing(sim.ctx, False)
    sim.sync()
    P = tuple(padded(v) for v in w.n)
    kb = kernel_bytes(w.n, P)
    kernels = {}
    for k, (tot_ms, cnt) in times.items():
        avg_us = 1e3 * tot_ms / max(cnt, 1)
        kernels[k] = {"avg_us": round(avg_us, 2), "launches": cnt, "bytes": kb[k],
                      "GBps": round(kb[k] / (avg_us * 1e-6) / 1e9, 1) if cnt else None}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    ach = kernels[dom]["GBps"]
    # bytes per step of the kernels that ran (launch counts over the region:
    # with the chained x-forward, the x-forward runs once per call)
    step_bytes_impl = sum(kb[k] * v["launches"] for k, v in kernels.items()) / max(args.profile_steps, 1)
    step_bytes = model_bytes(w.n, P)

    unfused = None
    if not args.no_unfused_leg and not args.no_fusion:
        print("bench: unfused step (x-inverse and update as two kernels)", file=sys.stderr, flush=True)
        unfused = unfused_leg(binding, sim, m, w, flags, args)

    sim.close()
    copy_bw = copy_bandwidth()
    comp = None
    if not args.no_compensated_leg:
        print("bench: plain vs compensated spectral multiply", file=sys.stderr, flush=True)
        comp = compensated_leg(binding, w, m0)
    adj = None
    if not args.no_adjoint:
        print("bench: adjoint/forward ratio on the 128x128x4 film", file=sys.stderr, flush=True)
        adj = adjoint_ratio(binding)

    small = None
    if not args.no_small:
        print("bench: latency-bound workloads (16x16x2 block, 256x64x1 film)", file=sys.stderr, flush=True)
        small = small_configs(binding)

    bat = None
    if not args.no_batch:
        print("bench: batched films", file=sys.stderr, flush=True)
        bat = batch_rate(binding)

    sweep = sp4 = None
    if args.sweep:
        print("bench: N^3 cube size sweep", file=sys.stderr, flush=True)
        sweep = size_sweep(binding, args.sweep_sizes, graphs=not args.no_graphs)
        if not args.sweep_sizes:
            print("bench: standard problem #4 film", file=sys.stderr, flush=True)
            sp4 = sp4_rate(binding)

    rk = None
    if args.integrators:
        print("bench: Runge-Kutta steps", file=sys.stderr, flush=True)
        rk = integrator_rates(binding)

    tun = None
    if args.tune:
        print("bench: autotuned launch shapes", file=sys.stderr, flush=True)
        tun = tuning_rates(binding)

    geo = None
    if args.geometry:
        print("bench: non-regular geometry", file=sys.stderr, flush=True)
        geo = geometry_rate(binding)

    cpu = cpu_full = None
    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, m0)
        cpu_full = cpu_full_steps()

    line = {
        "metric": "cell-steps/s (H_eff+LLG) at 256x256x32 FP32, %HBM peak; adjoint/fwd time ratio",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_steps": args.settle_steps,
        "profile_steps": args.profile_steps,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "block 256x256x32 cells, 5 nm cubes, padded FFT 512x512x64",
                   "cells": w.N, "dt": w.dt, "alpha": w.alpha, "Ms": w.Ms, "A": w.A,
                   "spectral_multiply": "compensated" if args.compensated else "plain",
                   "fusion_level": 0 if args.no_fusion else args.fusion_level},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom)},
        "cpu_baseline": cpu,
        "cpu_full_steps": cpu_full,
        "step_bytes": step_bytes,
        "step_bytes_impl": step_bytes_impl,
        "step_hbm_frac_impl": round(step_bytes_impl / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "unfused": unfused,
        "compensated": comp,
        "copy_GBps": copy_bw,
        "step_hbm_frac": round(step_bytes / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "kernels": kernels,
        "tensor_build_s": round(t_build, 3),
        "adjoint": adj,
        "batch": bat,
        "small_workloads": small,
        "size_sweep": sweep,
        "sp4": sp4,
        "integrators": rk,
        "geometry": geo,
        "tuning": tun,
    }
    print(json.dumps(line), flush=True)
    if args.calib_copy:
        calibration_copy()


if __name__ == "__main__":
    main()
