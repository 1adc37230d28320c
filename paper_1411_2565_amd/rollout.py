"""Differentiable Euler rollout with sqrt(T) checkpointing.

``LLGRollout.apply(m0, hext_map, ms_map, sim, T, dt)`` advances the state T
explicit-Euler steps of the LLG equation (Zhu, arXiv:1411.2565, eq. (3), with
the effective field of eq. (2)) on the GPU and returns m_T.  Its backward
pass returns dL/dm0, dL/dh_ext (per-cell map, A/m) and dL/dMs (per-cell map)
for any loss L(m_T), using the library's hand-written adjoint step.

Memory (``store``):
- "checkpoint" (default): the forward keeps one state every S =
  ceil(sqrt(T)) steps.  The backward walks the segments from last to first;
  for each it replays the S forward steps from the checkpoint while storing
  every state and its demagnetising field (mm_forward_store), then runs the
  S adjoint steps backwards in one call (mm_adjoint_segment).  The replay
  computes the same arithmetic as the forward pass (whose Euler steps fuse
  the x-inverse and the update, bit for bit equal to the replay's two
  passes), so the recomputed states are bitwise those of the forward.
- "all": the forward itself stores every state and its demagnetising field
  (2 T 3N floats of device memory) and the backward runs the T adjoint steps
  alone, with no replay.  The same kernels in the same order as the
  checkpointed form, so the same m_T and gradients bit for bit; it trades
  memory (3.1 GB for a 128x128x4 film over 2000 steps) for the replay.
"""
import math

import torch

from . import binding as B


def _segments(T, S):
    return [(k, min(S, T - k)) for k in range(0, T, S)]


class LLGRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, hext_map, ms_map, sim, T, dt, flags=0, seg=None, store="checkpoint"):
        T = int(T)
        if store not in ("checkpoint", "all"):
            raise ValueError(f"store must be 'checkpoint' or 'all', not {store!r}")
        S = T if store == "all" else (int(seg) if seg else max(1, math.ceil(math.sqrt(T))))
        sim.set_hext_map(hext_map.detach().contiguous())
        sim.set_ms_map(ms_map.detach().contiguous())
        m = m0.detach().contiguous().clone()
        ctx.sim, ctx.T, ctx.dt, ctx.flags, ctx.S = sim, T, dt, flags, S
        ctx.maps = (hext_map.detach().contiguous(), ms_map.detach().contiguous())
        ctx.traj = None
        if store == "all":
            N = sim.N
            mtraj = torch.empty((max(T, 1), 3 * N), dtype=torch.float32, device=m.device)
            hdtraj = torch.empty_like(mtraj)
            if T:
                sim._s()
                B.mm_forward_store(sim.ctx, m, T, dt, flags, mtraj[:T], hdtraj[:T], N)
            ctx.traj = (mtraj, hdtraj)
            ctx.ckpts = None
            return m
        ckpts = []
        for (_, n) in _segments(T, S):
            ckpts.append(m.clone())
            sim.step(m, n, dt, flags)
        ctx.ckpts = ckpts
        return m

    @staticmethod
    def backward(ctx, grad):
        sim, T, dt, flags, S = ctx.sim, ctx.T, ctx.dt, ctx.flags, ctx.S
        hmap, msmap = ctx.maps
        sim.set_hext_map(hmap)
        sim.set_ms_map(msmap)
        lam = grad.detach().contiguous().clone().float()
        g_h = torch.zeros_like(hmap)
        g_ms = torch.zeros_like(msmap)
        N = sim.N
        if ctx.traj is not None:  # store == "all": no replay
            mtraj, hdtraj = ctx.traj
            if T:
                sim._s()
                B.mm_adjoint_segment(sim.ctx, mtraj[:T], hdtraj[:T], T, lam, g_h, g_ms, dt, flags, N)
            ctx.traj = None
            return lam, g_h, g_ms, None, None, None, None, None, None
        segs = _segments(T, S)
        mtraj = torch.empty((S, 3 * N), dtype=torch.float32, device=lam.device)
        hdtraj = torch.empty_like(mtraj)
        for idx in range(len(segs) - 1, -1, -1):
            _, n = segs[idx]
            m = ctx.ckpts[idx].clone()
            sim._s()
            B.mm_forward_store(sim.ctx, m, n, dt, flags, mtraj[:n], hdtraj[:n], N)
            B.mm_adjoint_segment(sim.ctx, mtraj[:n], hdtraj[:n], n, lam, g_h, g_ms, dt, flags, N)
        ctx.ckpts = None
        return lam, g_h, g_ms, None, None, None, None, None, None


def rollout(m0, hext_map, ms_map, sim, T, dt, flags=0, seg=None, store="checkpoint"):
    """m_T of a T-step Euler rollout, differentiable in m0, hext_map, ms_map;
    store = "checkpoint" (sqrt(T) checkpoints, default) or "all"."""
    return LLGRollout.apply(m0, hext_map, ms_map, sim, T, dt, flags, seg, store)


class L2Loss(torch.autograd.Function):
    """L = 1/2 sum (m - t)^2 reduced in FP64 on the GPU (mm_reduce_loss),
    returned as a float64 scalar; the same kernel writes dL/dm = m - t, which
    the backward hands on (times the incoming gradient)."""

    @staticmethod
    def forward(ctx, m, target, sim):
        out, g = sim.loss(m.detach().contiguous(), target.detach().contiguous(), grad=True)
        ctx.save_for_backward(g)
        return out.reshape(())

    @staticmethod
    def backward(ctx, go):
        (g,) = ctx.saved_tensors
        return g * go.to(g.dtype), None, None


def l2_loss(m, target, sim):
    """FP64 GPU loss 1/2 sum (m - target)^2, differentiable in m."""
    return L2Loss.apply(m, target, sim)
