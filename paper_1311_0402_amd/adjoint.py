"""Trajectory gradients through the DPD step, behind torch.autograd.Function.

``trajectory_forces(a, gamma, x0, v0, spec)`` returns the forces F_1..F_K of
K velocity-Verlet steps started from (x0, v0) (forces F_0 evaluated at the
start with v0), in tag order, as a differentiable function of the
type-pair tables a and gamma and of x0, v0.  The pair Gaussian stream and
the pair sets along the trajectory are held fixed (they do not depend on the
differentiated quantities away from measure-zero cutoff crossings).

Memory: the forward pass keeps a checkpoint of the reordered state every
``spec.checkpoint`` steps; the backward pass re-runs each segment from its
checkpoint, keeping that segment's states and lists, then walks it in
reverse with ``dpd_step_backward`` (one HIP reverse step per step) and closes
with ``dpd_forces_backward`` for the initial forces.  All arithmetic runs in
libdpd; the Python side only orders the calls and moves arrays between the
tag order of the caller and the sorted order of each step.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Optional

import numpy as np
import torch

from . import dpd as D


@dataclass
class TrajectorySpec:
    params: D.Params            # box, r_c, dt, s, seed, ...; a and gamma come from the inputs
    tag: np.ndarray             # uint32 [N], the tags of x0 / v0 columns (a permutation of 0..N-1)
    type: np.ndarray            # uint8 [N]
    steps: int                  # K
    checkpoint: int = 10        # steps between stored states


def _params_with(spec: TrajectorySpec, a: torch.Tensor, gamma: torch.Tensor) -> D.Params:
    return replace(spec.params, a=a.detach().double().cpu().numpy(),
                   gamma=gamma.detach().double().cpu().numpy())


def _snapshot(sim: D.System):
    st = sim.state
    return (st.x.clone(), st.v.clone(), st.f.clone(), st.tag.clone(), st.type.clone(), int(sim.d_step.item()))


def _restore(sim: D.System, snap) -> None:
    x, v, f, tag, typ, step = snap
    st = sim.state
    st.x.copy_(x); st.v.copy_(v); st.f.copy_(f); st.tag.copy_(tag); st.type.copy_(typ)
    sim.d_step.fill_(step)
    sim.status.zero_()


def _keep_step(sim: D.System):
    """Everything the reverse of the last step needs."""
    st, c, nl = sim.state, sim.cells, sim.nlist
    nnz = int(nl.offset[sim.n].item())
    state = D.State(st.x.clone(), st.v.clone(), st.f.clone(), st.tag.clone(), st.type.clone())
    cells = D.Cells(c.cell_start, c.cell_xyz.clone(), c.perm.clone(), c.idx_of_tag.clone())
    nlist = D.NList(nl.offset.clone(), nl.index[:max(nnz, 1)].clone())
    return state, cells, nlist


def _load_device(sim: D.System, x0: torch.Tensor, v0: torch.Tensor, tag: np.ndarray, typ: np.ndarray) -> None:
    src = D.State.empty(sim.n, sim.device)
    src.x.copy_(x0.detach().double())
    src.v.copy_(v0.detach().double())
    src.tag.copy_(torch.as_tensor(np.ascontiguousarray(tag).astype(np.uint32).view(np.int32)))
    src.type.copy_(torch.as_tensor(np.ascontiguousarray(typ, dtype=np.uint8)))
    sim.d_step.zero_()
    sim.status.zero_()
    sim.reorder_from(src)
    sim.rebuild()
    sim.fit_capacity()
    sim.compute_forces(0)


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, gamma, x0, v0, spec: TrajectorySpec):
        params = _params_with(spec, a, gamma)
        n = x0.shape[1]
        sim = D.System(params, n, D.FP64)
        _load_device(sim, x0, v0, spec.tag, spec.type)
        perm0 = sim.cells.perm.clone()
        ckpts = {0: _snapshot(sim)}
        out = torch.empty((spec.steps, 3, n), dtype=torch.float64, device=x0.device)
        for k in range(1, spec.steps + 1):
            sim.step(1)
            out[k - 1].index_copy_(1, sim.state.tag.long(), sim.state.f)
            if k % spec.checkpoint == 0 and k < spec.steps:
                ckpts[k] = _snapshot(sim)
        sim.check_status()
        ctx.spec, ctx.params, ctx.ckpts, ctx.perm0, ctx.sim = spec, params, ckpts, perm0, sim
        ctx.a_meta = (a.dtype, a.device, a.shape)
        ctx.g_meta = (gamma.dtype, gamma.device, gamma.shape)
        return out

    @staticmethod
    def backward(ctx, g_out):
        spec, params, sim = ctx.spec, ctx.params, ctx.sim
        n, K, C = sim.n, spec.steps, spec.checkpoint
        dev = sim.device
        nt = params.n_types
        g_out = g_out.contiguous()
        ga = torch.zeros(nt * nt, dtype=torch.float64, device=dev)
        gg = torch.zeros(nt * nt, dtype=torch.float64, device=dev)
        cur = [torch.zeros((3, n), dtype=torch.float64, device=dev) for _ in range(3)]   # gx, gv, gf
        nxt = [torch.zeros((3, n), dtype=torch.float64, device=dev) for _ in range(3)]
        starts = list(range(0, K, C))
        first = True
        for s0 in reversed(starts):
            s1 = min(s0 + C, K)
            _restore(sim, ctx.ckpts[s0])
            kept: List = []
            for _ in range(s0 + 1, s1 + 1):
                sim.step(1)
                kept.append(_keep_step(sim))
            sim.check_status()
            for k in range(s1, s0, -1):
                state, cells, nlist = kept[k - s0 - 1]
                if first:
                    for t in cur:
                        t.zero_()
                    first = False
                # loss gradient of F_k, brought from tag order to this step's order
                cur[2].add_(g_out[k - 1].index_select(1, state.tag.long()))
                D.dpd_step_backward(params, state, cells, nlist, k, cur[0], cur[1], cur[2],
                                    nxt[0], nxt[1], nxt[2], ga, gg, sim.ws)
                cur, nxt = nxt, cur
        # the initial forces F_0 = F(x0, v0, 0) at the load-time order: re-bin
        # the restored (already sorted, so the order is kept) state to refresh
        # its cell list and FP32 offsets, then rebuild its neighbour list
        _restore(sim, ctx.ckpts[0])
        src = D.State(*(t.clone() for t in (sim.state.x, sim.state.v, sim.state.f, sim.state.tag,
                                            sim.state.type)))
        sim.reorder_from(src)
        sim.rebuild()
        sim.fit_capacity()
        D.dpd_forces_backward(params, sim.state, sim.cells, sim.nlist, 0, cur[2], cur[0], cur[1], ga, gg,
                              sim.ws, accumulate=True)
        perm0 = ctx.perm0.long()
        gx0 = torch.empty_like(cur[0]).index_copy_(1, perm0, cur[0])
        gv0 = torch.empty_like(cur[1]).index_copy_(1, perm0, cur[1])
        adt, adev, ashape = ctx.a_meta
        gdt, gdev, gshape = ctx.g_meta
        ga_t = ga.reshape(nt, nt).to(dtype=adt, device=adev).reshape(ashape)
        gg_t = gg.reshape(nt, nt).to(dtype=gdt, device=gdev).reshape(gshape)
        return ga_t, gg_t, gx0, gv0, None


def trajectory_forces(a: torch.Tensor, gamma: torch.Tensor, x0: torch.Tensor, v0: torch.Tensor,
                      spec: TrajectorySpec) -> torch.Tensor:
    """[K, 3, N] forces of steps 1..K (tag order), differentiable in a, gamma, x0, v0."""
    return _Trajectory.apply(a, gamma, x0, v0, spec)


def force_matching_loss(a, gamma, x0, v0, spec: TrajectorySpec, targets: torch.Tensor) -> torch.Tensor:
    """sum over steps 1..K of |F_k - F_target,k|^2 (targets [K, 3, N], tag order)."""
    f = trajectory_forces(a, gamma, x0, v0, spec)
    return ((f - targets) ** 2).sum()
