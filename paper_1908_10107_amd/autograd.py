"""Differentiable ORCA trajectories: torch.autograd.Function over the C ABI.

OrcaTrajectory.apply(pos0, vel0, pref_vel, max_speed, time_horizon, sim)
runs ``sim.n_steps`` steps with fixed preferred velocities and returns the
final (pos, vel).  Gradients flow to pos0, vel0, the preferred velocities
and the per-scene max speed and time horizon.  Memory is bounded by step
checkpointing: the forward keeps the state every ``sim.segment`` steps; the
backward replays each segment from its checkpoint with the steps recorded
(neighbour ids, half-plane choices and active constraints), then runs the
hand-written adjoint of its steps in reverse (orca_backward_steps).  The forward
records its last segment as it goes, so the backward replays that one only
if the context has stepped since (a recorded step is bitwise the plain one).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import torch

from . import orca as _orca


@dataclasses.dataclass
class TrajectorySpec:
    offsets: List[int]
    params: list            # scenes.SceneParams-like (max_speed / time_horizon replaced by leaves)
    n_steps: int
    segment: int = 20
    ctx: Optional[_orca.Context] = None
    radius: Optional[torch.Tensor] = None      # per-agent radii [N] (constants), or None
    max_speed: Optional[torch.Tensor] = None   # per-agent max speeds [N] (constants), or None

    def context(self, n):
        if self.ctx is None:
            k = max(1, max(p.max_neighbors for p in self.params))
            self.ctx = _orca.Context(max_agents=n, max_scenes=len(self.params), k_max=k,
                                     tape_steps=self.segment)
        self.ctx.set_agents(self.radius, self.max_speed)
        return self.ctx


def _params_with(spec, vmax, tau):
    out = []
    for s, p in enumerate(spec.params):
        out.append(dataclasses.replace(p, max_speed=float(vmax[s]), time_horizon=float(tau[s])))
    return out


class OrcaTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos0, vel0, pref, vmax, tau, spec: TrajectorySpec):
        n = pos0.shape[1]
        lib = spec.context(n)
        params = _params_with(spec, vmax.detach().cpu().tolist(), tau.detach().cpu().tolist())
        pos = pos0.detach().clone().contiguous()
        vel = vel0.detach().clone().contiguous()
        pref_c = pref.detach().contiguous()
        checkpoints = []
        done = 0
        while done < spec.n_steps:
            k = min(spec.segment, spec.n_steps - done)
            checkpoints.append((pos.clone(), vel.clone(), k))
            last = done + k == spec.n_steps
            lib.step(spec.offsets, params, pos, vel, pref_c, n_steps=k, save_tape=last)
            done += k
        ctx.spec = spec
        ctx.params = params
        ctx.checkpoints = checkpoints
        ctx.tape_epoch = lib.step_epoch  # the recording of the last segment
        ctx.save_for_backward(pref_c)
        return pos, vel

    @staticmethod
    def backward(ctx, g_pos, g_vel):
        (pref_c,) = ctx.saved_tensors
        spec, params = ctx.spec, ctx.params
        lib = spec.context(pref_c.shape[1])
        n_sc = len(params)
        gp = (torch.zeros_like(pref_c) if g_pos is None else g_pos).contiguous().clone()
        gv = (torch.zeros_like(pref_c) if g_vel is None else g_vel).contiguous().clone()
        g_pref = torch.zeros_like(pref_c)
        g_vmax = torch.zeros(n_sc, dtype=torch.float32, device=pref_c.device)
        g_tau = torch.zeros(n_sc, dtype=torch.float32, device=pref_c.device)
        for s, (pos_c, vel_c, k) in enumerate(reversed(ctx.checkpoints)):
            if not (s == 0 and lib.step_epoch == ctx.tape_epoch):
                pos = pos_c.clone()
                vel = vel_c.clone()
                lib.step(spec.offsets, params, pos, vel, pref_c, n_steps=k, save_tape=True)
            lib.backward_steps(0, k - 1, gp, gv, gp, gv, g_pref, g_vmax, g_tau)
        return gp, gv, g_pref, g_vmax, g_tau, None


def trajectory(pos0, vel0, pref, vmax, tau, spec: TrajectorySpec):
    """Final (pos, vel) after spec.n_steps steps; differentiable (see OrcaTrajectory)."""
    return OrcaTrajectory.apply(pos0, vel0, pref, vmax, tau, spec)
