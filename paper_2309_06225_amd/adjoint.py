"""Gradients of a trajectory of frozen-ghost RK4 steps (checkpointed adjoint).

Forward: n RK4 steps through libgrf, keeping the state every `every` steps.
Backward: for each segment, last first, the segment is re-run from its
checkpoint keeping every step-start state (and, if `keep_stages`, the three
stage states of every step), then libgrf's RK4-step adjoint is applied step by
step in reverse.  The couplings theta = (lambda_gb, g2) and the initial state
receive gradients.  All arithmetic runs in libgrf's kernels; this module only
orders the calls and owns the buffers.
"""
from __future__ import annotations

import torch

from . import grf as G


class Trajectory:
    def __init__(self, params: dict, box: G.Box, dt: float, nsteps: int, every: int = 10, keep_stages: bool = True):
        if box.bc != G.BC_FROZEN:
            raise ValueError("the trajectory adjoint is implemented for frozen ghosts")
        self.pdict, self.box, self.dt, self.nsteps = dict(params), box, float(dt), int(nsteps)
        self.every = max(1, int(every))
        self.keep_stages = keep_stages
        self._ws = None
        self._vws = None

    def _params(self, theta):
        return G.make_params(self.pdict, lambda_gb=float(theta[0]), g2=float(theta[1]))

    def _ws_fwd(self, dev):
        if self._ws is None:
            self._ws = G.alloc_workspace(G.workspace_bytes(self.box), dev)
        return self._ws

    def _ws_vjp(self, dev):
        if self._vws is None:
            self._vws = G.alloc_workspace(G.step_vjp_workspace_bytes(self.box), dev)
        return self._vws

    def step(self, P, u, acc, bufs=None):
        """One RK4 step from u; returns (u_new, (u2, u3, u4))."""
        ws = self._ws_fwd(u.device)
        u2, u3, u4, un = bufs if bufs is not None else (u.clone(), u.clone(), u.clone(), u.clone())
        G.rk4_stage(P, self.box, 1, self.dt, u, u, u2, acc, ws)
        G.rk4_stage(P, self.box, 2, self.dt, u, u2, u3, acc, ws)
        G.rk4_stage(P, self.box, 3, self.dt, u, u3, u4, acc, ws)
        G.rk4_stage(P, self.box, 4, self.dt, u, u4, un, acc, ws)
        return un, (u2, u3, u4)

    def _acc(self, u):
        b = self.box
        return torch.empty((G.NF, b.nx * b.ny * b.nz), dtype=torch.float64, device=u.device)

    def forward(self, theta, u0):
        """Returns (u_n, checkpoints)."""
        P = self._params(theta)
        acc = self._acc(u0)
        cps = {0: u0.clone()}
        u = u0
        for s in range(self.nsteps):
            u, _ = self.step(P, u, acc)
            if (s + 1) % self.every == 0 and s + 1 < self.nsteps:
                cps[s + 1] = u.clone()
        return u, cps

    def backward(self, theta, cps, ubar_n):
        """Given d J / d u_n, returns (d J / d u_0, d J / d theta)."""
        P = self._params(theta)
        dev = ubar_n.device
        acc = self._acc(ubar_n)
        vws = self._ws_vjp(dev)
        theta_bar = torch.zeros(2, dtype=torch.float64, device=dev)
        ubar = ubar_n.clone()
        out = torch.empty_like(ubar)
        starts = sorted(cps)
        for seg_start in reversed(starts):
            seg_end = min(seg_start + self.every, self.nsteps)
            # re-run the segment, keeping step-start (and stage) states
            states, stages = [cps[seg_start]], []
            u = cps[seg_start]
            for s in range(seg_start, seg_end):
                un, st = self.step(P, u, acc)
                stages.append(st if self.keep_stages else None)
                if s + 1 < seg_end:
                    states.append(un)
                u = un
            for s in reversed(range(seg_end - seg_start)):
                us = states[s]
                st = stages[s]
                if st is None:
                    _, st = self.step(P, us, acc)
                G.rk4_step_vjp(P, self.box, self.dt, us, st[0], st[1], st[2], ubar, out, theta_bar, vws)
                ubar, out = out, ubar
            del states, stages
        return ubar, theta_bar


class Evolve(torch.autograd.Function):
    """u_n = Evolve.apply(theta, u0, traj): theta = (lambda_gb, g2) as a float64
    tensor, u0 the initial state (device, state layout), traj a Trajectory."""

    @staticmethod
    def forward(ctx, theta, u0, traj):
        th = theta.detach().cpu().tolist()
        un, cps = traj.forward(th, u0.detach().contiguous())
        ctx.traj, ctx.th, ctx.cps, ctx.theta_dev = traj, th, cps, theta.device
        return un

    @staticmethod
    def backward(ctx, ubar_n):
        ubar0, theta_bar = ctx.traj.backward(ctx.th, ctx.cps, ubar_n.contiguous())
        return theta_bar.to(ctx.theta_dev), ubar0, None


def shell_phi2(u, mask):
    """Objective sum over shell cells of phi^2 (mask: bool over the interior)."""
    phi = u[25, 3:-3, 3:-3, 3:-3]
    return (phi * phi)[mask].sum()
