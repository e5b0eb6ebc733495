"""Gradients of a trajectory of frozen-ghost RK4 steps (checkpointed adjoint).

Forward: n RK4 steps through libgrf, keeping the state every `every` steps.
Backward: for each segment, last first, the segment is re-run from its
checkpoint keeping every step-start state and the three stage states of every
step, then libgrf's RK4-step adjoint is applied step by step in reverse.  The
couplings theta = (lambda_gb, g2) and the initial state receive gradients.
All arithmetic runs in libgrf's kernels; this module only orders the calls and
owns the buffers.  Buffers are allocated once per trajectory; with frozen
ghosts their ghost cells are set from the initial state once and never change.
"""
from __future__ import annotations

import torch

from . import grf as G


class Trajectory:
    def __init__(self, params: dict, box: G.Box, dt: float, nsteps: int, every: int = 10):
        if box.bc != G.BC_FROZEN:
            raise ValueError("the trajectory adjoint is implemented for frozen ghosts")
        self.pdict, self.box, self.dt, self.nsteps = dict(params), box, float(dt), int(nsteps)
        self.every = max(1, int(every))
        self._vws = None
        self._pool = None     # segment buffers: every x (start, u2, u3, u4) + output
        self._fwd = None      # forward ping-pong buffers
        self._acc = None

    def _params(self, theta):
        return G.make_params(self.pdict, lambda_gb=float(theta[0]), g2=float(theta[1]))

    def _ws_vjp(self, dev):
        # one workspace for the forward stages and the step adjoint: both start
        # with the status word and the derivative record and run one after the
        # other on one stream
        if self._vws is None:
            nbytes = max(G.step_vjp_workspace_bytes(self.box), G.workspace_bytes(self.box))
            self._vws = G.alloc_workspace(nbytes, dev)
        return self._vws

    def _ws_fwd(self, dev):
        return self._ws_vjp(dev)

    def _accbuf(self, dev):
        if self._acc is None:
            b = self.box
            self._acc = torch.empty((G.NF, b.nx * b.ny * b.nz), dtype=torch.float64, device=dev)
        return self._acc

    def step(self, P, u, acc, bufs):
        """One RK4 step from u into bufs = (u2, u3, u4, u_new); bufs carry u's ghosts."""
        ws = self._ws_fwd(u.device)
        u2, u3, u4, un = bufs
        G.rk4_stage(P, self.box, 1, self.dt, u, u, u2, acc, ws)
        G.rk4_stage(P, self.box, 2, self.dt, u, u2, u3, acc, ws)
        G.rk4_stage(P, self.box, 3, self.dt, u, u3, u4, acc, ws)
        G.rk4_stage(P, self.box, 4, self.dt, u, u4, un, acc, ws)
        return un

    def forward(self, theta, u0):
        """Returns (u_n, checkpoints); u_n is a fresh tensor."""
        P = self._params(theta)
        acc = self._accbuf(u0.device)
        if self._fwd is None or self._fwd[0].device != u0.device:
            self._fwd = [u0.clone() for _ in range(5)]
        else:
            for b in self._fwd:
                b.copy_(u0)  # ghosts (and everything) from this initial state
        cps = {0: u0.clone()}
        stage_bufs = self._fwd[:3]
        out_bufs = self._fwd[3:5]
        cur = u0
        for s in range(self.nsteps):
            nxt = out_bufs[s % 2]
            self.step(P, cur, acc, (*stage_bufs, nxt))
            cur = nxt
            if (s + 1) % self.every == 0 and s + 1 < self.nsteps:
                cps[s + 1] = cur.clone()
        return cur.clone(), cps

    def backward(self, theta, cps, ubar_n):
        """Given d J / d u_n, returns (d J / d u_0, d J / d theta)."""
        P = self._params(theta)
        dev = ubar_n.device
        acc = self._accbuf(dev)
        vws = self._ws_vjp(dev)
        theta_bar = torch.zeros(2, dtype=torch.float64, device=dev)
        ubar = ubar_n.clone()
        out = torch.empty_like(ubar)
        u0 = cps[0]
        if self._pool is None or self._pool[0].device != dev:
            self._pool = [u0.clone() for _ in range(4 * self.every + 1)]
        else:
            for b in self._pool:
                b.copy_(u0)
        for seg_start in reversed(sorted(cps)):
            seg_end = min(seg_start + self.every, self.nsteps)
            nseg = seg_end - seg_start
            # re-run the segment: step k starts from starts[k], keeps its stage states
            starts = [cps[seg_start]]
            stages = []
            for k in range(nseg):
                u2, u3, u4, un = self._pool[4 * k:4 * k + 4]
                self.step(P, starts[k], acc, (u2, u3, u4, un))
                stages.append((u2, u3, u4))
                starts.append(un)
            for k in reversed(range(nseg)):
                u2, u3, u4 = stages[k]
                G.rk4_step_vjp(P, self.box, self.dt, starts[k], u2, u3, u4, ubar, out, theta_bar, vws)
                ubar, out = out, ubar
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
