"""PyTorch autograd for the final positions of a PD trajectory as a function of
the per-element stiffness gamma_s (argument marshalling only: the trajectory,
its checkpoints and the discrete adjoint run in libvhpd).

    traj = Trajectory(ctx, X, tets, gamma_v, mass, pinned, gravity, dt,
                      pd_iters=10, n_subdomains=8, frames=30, ckpt_every=5)
    x = traj(gamma_s)            # [nv, 3] float64 tensor, from rest
    loss = 0.5 * ((x - target) ** 2).sum()
    loss.backward()              # gamma_s.grad via vh_mesh_adjoint_backward

The stiffness enters the global matrix, so a forward at a new gamma_s
refactors it (vh_mesh_refactor: host FP64 numeric factorization over the
structure of the first prefactor); a forward at the gamma_s already factored
reuses the factorization.  One trajectory holds one set of checkpoints (those of its
latest forward); the backward of an earlier output replays that output's
forward first, so every gradient belongs to its own gamma_s.
"""

from __future__ import annotations

import numpy as np
import torch

from . import vhpd


class _TrajectoryFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma_s, traj):
        gs = gamma_s.detach().cpu().numpy().astype(np.float64)
        xf = traj._run(gs)
        ctx.traj, ctx.gamma_s, ctx.generation = traj, gs, traj.generation
        return torch.as_tensor(xf, dtype=torch.float64, device=gamma_s.device)

    @staticmethod
    def backward(ctx, grad_x):
        traj = ctx.traj
        if traj.generation != ctx.generation:       # a later forward replaced the checkpoints
            traj._run(ctx.gamma_s)
            ctx.generation = traj.generation
        g = traj.mesh.adjoint_backward(grad_x.detach().cpu().numpy().astype(np.float64))
        return torch.as_tensor(g, dtype=grad_x.dtype, device=grad_x.device), None


class Trajectory:
    """Final positions after `frames` steps from rest (zero velocity) of one mesh."""

    def __init__(self, ctx: vhpd.Context, X, tets, gamma_v, mass, pinned, gravity, dt, pd_iters=10,
                 n_subdomains=8, frames=30, ckpt_every=5, refine_steps=0):
        self.mesh = vhpd.Mesh(ctx, X, tets)
        self.gamma_v = np.ascontiguousarray(gamma_v, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.pinned = np.ascontiguousarray(pinned, dtype=np.uint8)
        self.gravity = np.ascontiguousarray(gravity, dtype=np.float64)
        self.dt, self.pd_iters = float(dt), int(pd_iters)
        self.n_subdomains, self.refine_steps = int(n_subdomains), int(refine_steps)
        self.frames, self.ckpt_every = int(frames), int(ckpt_every)
        self.X = self.mesh.X
        self.generation = 0          # forwards run so far (each replaces the checkpoints)
        self._factored_gs = None     # the gamma_s of the current factorization

    def _run(self, gamma_s):
        m = self.mesh
        if self._factored_gs is None:
            m.set_params(gamma_s, self.gamma_v, self.mass, self.pinned, self.gravity, self.dt, self.pd_iters)
            m.prefactor(self.n_subdomains, self.refine_steps)
            self._factored_gs = np.array(gamma_s, dtype=np.float64)
        elif not np.array_equal(self._factored_gs, gamma_s):
            m.refactor(gamma_s, self.gamma_v)      # same structure, new factor values
            self._factored_gs = np.array(gamma_s, dtype=np.float64)
        self.generation += 1
        return m.adjoint_forward(self.X, np.zeros_like(self.X), self.frames, self.ckpt_every)

    def __call__(self, gamma_s: torch.Tensor) -> torch.Tensor:
        return _TrajectoryFn.apply(gamma_s, self)

    def close(self):
        self.mesh.close()
