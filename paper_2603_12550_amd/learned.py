"""Pipeline of the learned reduced step (include/vds_mlp.h): trajectories of the
particle scheme, a shared POD basis, training pairs, training and the checked
rollout.  Every computation is a call into libvds; this module only orders the
calls and moves tensors between them.
"""
from __future__ import annotations

import numpy as np
import torch

from ._vds import Context, Mlp


def run_states(ctx: Context, q0: torch.Tensor, nsteps: int, every: int):
    """Plain-scheme states q(0), q(every), ..., q(nsteps) (clones)."""
    q = q0.clone()
    out = [q.clone()]
    for _ in range(0, nsteps, every):
        ctx.step(q, nsteps=every)
        out.append(q.clone())
    return out


def snapshot_matrix(states) -> torch.Tensor:
    """Column-major snapshot matrix (ncols, 3P): columns (l, k) = bond k of state l."""
    nb, P, _ = states[0].shape
    return torch.stack(states).reshape(len(states) * nb, 3 * P).contiguous()


def reduced_trajectory(ctx: Context, U: torch.Tensor, q0: torch.Tensor, nsteps: int) -> torch.Tensor:
    """p(0..nsteps) = U^T q(t) of the plain scheme, rows of nb R."""
    R = U.shape[0]
    traj = torch.empty((nsteps + 1, ctx.nb * R), dtype=torch.float32, device=q0.device)
    q = q0.clone()
    traj[0] = ctx.pod_project(U, q).reshape(-1)
    for n in range(nsteps):
        ctx.step(q, nsteps=1)
        traj[n + 1] = ctx.pod_project(U, q).reshape(-1)
    return traj


def training_set(mlp: Mlp, trajectories):
    """[(traj, log_rate), ...] -> concatenated inputs X and increments T."""
    Xs, Ts = [], []
    for traj, log_rate in trajectories:
        X, T = mlp.make_pairs(traj, log_rate)
        Xs.append(X)
        Ts.append(T)
    return torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous()


def train(mlp: Mlp, X: torch.Tensor, T: torch.Tensor, epochs: int, batch: int, lr: float, seed: int = 0,
          input_noise: float = 0.0, lr_final=None):
    """Fits the scaling, then `epochs` passes in seeded random order (with input
    noise of `input_noise` increment standard deviations, vds_mlp_set_input_noise);
    returns the losses.  With `lr_final` the step size falls from `lr` to
    `lr_final` along a half cosine over the epochs, else it stays at `lr`."""
    mlp.fit_scaling(X, T)
    mlp.set_input_noise(input_noise, seed)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for e in range(epochs):
        rate = lr
        if lr_final is not None and epochs > 1:
            rate = lr_final + (lr - lr_final) * 0.5 * (1.0 + np.cos(np.pi * e / (epochs - 1)))
        order = torch.randperm(X.shape[0], generator=gen).to(torch.int32).to(X.device)
        losses.append(mlp.train_epoch(X, T, batch, rate, order=order))
    return np.array(losses)
