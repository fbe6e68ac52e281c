"""Differentiable rollout with checkpoint-every-K recomputation.

``rollout(level, theta, h0, g0, n_steps, every)`` runs ``n_steps`` steps of a
fully periodic level with the body-force field ``theta`` and returns the final
smoke scalar ``s = sum_i g_i``.  Gradients with respect to theta and the
initial populations come from the hand-written adjoint step of libcslbm
(``cslbm_adjoint_step``); only every ``every``-th state is kept during the
forward pass and each segment is recomputed with ``cslbm_step_store`` in the
backward pass.  Tensors are dense: theta [3][N], h0 [27][N] shifted
populations f - w, g0 [7][N].

``MultiscaleRollout`` does the same for the reference steps of a hierarchy
(Algorithm 1 over a chain of finer scales): ``forward(n_ref)`` keeps every
``every``-th set of scale states, ``backward`` recomputes each segment one
reference step at a time and applies ``cslbm_multiscale_adjoint_step`` in
reverse, giving dL/d(initial state) of every scale from dL/d(final state).
"""
from __future__ import annotations

import dataclasses

import torch

from .level import Level


def _dense_to_plane(lev: Level, x: torch.Tensor, rows: int) -> torch.Tensor:
    out = torch.zeros(rows, lev.plane, dtype=torch.float32, device=lev.device)
    out[:, : lev.n] = x.reshape(rows, lev.n)
    return out


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, h0, g0, lev: Level, n_steps: int, every: int):
        assert lev.force is not None and lev.g is not None, "level needs force and scalar buffers"
        lev.force.reshape(3, lev.plane)[:, : lev.n] = theta.detach().reshape(3, lev.n)
        lev.set_populations(h0.detach(), g0.detach(), shifted=True)
        checkpoints = []
        done = 0
        while done < n_steps:
            k = min(every, n_steps - done)
            checkpoints.append((done, k, lev.f.clone(), lev.g.clone()))
            lev.step(k)
            done += k
        _, _, s = lev.read_macro()
        ctx.lev, ctx.checkpoints = lev, checkpoints
        # the force and parameters of this forward pass: the level may run
        # other rollouts before backward is called
        ctx.theta = theta.detach().reshape(3, lev.n).to(torch.float32).clone()
        ctx.params = dataclasses.replace(lev.params)
        return s.clone()

    @staticmethod
    def backward(ctx, grad_s):
        lev: Level = ctx.lev
        saved_force, saved_params = lev.force.clone(), lev.params
        lev.force.reshape(3, lev.plane)[:, : lev.n] = ctx.theta
        lev.set_params(ctx.params)
        try:
            return _Rollout._reverse(ctx, lev, grad_s)
        finally:
            lev.force.copy_(saved_force)
            lev.set_params(saved_params)

    @staticmethod
    def _reverse(ctx, lev: Level, grad_s):
        P = lev.plane
        lam = torch.zeros(27 * P, dtype=torch.float32, device=lev.device)
        lam2 = torch.zeros_like(lam)
        mu = _dense_to_plane(lev, grad_s.detach().reshape(1, -1).expand(7, -1), 7).reshape(-1)
        mu2 = torch.zeros_like(mu)
        dtheta = torch.zeros(3 * P, dtype=torch.float32, device=lev.device)
        every = max((k for _, k, _, _ in ctx.checkpoints), default=1)
        f_buf = [torch.empty_like(lev.f) for _ in range(every - 1)]
        g_buf = [torch.empty_like(lev.g) for _ in range(every - 1)]
        for start, k, f0, g0 in reversed(ctx.checkpoints):
            if k > 1:
                lev.step_store(f0, g0, f_buf[: k - 1], g_buf[: k - 1])
            f_states = [f0] + f_buf[: k - 1]
            g_states = [g0] + g_buf[: k - 1]
            for n in reversed(range(k)):
                lev.adjoint_step(f_states[n], g_states[n], lam, mu, lam2, mu2, dtheta)
                lam, lam2 = lam2, lam
                mu, mu2 = mu2, mu
        n = lev.n
        return (dtheta.reshape(3, P)[:, :n].clone(), lam.reshape(27, P)[:, :n].clone(),
                mu.reshape(7, P)[:, :n].clone(), None, None, None)


def rollout(lev: Level, theta: torch.Tensor, h0: torch.Tensor, g0: torch.Tensor, n_steps: int,
            every: int = 20) -> torch.Tensor:
    return _Rollout.apply(theta, h0, g0, lev, int(n_steps), int(every))


class MultiscaleRollout:
    """Checkpointed reference steps of a hierarchy and their adjoint."""

    def __init__(self, H, every: int = 10):
        self.H = H
        self.every = max(1, int(every))
        self.checkpoints = []
        self.workspace = torch.empty(H.adjoint_workspace_bytes(), dtype=torch.uint8,
                                     device=H.levels[0].device)

    def _states(self):
        return ([lev.f.clone() for lev in self.H.levels],
                [None if lev.g is None else lev.g.clone() for lev in self.H.levels])

    def _restore(self, fs, gs):
        for lev, f, g in zip(self.H.levels, fs, gs):
            lev.f.copy_(f)
            if g is not None:
                lev.g.copy_(g)

    def forward(self, n_ref: int):
        """n_ref reference steps from the scales' current states."""
        self.checkpoints = []
        done = 0
        while done < n_ref:
            k = min(self.every, n_ref - done)
            self.checkpoints.append((k, *self._states()))
            self.H.step(k)
            done += k
        self.final = self._states()

    def backward(self, lam_f, lam_g=None):
        """lam_f[i]: dL/d(final populations of scale i), dense [27][N_i]
        (lam_g[i]: [7][N_i] with a scalar).  Returns the adjoints of the
        initial states in the same form.  The scales are left in their final
        forward state."""
        H = self.H
        scalar = H.levels[0].g is not None
        lam, mu = [], []
        for i, lev in enumerate(H.levels):
            lam.append(_dense_to_plane(lev, lam_f[i], 27).reshape(-1))
            mu.append(_dense_to_plane(lev, lam_g[i], 7).reshape(-1) if scalar else None)
        for k, fs, gs in reversed(self.checkpoints):
            states = [(fs, gs)]
            if k > 1:
                self._restore(fs, gs)
                for _ in range(k - 1):
                    H.step(1)
                    states.append(self._states())
            for f_n, g_n in reversed(states):
                H.adjoint_step(f_n, g_n if scalar else None, lam, mu if scalar else None,
                               self.workspace)
        self._restore(*self.final)
        out_f = [l.reshape(27, lev.plane)[:, : lev.n].clone() for l, lev in zip(lam, H.levels)]
        out_g = ([m.reshape(7, lev.plane)[:, : lev.n].clone() for m, lev in zip(mu, H.levels)]
                 if scalar else None)
        return out_f, out_g
