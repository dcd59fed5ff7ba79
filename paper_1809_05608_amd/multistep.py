"""Consecutive implicit transport steps with a per-step checkpointed adjoint.

Host-side sequencing over the C ABI only (every arithmetic step runs in libtm):

* forward: for s = 1..S, psi^s = step(psi^{s-1}; theta_s) by tm_newton_step, keeping one
  checkpoint psi^s per step;
* reverse, for J = sum_s L_N(psi^s) (the number leaving the outer surface, eq. a62):
  lambda_s = dL/dpsi^s + mu_{s+1} (tm_luminosity_seed with `add`), J_s^T mu_s = lambda_s and the
  step's parameter gradients (tm_adjoint_step at the checkpoint psi^s), with dJ/dpsi^0 = mu_1.

The inputs of a step are produced by a callback `fields_at(s)` so that a caller can
regenerate them instead of holding every step's opacities in memory.
"""
from __future__ import annotations

from typing import Callable, List, Optional

import torch

from .tm import Context, DeviceFields


def forward(ctx: Context, fields_at: Callable[[int], DeviceFields], psi0: torch.Tensor, steps: int,
            max_iter: int = 30, rtol: float = 1e-12, checkpoints: Optional[List[torch.Tensor]] = None):
    """Run `steps` implicit steps from psi0; returns (checkpoints psi^1..psi^S, per-step stats)."""
    cps = checkpoints if checkpoints is not None else []
    stats = []
    prev = psi0
    for s in range(steps):
        f = fields_at(s)
        psi = cps[s] if s < len(cps) else torch.empty_like(psi0)
        psi.copy_(prev)                                  # initial guess psi^n
        _, st = ctx.newton_step(f, prev, psi, max_iter, rtol)
        if s >= len(cps):
            cps.append(psi)
        stats.append(st)
        prev = psi
    return cps, stats


def adjoint(ctx: Context, fields_at: Callable[[int], DeviceFields], psi0: torch.Tensor,
            checkpoints: List[torch.Tensor],
            on_grad: Optional[Callable[[int, torch.Tensor, dict], None]] = None,
            want=("kappa_a", "eta", "kappa_s")) -> torch.Tensor:
    """dJ/dpsi^0 of J = sum_s L_N(psi^s); `on_grad(s, mu_s, grads_s)` sees each step's adjoint and
    parameter gradients (buffers are reused between steps: copy what must be kept)."""
    S = len(checkpoints)
    seed = torch.empty_like(psi0)
    mu = torch.empty_like(psi0)
    mu_next = None
    g = {n: torch.empty_like(psi0) for n in want}
    gamp = None
    for s in range(S - 1, -1, -1):
        f = fields_at(s)
        if gamp is None:
            gamp = torch.empty_like(f.nes_amp)
        ctx.luminosity_seed(f, seed, add=mu_next)
        psi_n = checkpoints[s - 1] if s > 0 else psi0
        ctx.adjoint_step(f, psi_n, checkpoints[s], seed, mu, g.get("kappa_a"), g.get("eta"), g.get("kappa_s"), gamp)
        if on_grad is not None:
            on_grad(s, mu, dict(g, nes_amp=gamp))
        if mu_next is None:
            mu_next = torch.empty_like(psi0)
        mu, mu_next = mu_next, mu                        # mu_next now holds mu_s
    return mu_next
