"""Differentiable PM forward model over the C ABI (host loop only; every step of the
forward and reverse passes runs in the library's kernels).

Forward map (Newtonian): white noise w -> Zel'dovich (pos, mom) at a_0 ->
leapfrog cycles to a_n (force at a_j, kick, drift) -> CIC counting density ->
binned P(k).  The final closing half-kick is omitted: it does not change the
positions, so P(k) is unaffected.

Reverse pass: ``pk_adjoint`` gives dL/dx_n from dL/dP; then, segment by segment
from the end, the forward cycles of the segment are recomputed from a checkpoint
of (pos, mom) taken every ``ckpt_every`` cycles, keeping each cycle's input
positions and force meshes, and ``pm_step_adjoint`` pulls the cotangents back
through the cycles in reverse order; ``pm_ic_zeldovich_adjoint`` finally maps
them onto the noise.  Memory: n/ckpt_every checkpoints of (pos, mom) plus one
segment's positions and force meshes.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import (FIDUCIAL, ICParams, PM_GRAD_SPECTRAL, Plan, StepParams, kdk_factors, newton_params, pk_adjoint,
               pk_estimate, pm_deposit, pm_ic_zeldovich, pm_ic_zeldovich_adjoint, pm_step, pm_step_adjoint)

__all__ = ["Schedule", "ForwardTape", "forward", "backward", "PowerSpectrumModel", "power_spectrum_model"]


@dataclass
class Schedule:
    """Leapfrog cycles of a run: cycle j has force at a_j, kick K2(j-1) + K1(j) and
    drift Dr(a_j, a_{j+1})."""
    a_steps: list
    cosmo: object = FIDUCIAL
    grad: int = PM_GRAD_SPECTRAL

    def cycles(self):
        out = []
        k2_prev = 0.0
        for j in range(len(self.a_steps) - 1):
            k1, dr, k2 = kdk_factors(self.a_steps[j], self.a_steps[j + 1], self.cosmo)
            out.append(StepParams(kick=k2_prev + k1, drift=dr, solve=newton_params(self.cosmo, self.grad)))
            k2_prev = k2
        return out


@dataclass
class ForwardTape:
    plan: Plan
    ic: ICParams
    steps: list          # StepParams per cycle
    n_bins: int
    ckpt_every: int
    checkpoints: dict    # cycle index -> (pos, mom) before that cycle
    pos_final: torch.Tensor


def forward(plan: Plan, noise: torch.Tensor, ic: ICParams, schedule: Schedule, n_bins: int, ckpt_every: int = 5):
    """Run the forward model; returns ((k_mean, pk, n_modes), tape)."""
    if ckpt_every < 1:
        raise ValueError("ckpt_every must be >= 1")
    n = plan.n
    pos = torch.empty((3, n ** 3), dtype=plan.dtype, device=plan.device)
    mom = torch.empty_like(pos)
    disp = plan.mesh(3)
    pm_ic_zeldovich(plan, noise, ic, disp, pos, mom)
    del disp
    steps = schedule.cycles()
    force = plan.mesh(3)
    ckpts = {}
    for j, st in enumerate(steps):
        if j % ckpt_every == 0:
            ckpts[j] = (pos.clone(), mom.clone())
        pm_step(plan, pos, mom, st, force)
    delta = pm_deposit(plan, pos)
    k, pk, cnt = pk_estimate(plan, delta, n_bins)
    return (k, pk, cnt), ForwardTape(plan, ic, steps, n_bins, ckpt_every, ckpts, pos)


def backward(tape: ForwardTape, dpk: torch.Tensor) -> torch.Tensor:
    """dL/dnoise for the cotangent dpk = dL/dP (device float64 [n_bins]).  Consumes
    the tape (its checkpoints are released as the reverse pass passes them)."""
    plan = tape.plan
    lam_pos = pk_adjoint(plan, tape.pos_final, tape.n_bins, dpk.detach().to(torch.float64).contiguous())
    tape.pos_final = None
    lam_mom = torch.zeros_like(lam_pos)
    n3 = plan.n ** 3
    scratch = torch.empty(3 * n3, dtype=plan.dtype, device=plan.device)
    nsteps = len(tape.steps)
    for s0 in reversed(range(0, nsteps, tape.ckpt_every)):
        s1 = min(s0 + tape.ckpt_every, nsteps)
        pos, mom = tape.checkpoints.pop(s0)
        xs, fs = [], []
        for j in range(s0, s1):
            xs.append(pos.clone())
            f = plan.mesh(3)
            pm_step(plan, pos, mom, tape.steps[j], f)
            fs.append(f)
        del pos, mom
        for j in reversed(range(s0, s1)):
            pm_step_adjoint(plan, xs[j - s0], tape.steps[j], lam_pos, lam_mom, force=fs[j - s0],
                            mesh_scratch=scratch)
            xs[j - s0] = fs[j - s0] = None
    return pm_ic_zeldovich_adjoint(plan, tape.ic, lam_pos, lam_mom)


class PowerSpectrumModel(torch.autograd.Function):
    """pk = P(k) of the forward model at a_n, differentiable with respect to the
    noise field through the hand-written adjoint."""

    @staticmethod
    def forward(ctx, noise, plan, ic, schedule, n_bins, ckpt_every):
        (_, pk, _), tape = forward(plan, noise.detach().contiguous(), ic, schedule, n_bins, ckpt_every)
        ctx.tape = tape
        return pk

    @staticmethod
    def backward(ctx, dpk):
        g = backward(ctx.tape, dpk)
        ctx.tape = None
        return g, None, None, None, None, None


def power_spectrum_model(noise, plan: Plan, ic: ICParams, schedule: Schedule, n_bins: int, ckpt_every: int = 5):
    return PowerSpectrumModel.apply(noise, plan, ic, schedule, n_bins, ckpt_every)
