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
through the cycles in reverse order; ``pm_ic_zeldovich_adjoint`` (or
``pm_ic_2lpt_adjoint`` for the second-order start, ``Schedule.lpt_order = 2``)
finally maps them onto the noise.  Memory: n/ckpt_every checkpoints of (pos, mom) plus one
segment's positions and force meshes.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import (FIDUCIAL, ICParams, PM_GRAD_SPECTRAL, PM_STEP_DENSITY_READY, PM_STEP_DEPOSIT_NEXT, Plan, StepParams,
               leapfrog_factors, newton_params, pk_adjoint,
               pk_estimate, pm_deposit, pm_ic_2lpt, pm_ic_2lpt_adjoint, pm_ic_zeldovich, pm_ic_zeldovich_adjoint,
               pm_step, pm_step_adjoint)

__all__ = ["Schedule", "ForwardTape", "forward", "backward", "GraphedModel", "PowerSpectrumModel",
           "power_spectrum_model"]


@dataclass
class Schedule:
    """Leapfrog cycles of a run: cycle j has force at a_j, kick K2(j-1) + K1(j) and
    drift Dr(a_j, a_{j+1})."""
    a_steps: list
    cosmo: object = FIDUCIAL
    grad: int = PM_GRAD_SPECTRAL
    lpt_order: int = 1   # 1: Zel'dovich ICs, 2: second-order (2LPT) ICs

    def cycles(self):
        kick, drift = leapfrog_factors(self.a_steps, self.cosmo)
        return [StepParams(kick=kick[j], drift=drift[j], solve=newton_params(self.cosmo, self.grad))
                for j in range(len(self.a_steps) - 1)]


@dataclass
class ForwardTape:
    plan: Plan
    ic: ICParams
    steps: list          # StepParams per cycle
    n_bins: int
    ckpt_every: int
    checkpoints: dict    # cycle index -> (pos, mom) before that cycle
    pos_final: torch.Tensor
    noise: torch.Tensor = None   # kept for the 2LPT adjoint (the set is quadratic in it)
    lpt_order: int = 1


def _chained(st: StepParams, first: bool, last: bool) -> StepParams:
    """st as one cycle of a chain of consecutive cycles on one plan: every cycle but the
    last leaves the density of its drifted positions for the next (PM_STEP_DEPOSIT_NEXT,
    deposited by the fused gather kernel where it applies), every cycle but the first
    starts from it (PM_STEP_DENSITY_READY)."""
    fl = (0 if first else PM_STEP_DENSITY_READY) | (0 if last else PM_STEP_DEPOSIT_NEXT)
    return StepParams(kick=st.kick, drift=st.drift, solve=st.solve, flags=fl)


def forward(plan: Plan, noise: torch.Tensor, ic: ICParams, schedule: Schedule, n_bins: int, ckpt_every: int = 5):
    """Run the forward model; returns ((k_mean, pk, n_modes), tape)."""
    if ckpt_every < 1:
        raise ValueError("ckpt_every must be >= 1")
    if schedule.lpt_order not in (1, 2):
        raise ValueError("lpt_order must be 1 or 2")
    n = plan.n
    pos = torch.empty((3, n ** 3), dtype=plan.dtype, device=plan.device)
    mom = torch.empty_like(pos)
    disp = plan.mesh(3)
    (pm_ic_zeldovich if schedule.lpt_order == 1 else pm_ic_2lpt)(plan, noise, ic, disp, pos, mom)
    del disp
    steps = schedule.cycles()
    force = plan.mesh(3)
    ckpts = {}
    for j, st in enumerate(steps):
        if j % ckpt_every == 0:
            ckpts[j] = (pos.clone(), mom.clone())
        pm_step(plan, pos, mom, _chained(st, j == 0, j == len(steps) - 1), force)
    delta = pm_deposit(plan, pos)
    k, pk, cnt = pk_estimate(plan, delta, n_bins)
    return (k, pk, cnt), ForwardTape(plan, ic, steps, n_bins, ckpt_every, ckpts, pos,
                                     noise if schedule.lpt_order == 2 else None, schedule.lpt_order)


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
            pm_step(plan, pos, mom, _chained(tape.steps[j], j == s0, j == s1 - 1), f)
            fs.append(f)
        del pos, mom
        for j in reversed(range(s0, s1)):
            pm_step_adjoint(plan, xs[j - s0], tape.steps[j], lam_pos, lam_mom, force=fs[j - s0],
                            mesh_scratch=scratch)
            xs[j - s0] = fs[j - s0] = None
    if tape.lpt_order == 2:
        return pm_ic_2lpt_adjoint(plan, tape.noise, tape.ic, lam_pos, lam_mom)
    return pm_ic_zeldovich_adjoint(plan, tape.ic, lam_pos, lam_mom)


class GraphedModel:
    """The same forward model and reverse pass with every buffer allocated once and
    both passes captured as HIP graphs (``torch.cuda.CUDAGraph``), for sizes where
    launch and host overheads dominate (e.g. 128^3).  ``forward(noise)`` returns P(k);
    ``backward(dpk)`` returns dL/dnoise for the last forward.  Memory is that of the
    eager model with every checkpoint and one segment resident."""

    def __init__(self, plan: Plan, ic: ICParams, schedule: Schedule, n_bins: int, ckpt_every: int = 5):
        self.plan, self.ic, self.n_bins, self.ckpt = plan, ic, n_bins, ckpt_every
        self.steps = schedule.cycles()
        self.lpt_order = schedule.lpt_order
        n3 = plan.n ** 3
        dev, dt = plan.device, plan.dtype
        part = lambda: torch.empty((3, n3), dtype=dt, device=dev)  # noqa: E731
        self.noise = plan.mesh()
        self.pos, self.mom, self.disp, self.force = part(), part(), plan.mesh(3), plan.mesh(3)
        self.delta = plan.mesh()
        self.starts = list(range(0, len(self.steps), ckpt_every))
        self.ckpts = {s0: (part(), part()) for s0 in self.starts}
        self.seg_x = [part() for _ in range(ckpt_every)]
        self.seg_f = [plan.mesh(3) for _ in range(ckpt_every)]
        self.wpos, self.wmom = part(), part()
        self.lam_pos, self.lam_mom = part(), part()
        self.scratch = torch.empty(3 * n3, dtype=dt, device=dev)
        self.dpk = torch.zeros(n_bins, dtype=torch.float64, device=dev)
        self.lam_noise = plan.mesh()
        self.ic_scratch = plan.mesh(9) if self.lpt_order == 2 else None
        self.out = None
        self.g_fwd = self.g_bwd = None

    def _forward(self):
        (pm_ic_zeldovich if self.lpt_order == 1 else pm_ic_2lpt)(self.plan, self.noise, self.ic, self.disp, self.pos,
                                                                  self.mom)
        for j, st in enumerate(self.steps):
            if j in self.ckpts:
                self.ckpts[j][0].copy_(self.pos)
                self.ckpts[j][1].copy_(self.mom)
            pm_step(self.plan, self.pos, self.mom, _chained(st, j == 0, j == len(self.steps) - 1), self.force)
        pm_deposit(self.plan, self.pos, self.delta)
        self.out = pk_estimate(self.plan, self.delta, self.n_bins)

    def _backward(self):
        plan = self.plan
        pk_adjoint(plan, self.pos, self.n_bins, self.dpk, self.lam_pos)
        self.lam_mom.zero_()
        nsteps = len(self.steps)
        for s0 in reversed(self.starts):
            s1 = min(s0 + self.ckpt, nsteps)
            self.wpos.copy_(self.ckpts[s0][0])
            self.wmom.copy_(self.ckpts[s0][1])
            for j in range(s0, s1):
                self.seg_x[j - s0].copy_(self.wpos)
                pm_step(plan, self.wpos, self.wmom, _chained(self.steps[j], j == s0, j == s1 - 1),
                        self.seg_f[j - s0])
            for j in reversed(range(s0, s1)):
                pm_step_adjoint(plan, self.seg_x[j - s0], self.steps[j], self.lam_pos, self.lam_mom,
                                force=self.seg_f[j - s0], mesh_scratch=self.scratch)
        if self.lpt_order == 2:
            pm_ic_2lpt_adjoint(plan, self.noise, self.ic, self.lam_pos, self.lam_mom, self.ic_scratch, self.lam_noise)
        else:
            pm_ic_zeldovich_adjoint(plan, self.ic, self.lam_pos, self.lam_mom, self.disp, self.lam_noise)

    def capture(self):
        """Warm both passes eagerly, then capture each into its own graph."""
        self._forward()
        self._backward()
        torch.cuda.synchronize()
        self.g_fwd = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g_fwd):
            self._forward()
        self.g_bwd = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g_bwd):
            self._backward()
        return self

    def forward(self, noise):
        self.noise.copy_(noise.reshape(self.noise.shape))
        self.g_fwd.replay()
        return self.out[1]

    def __del__(self):
        # the captured graphs go before the plan and buffers they were captured from
        self.g_fwd = self.g_bwd = None

    def backward(self, dpk):
        self.dpk.copy_(dpk)
        self.g_bwd.replay()
        return self.lam_noise


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
