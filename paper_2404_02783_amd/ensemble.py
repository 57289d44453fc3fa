"""Batched ensembles of independent periodic boxes with uneven meshes (host loop
over the C ABI; every step runs in the library's kernels).

Boxes of equal mesh size form one batched plan, so each kernel of a leapfrog cycle
is one launch per size group whatever the number of boxes.  The whole run of every
group -- Zel'dovich ICs, the leapfrog cycles and the final P(k) -- can be captured
once into a single HIP graph (``torch.cuda.CUDAGraph`` is HIP's graph API on ROCm)
and replayed, which removes the per-launch host cost that dominates small boxes.
Inputs (noise fields) are device-resident before the run.

Not part of the paper's pipeline: ensembles of independent realisations are what
the paper's ensemble error bars on the scale-dependent bias would need (Sec. 5.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import (FIDUCIAL, ICParams, PM_PK_EH98, PM_STEP_DENSITY_READY, PM_STEP_DEPOSIT_NEXT, Plan, StepParams,
               kdk_factors, newton_params, pk_estimate, pm_deposit, pm_ic_zeldovich, pm_noise_fix, pm_step,
               power_eh98_amplitude)
from .sim import log_steps
from .tuning import tune

__all__ = ["Group", "Ensemble", "default_groups", "schedule", "run_sequential"]


@dataclass
class Group:
    n: int                 # mesh cells per axis (= particles per axis)
    box: float             # Mpc/h
    seeds: list            # one noise seed per box
    n_bins: int = 0        # P(k) bins (default N/2: width one fundamental mode)

    def bins(self) -> int:
        return self.n_bins or self.n // 2


def default_groups(first_seed: int = 100):
    """64 boxes at a fixed cell size of 7.8125 Mpc/h: 16 x 64^3, 24 x 128^3,
    16 x 192^3, 8 x 256^3, seeds first_seed .. first_seed + 63."""
    spec = [(64, 500.0, 16), (128, 1000.0, 24), (192, 1500.0, 16), (256, 2000.0, 8)]
    out, s = [], first_seed
    for n, box, count in spec:
        out.append(Group(n, box, list(range(s, s + count))))
        s += count
    return out


@dataclass
class _State:
    group: Group
    plan: Plan
    noise: torch.Tensor
    pos: torch.Tensor
    mom: torch.Tensor
    force: torch.Tensor
    disp: torch.Tensor
    delta: torch.Tensor
    out: tuple = field(default=None)
    tuning: tuple = field(default=None)
    pk_out: tuple = field(default=None)
    stream: object = field(default=None)


def schedule(a_start=0.02, a_end=1.0, n_steps=30, n_s=0.965, sigma8=0.81, cosmo=FIDUCIAL):
    """(a_steps, IC parameters, StepParams per leapfrog cycle) of an ensemble run:
    EH98 no-wiggle ICs normalised to sigma8 at a = 1, n_steps log-spaced cycles."""
    a_steps = log_steps(a_start, a_end, n_steps)
    ic = ICParams(pk_kind=PM_PK_EH98, amp=power_eh98_amplitude(n_s, sigma8, cosmo), index=n_s, a_init=a_start,
                  a_norm=1.0, cosmo=cosmo)
    cycles = []
    k2_prev = 0.0
    for j in range(n_steps):
        k1, dr, k2 = kdk_factors(a_steps[j], a_steps[j + 1], cosmo)
        cycles.append(StepParams(kick=k2_prev + k1, drift=dr, solve=newton_params(cosmo)))
        k2_prev = k2
    return a_steps, ic, cycles


class Ensemble:
    """All groups of an ensemble with their device buffers.  ``noise_fn(n, seed)``
    returns the host white-noise field of one box (float64 numpy [n, n, n]).

    ``paired_fixed``: every seed gives two boxes, 2j and 2j + 1, run from the
    paired-and-fixed noise of that seed (fixed mode amplitudes; the partner's field
    negated); ``paired_power_spectra`` averages each pair.  ``autotune``: each size
    group's FFT launch shapes are measured for its batch (or read from
    ``tuning_cache``, a JSON file) before the run."""

    def __init__(self, groups, noise_fn, a_start=0.02, a_end=1.0, n_steps=30, dtype=torch.float32, device=None,
                 n_s=0.965, sigma8=0.81, cosmo=FIDUCIAL, paired_fixed: bool = False, autotune: bool = False,
                 tuning_cache: str | None = None, concurrent: bool = False):
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.dtype = dtype
        self.paired_fixed = paired_fixed
        self.a_steps, self.ic, self.cycles = schedule(a_start, a_end, n_steps, n_s, sigma8, cosmo)
        self.states = []
        for g in groups:
            reps = 2 if paired_fixed else 1
            plan = Plan(g.n, g.box, dtype, self.device, batch=reps * len(g.seeds))
            noise = torch.stack([torch.from_numpy(noise_fn(g.n, s)) for s in g.seeds for _ in range(reps)])
            noise = noise.to(dtype).to(self.device).contiguous()
            if paired_fixed:
                pm_noise_fix(plan, noise, 2, out=noise)
            st = _State(g, plan, noise, plan.particles(), plan.particles(), plan.mesh(3), plan.mesh(3), plan.mesh())
            if autotune:   # FFT launch shapes measured for this group's batch (delta as scratch)
                st.tuning = tune(plan, tuning_cache, mesh_scratch=st.delta)
            shape = (plan.batch, g.bins())
            st.pk_out = (torch.empty(shape, dtype=torch.float64, device=self.device),
                         torch.empty(shape, dtype=torch.float64, device=self.device),
                         torch.empty(shape, dtype=torch.int64, device=self.device))
            st.stream = torch.cuda.Stream(device=self.device) if concurrent else None
            self.states.append(st)
        self.concurrent = concurrent
        self.graph = None

    def _run_group(self, st):
        """The whole run of one group, in order, on the current stream."""
        pm_ic_zeldovich(st.plan, st.noise, self.ic, st.disp, st.pos, st.mom)
        for j, cyc in enumerate(self.cycles):
            fl = (PM_STEP_DENSITY_READY if j > 0 else 0) | (PM_STEP_DEPOSIT_NEXT if j + 1 < len(self.cycles) else 0)
            pm_step(st.plan, st.pos, st.mom, StepParams(kick=cyc.kick, drift=cyc.drift, solve=cyc.solve, flags=fl),
                    st.force)
        pm_deposit(st.plan, st.pos, st.delta)
        pk_estimate(st.plan, st.delta, st.group.bins(), out=st.pk_out)
        st.out = st.pk_out

    def run(self):
        """Issue the whole run of every group: ICs, the leapfrog cycles (without the
        final half kick) and P(k) at a_end.  On the current stream, cycle by cycle
        over the groups; with ``concurrent`` each group runs on a stream of its own
        (forked from and joined back into the current stream), so that the groups'
        kernels may overlap on the GPU."""
        if self.concurrent:
            cur = torch.cuda.current_stream()
            for st in self.states:
                st.stream.wait_stream(cur)
                with torch.cuda.stream(st.stream):
                    self._run_group(st)
            for st in self.states:
                cur.wait_stream(st.stream)
            return
        for st in self.states:
            pm_ic_zeldovich(st.plan, st.noise, self.ic, st.disp, st.pos, st.mom)
        for j, cyc in enumerate(self.cycles):
            # each cycle leaves the density of the drifted positions for the next one
            fl = (PM_STEP_DENSITY_READY if j > 0 else 0) | (PM_STEP_DEPOSIT_NEXT if j + 1 < len(self.cycles) else 0)
            c = StepParams(kick=cyc.kick, drift=cyc.drift, solve=cyc.solve, flags=fl)
            for st in self.states:
                pm_step(st.plan, st.pos, st.mom, c, st.force)
        for st in self.states:
            pm_deposit(st.plan, st.pos, st.delta)
            pk_estimate(st.plan, st.delta, st.group.bins(), out=st.pk_out)
            st.out = st.pk_out   # [boxes, bins], also for a one-box group

    def capture(self):
        """Capture run() into one HIP graph (after one eager warm-up run)."""
        self.run()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def power_spectra(self):
        """[(k_mean, P, n_modes) per group], each [boxes, bins] on the device."""
        return [st.out for st in self.states]

    def paired_power_spectra(self):
        """For a paired-and-fixed ensemble: [(k_mean, P averaged over each pair,
        n_modes) per group], each [seeds, bins]."""
        if not self.paired_fixed:
            raise ValueError("not a paired-and-fixed ensemble")
        return [(k[0::2], 0.5 * (p[0::2] + p[1::2]), c[0::2]) for k, p, c in self.power_spectra()]


def run_sequential(groups, noise_fn, a_start=0.02, a_end=1.0, n_steps=30, dtype=torch.float32, device=None,
                   plans=None, noises=None):
    """Reference: every box on its own single-box plan, one after another, eager
    launches.  ``plans``/``noises`` (dicts keyed by (n, box) and seed) may hold
    pre-built plans and device noise so that only the run itself is timed.
    Returns [P per group, each [boxes, bins]]."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    _, ic, cycles = schedule(a_start, a_end, n_steps)
    outs = []
    for g in groups:
        plan = plans[(g.n, g.box)] if plans else Plan(g.n, g.box, dtype, dev)
        pos, mom = plan.particles(), plan.particles()
        force, disp = plan.mesh(3), plan.mesh(3)
        delta = plan.mesh()
        ps = []
        for s in g.seeds:
            noise = noises[s] if noises else torch.from_numpy(noise_fn(g.n, s)).to(dtype).to(dev)
            pm_ic_zeldovich(plan, noise, ic, disp, pos, mom)
            for j, cyc in enumerate(cycles):
                fl = (PM_STEP_DENSITY_READY if j > 0 else 0) | (PM_STEP_DEPOSIT_NEXT if j + 1 < len(cycles) else 0)
                pm_step(plan, pos, mom, StepParams(kick=cyc.kick, drift=cyc.drift, solve=cyc.solve, flags=fl), force)
            pm_deposit(plan, pos, delta)
            ps.append(pk_estimate(plan, delta, g.bins())[1])
        outs.append(torch.stack(ps))
    return outs
