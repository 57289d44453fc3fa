"""Batched ensembles of independent periodic boxes with uneven meshes (host loop
over the C ABI; every step runs in the library's kernels).

The boxes form one ``Batch`` (pm_batch_*): boxes of equal mesh size and side are a
size group advanced by one launch per kernel whatever the number of boxes, and a
whole run -- Zel'dovich ICs, the leapfrog cycles and the final P(k) -- is a handful of
batch calls per cycle, which can be captured once into a single HIP graph
(``torch.cuda.CUDAGraph`` is HIP's graph API on ROCm) and replayed, removing the
per-launch host cost that dominates small boxes.  Inputs (noise fields) are
device-resident before the run.

Not part of the paper's pipeline: ensembles of independent realisations are what
the paper's ensemble error bars on the scale-dependent bias would need (Sec. 5.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import (FIDUCIAL, Batch, ICParams, PM_PK_EH98, PM_STEP_DENSITY_READY, PM_STEP_DEPOSIT_NEXT, Plan,
               StepParams, leapfrog_factors, newton_params, pk_estimate, pm_batch_ic_zeldovich, pm_batch_pk_estimate,
               pm_batch_step, pm_deposit, pm_ic_zeldovich, pm_noise_fix, pm_step, power_eh98_amplitude)
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
    noise: torch.Tensor    # [boxes, N, N, N]
    pos: torch.Tensor      # [boxes, 3, N^3]
    mom: torch.Tensor
    first: int             # index of the group's first box in the batch
    out: tuple = field(default=None)
    tuning: tuple = field(default=None)


def schedule(a_start=0.02, a_end=1.0, n_steps=30, n_s=0.965, sigma8=0.81, cosmo=FIDUCIAL):
    """(a_steps, IC parameters, StepParams per leapfrog cycle) of an ensemble run:
    EH98 no-wiggle ICs normalised to sigma8 at a = 1, n_steps log-spaced cycles."""
    a_steps = log_steps(a_start, a_end, n_steps)
    ic = ICParams(pk_kind=PM_PK_EH98, amp=power_eh98_amplitude(n_s, sigma8, cosmo), index=n_s, a_init=a_start,
                  a_norm=1.0, cosmo=cosmo)
    kick, drift = leapfrog_factors(a_steps, cosmo)
    cycles = [StepParams(kick=kick[j], drift=drift[j], solve=newton_params(cosmo)) for j in range(n_steps)]
    return a_steps, ic, cycles


class Ensemble:
    """All boxes of an ensemble as one Batch, with their device buffers.
    ``noise_fn(n, seed)`` returns the host white-noise field of one box (float64 numpy
    [n, n, n]).

    ``paired_fixed``: every seed gives two boxes, 2j and 2j + 1, run from the
    paired-and-fixed noise of that seed (fixed mode amplitudes; the partner's field
    negated); ``paired_power_spectra`` averages each pair.  ``autotune``: each size
    group's FFT launch shapes are measured for its batch (or read from
    ``tuning_cache``, a JSON file) before the run.  ``concurrent``: each size group
    runs on a stream of its own inside the batch calls (forked from and joined back
    into the current stream)."""

    def __init__(self, groups, noise_fn, a_start=0.02, a_end=1.0, n_steps=30, dtype=torch.float32, device=None,
                 n_s=0.965, sigma8=0.81, cosmo=FIDUCIAL, paired_fixed: bool = False, autotune: bool = False,
                 tuning_cache: str | None = None, concurrent: bool = False):
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.dtype = dtype
        self.paired_fixed = paired_fixed
        self.concurrent = concurrent
        self.a_steps, self.ic, self.cycles = schedule(a_start, a_end, n_steps, n_s, sigma8, cosmo)
        reps = 2 if paired_fixed else 1
        self.states = []
        n_mesh, sides, first = [], [], 0
        for g in groups:
            nb = reps * len(g.seeds)
            noise = torch.stack([torch.from_numpy(noise_fn(g.n, s)) for s in g.seeds for _ in range(reps)])
            noise = noise.to(dtype).to(self.device).contiguous()
            if paired_fixed:   # setup: a temporary batched plan fixes and pairs the noise
                fix_plan = Plan(g.n, g.box, dtype, self.device, batch=nb)
                pm_noise_fix(fix_plan, noise, 2, out=noise)
                torch.cuda.synchronize()
                del fix_plan
            pos = torch.empty((nb, 3, g.n ** 3), dtype=dtype, device=self.device)
            self.states.append(_State(g, noise, pos, torch.empty_like(pos), first))
            n_mesh += [g.n] * nb
            sides += [g.box] * nb
            first += nb
        self.batch = Batch(n_mesh, sides, dtype, self.device, concurrent=concurrent)
        self.noise = [st.noise[i] for st in self.states for i in range(st.noise.shape[0])]
        self.pos = [st.pos[i] for st in self.states for i in range(st.pos.shape[0])]
        self.mom = [st.mom[i] for st in self.states for i in range(st.mom.shape[0])]
        self.bins = [st.group.bins() for st in self.states for _ in range(st.noise.shape[0])]
        total = sum(self.bins)
        self.pk_out = (torch.empty(total, dtype=torch.float64, device=self.device),
                       torch.empty(total, dtype=torch.float64, device=self.device),
                       torch.empty(total, dtype=torch.int64, device=self.device))
        self.group_tuning = []
        if autotune:   # FFT launch shapes measured for each size group of the batch
            for n, box, cnt, gplan in self.batch.groups():
                scratch = gplan.mesh()
                self.group_tuning.append(((n, box, cnt), tune(gplan, tuning_cache, mesh_scratch=scratch)))
                del scratch
            by_size = {key[:2]: t for key, t in self.group_tuning}
            for st in self.states:
                st.tuning = by_size[(st.group.n, st.group.box)]
        self.graph = None

    def run(self):
        """Issue the whole run of every box: ICs, the leapfrog cycles (without the
        final half kick) and P(k) at a_end, as batch calls on the current stream."""
        pm_batch_ic_zeldovich(self.batch, self.noise, self.ic, self.pos, self.mom)
        for j, cyc in enumerate(self.cycles):
            # each cycle leaves the density of the drifted positions for the next one
            fl = (PM_STEP_DENSITY_READY if j > 0 else 0) | (PM_STEP_DEPOSIT_NEXT if j + 1 < len(self.cycles) else 0)
            pm_batch_step(self.batch, self.pos, self.mom,
                          StepParams(kick=cyc.kick, drift=cyc.drift, solve=cyc.solve, flags=fl))
        pm_batch_pk_estimate(self.batch, self.pos, self.bins, out=self.pk_out)
        k, p, c = self.pk_out
        o = 0
        for st in self.states:
            nb, b = st.noise.shape[0], st.group.bins()
            st.out = (k[o:o + nb * b].view(nb, b), p[o:o + nb * b].view(nb, b), c[o:o + nb * b].view(nb, b))
            o += nb * b

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

    def close(self):
        """Release the captured graph before the batch whose plans, streams and device
        tables it was captured from (and which it may still reference), then the batch."""
        self.graph = None
        if getattr(self, "batch", None) is not None:
            self.batch.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

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
