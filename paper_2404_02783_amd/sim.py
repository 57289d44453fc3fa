"""Leapfrog over the C ABI (host loop only; every step runs in the kernels).

A kick-drift-kick leapfrog from a_0 to a_n with half steps at sqrt(a_j a_{j+1}) is
issued as n+1 ``pm_step`` cycles (force at a_j, kick, drift): the cycle at a_j
kicks by K2(previous step) + K1(this step) and drifts by Dr(a_j, a_{j+1}); the
closing cycle at a_n kicks by K2(last step) and does not drift.  The
Poisson-gauge set carries its potential between force evaluations; its first
evaluation is quasi-static.
"""
from __future__ import annotations

from . import (FIDUCIAL, PM_GRAD_SPECTRAL, PM_STEP_DENSITY_READY, PM_STEP_DEPOSIT_NEXT, Plan, StepParams,
               gauge_params, leapfrog_factors, newton_params, pm_step)
from . import log_steps as _log_steps

__all__ = ["log_steps", "Run"]


def log_steps(a_start: float, a_end: float, n_steps: int):
    """n_steps + 1 scale factors equally spaced in ln a (pm_log_steps)."""
    return _log_steps(a_start, a_end, n_steps)


class Run:
    """Particles (pos, mom) of one set on one plan.  ``gauge=True`` selects the
    Poisson-gauge force; otherwise Newtonian.  Consecutive cycles hand the density of
    the drifted positions to the next cycle (PM_STEP_DEPOSIT_NEXT / DENSITY_READY);
    call ``invalidate()`` after changing ``pos`` or using the plan for anything else
    between cycles."""

    def __init__(self, plan: Plan, pos, mom, cosmo=FIDUCIAL, gauge: bool = False, grad: int = PM_GRAD_SPECTRAL):
        self.plan, self.pos, self.mom, self.cosmo, self.gauge, self.grad = plan, pos, mom, cosmo, gauge, grad
        self.force = plan.mesh(3)
        self.phi = plan.spectrum() if gauge else None
        self.a_prev = 0.0
        self.dens_ready = False

    def invalidate(self):
        self.dens_ready = False

    def solve_params(self, a: float):
        if self.gauge:
            sp = gauge_params(self.plan.box, self.plan.n, a, self.a_prev, self.cosmo)
            sp.grad = self.grad
        else:
            sp = newton_params(self.cosmo, self.grad)
        return sp

    def cycle(self, a: float, kick: float, drift: float, last: bool = False):
        flags = (PM_STEP_DENSITY_READY if self.dens_ready else 0) | (0 if last else PM_STEP_DEPOSIT_NEXT)
        st = StepParams(kick=kick, drift=drift, solve=self.solve_params(a), flags=flags)
        self.dens_ready = False
        pm_step(self.plan, self.pos, self.mom, st, self.force, self.phi)
        self.dens_ready = not last
        self.a_prev = a

    def leapfrog(self, a_steps, close: bool = True, on_cycle=None):
        """Run the whole schedule; ``on_cycle(j)`` is called after each cycle."""
        kick, drift = leapfrog_factors(a_steps, self.cosmo)
        n = len(a_steps) - 1
        for j in range(n):
            self.cycle(a_steps[j], kick[j], drift[j])
            if on_cycle is not None:
                on_cycle(j)
        if close:
            self.cycle(a_steps[-1], kick[n], 0.0, last=True)
        else:
            self.invalidate()
