"""Kick-drift-kick leapfrog for the PM particle sets (FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper's runs are particle-mesh simulations (Sec. 2; Sec. 4.1 ties the
small-scale power deficit to the particle-mesh force).  The integrator is not
stated; the reading here is the symplectic kick-drift-kick leapfrog in the
scale factor with half steps at the geometric mean:
    p += F(x_j) K(a_j, a_h);   x = wrap(x + p Dr(a_j, a_{j+1}));
    p += F(x_{j+1}) K(a_h, a_{j+1});   a_h = sqrt(a_j a_{j+1}),
with one force evaluation per step plus one at the start.  F is the CIC
interpolation of the PM force meshes to the particles (same weights as the
deposit).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import cic, cosmology as cm, solve


@dataclass
class NewtonForce:
    """Newtonian PM force at any scale factor (the force in grid units has no
    explicit a-dependence)."""
    n: int
    cosmo: cm.Cosmo = cm.FIDUCIAL
    grad: str = "spectral"

    def __call__(self, pos: torch.Tensor, a: float) -> torch.Tensor:
        meshes = solve.newton_forces(cic.deposit_delta(pos, self.n), self.cosmo.omega_m, self.grad)
        return cic.gather(meshes, pos)


@dataclass
class GaugeForce:
    """Poisson-gauge force with the potential carried between evaluations.
    The first evaluation is quasi-static (1/dtau = 0)."""
    n: int
    dx: float
    cosmo: cm.Cosmo = cm.FIDUCIAL
    grad: str = "spectral"
    c_g_override: float | None = None
    phi_hat: torch.Tensor | None = None
    a_prev: float | None = None

    def params(self, a: float) -> solve.GaugeParams:
        c_g = self.c_g_override if self.c_g_override is not None else cm.c_grid(self.dx)
        calh = a * cm.hubble_e(self.cosmo, a) / c_g
        inv_dtau = 0.0 if self.a_prev is None else 1.0 / (c_g * cm.kick_factor(self.cosmo, self.a_prev, a))
        return solve.GaugeParams(a=a, om_a=cm.omega_m_of_a(self.cosmo, a), calh=calh, c_g=c_g, inv_dtau=inv_dtau)

    def __call__(self, pos: torch.Tensor, a: float) -> torch.Tensor:
        if self.phi_hat is None:
            self.phi_hat = torch.zeros((self.n, self.n, self.n // 2 + 1), dtype=torch.complex128)
        gp = self.params(a)
        meshes, self.phi_hat = solve.poisson_gauge_forces(cic.deposit_delta(pos, self.n), self.phi_hat, gp, self.grad)
        self.a_prev = a
        return cic.gather(meshes, pos)


def kdk_factors(cosmo: cm.Cosmo, a0: float, a1: float):
    """(K(a0, a_h), Dr(a0, a1), K(a_h, a1)) with a_h = sqrt(a0 a1)."""
    ah = math.sqrt(a0 * a1)
    return cm.kick_factor(cosmo, a0, ah), cm.drift_factor(cosmo, a0, a1), cm.kick_factor(cosmo, ah, a1)


def run_kdk(pos: torch.Tensor, mom: torch.Tensor, a_steps, force, n: int, cosmo: cm.Cosmo = cm.FIDUCIAL):
    """Leapfrog from a_steps[0] to a_steps[-1]; returns new (pos, mom)."""
    pos = pos.clone()
    mom = mom.clone()
    f = force(pos, a_steps[0])
    for a0, a1 in zip(a_steps[:-1], a_steps[1:]):
        k1, dr, k2 = kdk_factors(cosmo, a0, a1)
        mom = mom + k1 * f
        pos = cic.wrap(pos + dr * mom, n)
        f = force(pos, a1)
        mom = mom + k2 * f
    return pos, mom


def force_then_kick_drift(pos: torch.Tensor, mom: torch.Tensor, kick: float, drift: float, force, a: float, n: int):
    """One 'force, kick, drift' cycle: F = force(x); p += kick F; x = wrap(x + drift p).
    A leapfrog run is a chain of these with kick = K2(previous) + K1(current) and a
    closing kick with drift = 0."""
    f = force(pos, a)
    mom = mom + kick * f
    pos = cic.wrap(pos + drift * mom, n)
    return pos, mom
