"""Fourier-space potential solves and PM forces (FP64).

Test infrastructure only (see ``oracle/__init__``).

Newtonian solve (N-body gauge; paper Sec. 2 states that the Newtonian Poisson
equation and particle equations of motion coincide with those of the N-body
gauge): laplacian(phi) = (3/2) Omega_m delta in grid units, so
    phi_hat(n) = -(3/2) Omega_m delta_hat(n) / k_g^2     (n != 0),  phi_hat(0) = 0,
and the force F = -grad(phi) has F_hat_d = -D_d(n) phi_hat(n) with the
gradient symbol D_d.  The default symbol is the exact spectral one, i k_d,
set to zero on the Nyquist plane of axis d; two finite-difference symbols are
kept because the paper attributes a large-scale power deficit of its PM code to
its first-order gradient (Sec. 4.1):
    "fd2": i sin(k_d)          (second-order central difference)
    "fd1": exp(i k_d) - 1      (first-order one-sided difference).
No CIC deconvolution is applied.

Poisson-gauge solve (weak-field scalar sector, linear-metric reading).  The
paper does not write the field equations; it states the linear relation
between counting and physical density in Poisson gauge (eq.
physical_density: delta_count = delta_phys - 3 phi) and the resulting
scale-dependent bias (eqs. b1, bgr).  The reading implemented here is the
linear 00 Einstein equation in conformal time with psi = phi,
    -k^2 phi - 3 H (phi' + H phi) = (3/2) H^2 Omega_m(a) delta_phys,
with delta_phys = delta_count + 3 phi (eq. physical_density) and phi' by a
backward difference over the last step dtau.  Both are moved to the left so the
solve stays diagonal in Fourier space:
    phi_new = [(3/2) H^2 Om_a delta_c_hat - 3 H phi_old / dtau]
              / [-k^2 - 3 H^2 - 3 H / dtau - (9/2) H^2 Om_a],
where H is the conformal Hubble rate in inverse cells and dtau is in cells
(1/dtau = 0 gives the quasi-static solve used at the first evaluation).  The
particle force is F = -grad(a c_g^2 phi_new), which reduces to the Newtonian
force when c_g -> infinity.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import fourier


def gradient_symbol(n: int, kind: str = "spectral"):
    """Gradient symbols (D_x, D_y, D_z) on the r2c grid, complex128, broadcastable."""
    ks = fourier.kgrid(n)
    nyq = fourier.nyquist_masks(n)
    out = []
    for k, m in zip(ks, nyq):
        if kind == "spectral":
            d = torch.complex(torch.zeros_like(k), torch.where(m, torch.zeros_like(k), k))
        elif kind == "fd2":
            d = torch.complex(torch.zeros_like(k), torch.sin(k))
        elif kind == "fd1":
            d = torch.complex(torch.cos(k) - 1.0, torch.sin(k))
        else:
            raise ValueError(kind)
        out.append(d)
    return out


def k_squared(n: int) -> torch.Tensor:
    """|k_g|^2 on the r2c grid, broadcast to [N,N,N/2+1]."""
    kx, ky, kz = fourier.kgrid(n)
    return kx * kx + ky * ky + kz * kz


def newton_potential_k(dhat: torch.Tensor, omega_m: float) -> torch.Tensor:
    """phi_hat = -(3/2) Omega_m delta_hat / k^2, zero at k = 0."""
    n = dhat.shape[0]
    k2 = k_squared(n)
    inv = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)), torch.zeros_like(k2))
    return -1.5 * omega_m * dhat * inv


def forces_from_potential_k(phi_hat: torch.Tensor, grad: str = "spectral") -> torch.Tensor:
    """F_d = IDFT(-D_d phi_hat) for d = x, y, z -> [3, N, N, N]."""
    n = phi_hat.shape[0]
    ds = gradient_symbol(n, grad)
    return torch.stack([fourier.irfft3(-d * phi_hat, n) for d in ds])


def newton_forces(delta: torch.Tensor, omega_m: float, grad: str = "spectral") -> torch.Tensor:
    """PM acceleration meshes F = -grad(phi) for a density contrast mesh."""
    dhat = fourier.rfft3(delta)
    return forces_from_potential_k(newton_potential_k(dhat, omega_m), grad)


@dataclass(frozen=True)
class GaugeParams:
    """Scalars of one Poisson-gauge force evaluation (all in grid units)."""
    a: float          # scale factor of the evaluation
    om_a: float       # Omega_m(a)
    calh: float       # conformal Hubble rate, 1/cells
    c_g: float        # speed of light, cells per (1/H0)
    inv_dtau: float   # 1 / (conformal time since the previous evaluation), 0 = quasi-static


def poisson_gauge_potential_k(dc_hat: torch.Tensor, phi_old_hat: torch.Tensor, gp: GaugeParams) -> torch.Tensor:
    """Implicit Poisson-gauge update phi_old -> phi_new for counting density delta_c."""
    n = dc_hat.shape[0]
    k2 = k_squared(n)
    h, h2 = gp.calh, gp.calh * gp.calh
    num = 1.5 * h2 * gp.om_a * dc_hat - 3.0 * h * gp.inv_dtau * phi_old_hat
    den = -k2 - 3.0 * h2 - 3.0 * h * gp.inv_dtau - 4.5 * h2 * gp.om_a
    phi = num / den
    phi = torch.where(k2 > 0, phi, torch.zeros_like(phi))
    return phi


def poisson_gauge_forces(delta_c: torch.Tensor, phi_old_hat: torch.Tensor, gp: GaugeParams,
                         grad: str = "spectral"):
    """Forces on the relativistic particle set and the new potential.

    Returns (F [3,N,N,N], phi_new_hat [N,N,N/2+1])."""
    dc_hat = fourier.rfft3(delta_c)
    phi = poisson_gauge_potential_k(dc_hat, phi_old_hat, gp)
    return forces_from_potential_k(gp.a * gp.c_g * gp.c_g * phi, grad), phi
