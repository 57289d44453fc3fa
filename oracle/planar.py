"""Plane-parallel reduction of the Newtonian force-kick-drift cycle (FP64).

Test infrastructure only (see ``oracle/__init__``).

Take a particle lattice (one particle per cell, Lagrangian index q) whose planes
normal to one axis move rigidly: every particle of the plane q_axis = j has the
coordinate c_axis[j] along that axis, and q_b + 1/2 + c_b[j] along each
transverse axis b (an offset common to the plane).  Along a transverse axis the
CIC weights a node receives from its two neighbouring particles of a plane are
(1 - t) and t with the same t, so the counting density of Sec. 4 is constant on
mesh planes normal to the axis: delta(c) = rho_1(c_axis) - 1, with rho_1 the
one-dimensional CIC deposit of the N plane coordinates (nbar = 1).

The DFT of a field constant along two axes vanishes off the line of wavevectors
along the third, where it is N^2 times the one-dimensional DFT; on that line the
Newtonian Green's function of Sec. 2 (see ``solve``) and the gradient symbol of
the axis take their one-dimensional values and the transverse symbols vanish.
With the 1/N^3 of the inverse transform the force meshes are F_axis(c) =
f_1(c_axis) and F_b = 0, f_1 being the one-dimensional solve with 1/N.  The
gathered force of a particle is the one-dimensional CIC interpolation of f_1 at
its plane coordinate (the transverse weights sum to one), so the whole cycle is
a cycle of N planes.
"""
from __future__ import annotations

import math

import torch

from . import cic, estimators


def deposit_delta_line(x: torch.Tensor, n: int) -> torch.Tensor:
    """Counting-density contrast on the N mesh planes from the N plane coordinates x."""
    base = torch.floor(x)
    t = x - base
    i = base.long()
    rho = torch.zeros(n, dtype=torch.float64)
    rho = rho.index_add(0, i % n, 1.0 - t).index_add(0, (i + 1) % n, t)
    return rho - 1.0


def newton_force_line(delta: torch.Tensor, omega_m: float, grad: str = "spectral") -> torch.Tensor:
    """f_1 = IDFT_1(-D(k) phi_hat), phi_hat = -(3/2) Omega_m delta_hat / k^2 (zero at k = 0),
    k = 2 pi m / N, m = 0..N/2, with the gradient symbol D of ``solve.gradient_symbol``."""
    n = delta.shape[0]
    dh = torch.fft.rfft(delta)
    m = torch.arange(n // 2 + 1, dtype=torch.float64)
    k = 2.0 * math.pi * m / n
    k2 = torch.where(m > 0, k * k, torch.ones_like(k))
    phi = torch.where(m > 0, -1.5 * omega_m * dh / k2, torch.zeros_like(dh))
    if grad == "spectral":
        dsym = torch.complex(torch.zeros_like(k), torch.where(m == n // 2, torch.zeros_like(k), k))
    elif grad == "fd2":
        dsym = torch.complex(torch.zeros_like(k), torch.sin(k))
    elif grad == "fd1":
        dsym = torch.complex(torch.cos(k) - 1.0, torch.sin(k))
    else:
        raise ValueError(grad)
    return torch.fft.irfft(-dsym * phi, n=n)


def gather_line(f: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """One-dimensional CIC interpolation of the node values f to the coordinates x."""
    n = f.shape[0]
    base = torch.floor(x)
    t = x - base
    i = base.long()
    return (1.0 - t) * f[i % n] + t * f[(i + 1) % n]


def cycle_line(coord: torch.Tensor, mom: torch.Tensor, axis: int, kick: float, drift: float, n: int,
               omega_m: float, grad: str = "spectral"):
    """One force-kick-drift cycle of a plane-parallel lattice given per plane:
    coord [3, N] (axis row: plane coordinate in [0, N); other rows: transverse
    offsets), mom [3, N].  Returns (coord', mom', f_1) with f_1 the force on the N
    mesh planes before the kick; transverse offsets are not wrapped."""
    f1 = newton_force_line(deposit_delta_line(coord[axis], n), omega_m, grad)
    mom = mom.clone()
    mom[axis] = mom[axis] + kick * gather_line(f1, coord[axis])
    coord = coord + drift * mom
    coord[axis] = cic.wrap(coord[axis], n)
    return coord, mom, f1


def particle_coords(coord: torch.Tensor, axis: int, n: int, q: torch.Tensor) -> torch.Tensor:
    """Coordinates [3, M] of the particles with lattice indices q ([3, M]) of the
    configuration given per plane by coord."""
    out = torch.empty(q.shape, dtype=torch.float64)
    qa = q[axis]
    for b in range(3):
        if b == axis:
            out[b] = coord[b][qa]
        else:
            out[b] = cic.wrap(q[b].double() + 0.5 + coord[b][qa], n)
    return out


def cycle_line_vjp(coord: torch.Tensor, mom: torch.Tensor, axis: int, kick: float, drift: float, n: int,
                   omega_m: float, lam_coord: torch.Tensor, lam_mom: torch.Tensor, grad: str = "spectral"):
    """Reverse-mode derivative of ``cycle_line``: cotangents (lam_coord [3, N],
    lam_mom [3, N]) of its outputs (coord', mom') -> cotangents of (coord, mom), by
    autograd through the one-dimensional cycle (floor has zero derivative, so CIC
    weights are differentiated from the right at cell edges).

    For a plane-parallel lattice and cotangents that are constant on each lattice
    plane, this is also the cotangent of every single particle of the plane in the
    3-D cycle: moving one particle changes the transverse mean of the density by
    1/N^2 of what moving its plane does, the transverse forces it induces average
    to zero over a plane, and each plane's N^2 particles share the cotangent."""
    c = coord.detach().clone().requires_grad_(True)
    m = mom.detach().clone().requires_grad_(True)
    c1, m1, _ = cycle_line(c, m, axis, kick, drift, n, omega_m, grad)
    gc, gm = torch.autograd.grad((c1, m1), (c, m), grad_outputs=(lam_coord, lam_mom), allow_unused=True)
    return (torch.zeros_like(c) if gc is None else gc), (torch.zeros_like(m) if gm is None else gm)


def power_spectrum_line(x: torch.Tensor, n: int, box: float, n_bins: int, counts: torch.Tensor) -> torch.Tensor:
    """The P(k) estimator (eq. powerspectrum, bins of ``estimators.pk_bin_index``) of
    the counting density of a plane-parallel lattice with plane coordinates x: only
    the wavevectors on the axis line carry power, with 3-D amplitude N^2 times the
    one-dimensional DFT.  ``counts`` are the estimator's mode counts per bin (all 3-D
    modes, e.g. from ``estimators.power_spectrum_sparse``).  Differentiable in x."""
    d = deposit_delta_line(x, n)
    dh = torch.fft.fft(d.to(torch.complex128))
    m = torch.fft.fftfreq(n, d=1.0 / n).round().long()
    b = estimators.bin_of_norm2(m * m, n, n_bins)
    p2 = (dh.real ** 2 + dh.imag ** 2) * float(n) ** 4
    sel = b >= 0
    sp = torch.zeros(n_bins, dtype=torch.float64).index_add(0, b[sel], p2[sel])
    cnt = counts.to(torch.float64)
    return torch.where(cnt > 0, box ** 3 / float(n) ** 6 * sp / torch.where(cnt > 0, cnt, torch.ones_like(cnt)),
                       torch.zeros_like(sp))


def power_spectrum_line_vjp(x: torch.Tensor, n: int, box: float, n_bins: int, counts: torch.Tensor,
                            dpk: torch.Tensor) -> torch.Tensor:
    """Cotangent of every particle's coordinate along the axis for the loss
    sum_b dpk_b P_b: the derivative with respect to a plane coordinate (which moves
    the plane's N^2 particles) divided by N^2, since moving one particle changes the
    transverse mean of the density by 1/N^2 of that and off-axis modes, zero at the
    plane-parallel lattice, only to second order.  The transverse cotangents are 0.
    Returns [N] (one value per lattice plane)."""
    xr = x.detach().clone().requires_grad_(True)
    pk = power_spectrum_line(xr, n, box, n_bins, counts)
    (g,) = torch.autograd.grad(pk, xr, grad_outputs=dpk.to(torch.float64))
    return g / float(n) ** 2
