"""GR-minus-Newton displacement and the combined particle set (FP64).

Test infrastructure only (see ``oracle/__init__``).

eq. xiGR: xi = x_GR - x_Newton, per particle, between two runs that share their
initial phases and particle identities; eq. combined: x = x_fine + xi, in
configuration space (Sec. 2).  The paper combines at equal particle number.
When the fine run has more particles than the coarse pair, xi is treated as a
function of the Lagrangian coordinate and interpolated with CIC weights from
the coarse lattice to the fine lattice points (reading for unequal counts).

Periodicity: xi is the minimum-image difference,
    xi = ((x_GR - x_N + N_c/2) mod N_c) - N_c/2   (coarse cells),
and it is scaled by N_f/N_c to fine cells before it is added.
Fine particle j (per axis) sits at coarse-lattice coordinate
    u = ((2 j + 1) N_c - N_f) / (2 N_f),
so its base coarse particle i0 = floor(u) and offset t = u - i0 are exact
rationals computed from integers.
"""
from __future__ import annotations

import itertools

import torch

from . import cic


def xi_min_image(x_gr: torch.Tensor, x_n: torch.Tensor, n_c: int) -> torch.Tensor:
    """eq. xiGR with the periodic minimum image; [3, Nc^3] in coarse cells."""
    d = x_gr - x_n + 0.5 * n_c
    return d - n_c * torch.floor(d / n_c) - 0.5 * n_c


def fine_to_coarse_axis(n_c: int, n_f: int):
    """Per-axis (i0, t) for fine lattice index j = 0..N_f-1 (integers, then one division)."""
    j = torch.arange(n_f, dtype=torch.long)
    num = (2 * j + 1) * n_c - n_f
    den = 2 * n_f
    i0 = torch.div(num, den, rounding_mode="floor")
    rem = num - i0 * den
    return i0, rem.double() / den


def interpolate_lagrangian(xi: torch.Tensor, n_c: int, n_f: int) -> torch.Tensor:
    """CIC interpolation of a coarse-lattice field [3, Nc^3] to the fine lattice [3, Nf^3]."""
    i0, t = fine_to_coarse_axis(n_c, n_f)
    grid = xi.view(3, n_c, n_c, n_c)
    out = torch.zeros((3, n_f, n_f, n_f), dtype=torch.float64)
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        wx = (t if dx else 1.0 - t).view(n_f, 1, 1)
        wy = (t if dy else 1.0 - t).view(1, n_f, 1)
        wz = (t if dz else 1.0 - t).view(1, 1, n_f)
        ix = ((i0 + dx) % n_c).view(n_f, 1, 1)
        iy = ((i0 + dy) % n_c).view(1, n_f, 1)
        iz = ((i0 + dz) % n_c).view(1, 1, n_f)
        out = out + grid[:, ix, iy, iz] * (wx * wy * wz)
    return out.reshape(3, -1)


def combine(x_gr: torch.Tensor, x_n: torch.Tensor, n_c: int, x_fine: torch.Tensor, n_f: int) -> torch.Tensor:
    """eq. combined: x = wrap(x_fine + (N_f/N_c) * CIC_q[xi](q_fine)) in fine cells."""
    xi = xi_min_image(x_gr, x_n, n_c)
    xi_f = xi if n_f == n_c else interpolate_lagrangian(xi, n_c, n_f)
    return cic.wrap(x_fine + (n_f / n_c) * xi_f, n_f)


def combine_at(x_gr: torch.Tensor, x_n: torch.Tensor, n_c: int, x_fine: torch.Tensor, j_fine: torch.Tensor,
               n_f: int) -> torch.Tensor:
    """``combine`` for a sample of fine particles only: j_fine [3, M] are their
    lattice indices per axis, x_fine [3, M] their positions.  xi is evaluated at the
    eight coarse particles around each fine lattice point (same weights and wrap)."""
    i0_ax, t_ax = fine_to_coarse_axis(n_c, n_f)
    i0 = torch.stack([i0_ax[j_fine[d]] for d in range(3)])
    t = torch.stack([t_ax[j_fine[d]] for d in range(3)])
    xi_f = torch.zeros(x_fine.shape, dtype=torch.float64)
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        c = [(i0[0] + dx) % n_c, (i0[1] + dy) % n_c, (i0[2] + dz) % n_c]
        idx = (c[0] * n_c + c[1]) * n_c + c[2]
        w = (t[0] if dx else 1.0 - t[0]) * (t[1] if dy else 1.0 - t[1]) * (t[2] if dz else 1.0 - t[2])
        xi_f = xi_f + xi_min_image(x_gr[:, idx], x_n[:, idx], n_c) * w
    return cic.wrap(x_fine + (n_f / n_c) * xi_f, n_f)


def add_displacement(xi: torch.Tensor, n_c: int, x_fine: torch.Tensor, n_f: int) -> torch.Tensor:
    """eq. combined with a displacement field given directly (e.g. the linear
    Poisson-gauge shift xi_lin(a) in place of the GR-minus-Newton difference of two
    runs): x = wrap(x_fine + (N_f/N_c) * CIC_q[xi](q_fine)), xi [3, Nc^3] in coarse
    cells on the coarse lattice."""
    xi_f = xi if n_f == n_c else interpolate_lagrangian(xi, n_c, n_f)
    return cic.wrap(x_fine + (n_f / n_c) * xi_f, n_f)


def add_displacement_at(xi: torch.Tensor, n_c: int, x_fine: torch.Tensor, j_fine: torch.Tensor,
                        n_f: int) -> torch.Tensor:
    """``add_displacement`` for a sample of fine particles (lattice indices j_fine
    [3, M], positions x_fine [3, M])."""
    i0_ax, t_ax = fine_to_coarse_axis(n_c, n_f)
    i0 = torch.stack([i0_ax[j_fine[d]] for d in range(3)])
    t = torch.stack([t_ax[j_fine[d]] for d in range(3)])
    xi_f = torch.zeros(x_fine.shape, dtype=torch.float64)
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        idx = (((i0[0] + dx) % n_c) * n_c + (i0[1] + dy) % n_c) * n_c + (i0[2] + dz) % n_c
        w = (t[0] if dx else 1.0 - t[0]) * (t[1] if dy else 1.0 - t[1]) * (t[2] if dz else 1.0 - t[2])
        xi_f = xi_f + xi[:, idx] * w
    return cic.wrap(x_fine + (n_f / n_c) * xi_f, n_f)
