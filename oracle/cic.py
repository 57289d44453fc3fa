"""Cloud-in-cell counting density and interpolation (FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper measures the matter field with the counting density of a CIC
assignment (Sec. 4, "Matter density statistics"): every particle carries the
same mass and is shared between the 8 mesh nodes around it with trilinear
weights.  Mesh node c sits at integer coordinates; a particle at x has base
node i = floor(x) and offsets t = x - i, and gives weight (1 - t_d) to node i_d
and t_d to node i_d + 1 (mod N) along each axis.  The density contrast is
delta = rho / nbar - 1 with nbar = Np / N^3.

Positions are [3, Np] tensors in grid units; axis 0 indexes the slowest mesh
axis.  The same weights interpolate a mesh back to the particles.
"""
from __future__ import annotations

import itertools

import torch


def wrap(x: torch.Tensor, n: int) -> torch.Tensor:
    """Periodic wrap into [0, N): x - N floor(x/N); a rounded quotient that
    overshoots (N not a power of two) is corrected by +N, and a result that rounds
    up to exactly N is set to 0 (the wrap-rule reading for finite precision)."""
    y = x - n * torch.floor(x / n)
    y = torch.where(y < 0, y + n, y)
    return torch.where(y >= n, torch.zeros_like(y), y)


def _corners(pos: torch.Tensor, n: int):
    """Yield (flat node index, weight) for the 8 CIC corners of every particle."""
    base = torch.floor(pos)
    t = pos - base
    i = base.long()
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        wx = t[0] if dx else 1.0 - t[0]
        wy = t[1] if dy else 1.0 - t[1]
        wz = t[2] if dz else 1.0 - t[2]
        ix = (i[0] + dx) % n
        iy = (i[1] + dy) % n
        iz = (i[2] + dz) % n
        yield (ix * n + iy) * n + iz, wx * wy * wz


def cell_index(pos: torch.Tensor) -> torch.Tensor:
    """Base node index floor(x) per axis (the integer assignment decision), int64 [3, Np]."""
    return torch.floor(pos).long()


def deposit_rho(pos: torch.Tensor, n: int, mass: torch.Tensor | float = 1.0) -> torch.Tensor:
    """Sum of CIC weights (times ``mass``) per node: rho(c) = sum_p m_p W(x_p - c), [N,N,N]."""
    rho = torch.zeros(n ** 3, dtype=torch.float64)
    for idx, w in _corners(pos, n):
        rho = rho.index_add(0, idx, w * mass)
    return rho.view(n, n, n)


def deposit_delta(pos: torch.Tensor, n: int) -> torch.Tensor:
    """Counting-density contrast delta = rho/nbar - 1 (paper Sec. 4)."""
    nbar = pos.shape[1] / n ** 3
    return deposit_rho(pos, n) / nbar - 1.0


def gather(mesh: torch.Tensor, pos: torch.Tensor) -> torch.Tensor:
    """CIC interpolation of one or more meshes ([..., N, N, N]) to the particles:
    f_p = sum_c W(x_p - c) f(c).  Returns [..., Np]."""
    n = mesh.shape[-1]
    flat = mesh.reshape(*mesh.shape[:-3], n ** 3)
    out = None
    for idx, w in _corners(pos, n):
        term = flat[..., idx] * w
        out = term if out is None else out + term
    return out


def rho_at_nodes(nodes: torch.Tensor, pos: torch.Tensor, n: int) -> torch.Tensor:
    """rho(c) = sum_p W(x_p - c) at the nodes ``nodes`` ([3, M] integer) from the
    particles ``pos`` ([3, Np]) only, written as the product over axes of the
    periodic tent max(0, 1 - |x_d - c_d|) (minimum-image distance).  This is the
    CIC weight above seen from the node: a particle within one cell of the node
    along every axis gives it 1 - |x_d - c_d| per axis.  Returns [M]."""
    c = nodes.to(torch.float64).unsqueeze(-1)          # [3, M, 1]
    x = pos.to(torch.float64).unsqueeze(1)             # [3, 1, Np]
    d = torch.remainder(x - c + n / 2, n) - n / 2
    w = torch.clamp(1.0 - d.abs(), min=0.0).prod(dim=0)
    return w.sum(dim=-1)
