"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only draws random numbers and lays them out in the array shapes the
library consumes.  It holds none of the particle-mesh arithmetic: no Fourier
transforms, no mass assignment, no cosmology.  Everything here is a pure
function of (shape, seed), built on NumPy's counter-based Philox generator.

Conventions shared by every caller:
  * real meshes are ``[N, N, N]`` row-major, float64 unless asked otherwise;
  * particle arrays are structure-of-arrays ``[3, Np]`` in grid units
    (a coordinate lies in ``[0, N)``).

Full-size configurations (N up to 1024, built on the device) use a second,
counter-based source: a 32-bit integer hash of (seed, stream, particle index)
evaluated with torch integer operations, bit-identical on every device, so a
test can regenerate any single particle on the CPU.  Their coordinates and
momenta are integer multiples of 2^-13 cells below 2^10 ("quanta"), exactly
representable in float32 and float64 alike.
"""
from __future__ import annotations

import numpy as np
import torch

__all__ = [
    "rng",
    "white_noise",
    "uniform_particles",
    "clustered_particles",
    "lattice_jitter_particles",
    "random_complex_mesh",
    "random_real_mesh",
    "QUANTUM",
    "hash32",
    "counter_bits",
    "hashed_lattice_quanta",
    "hashed_lattice_particles",
    "planar_profile",
    "expand_planar",
    "broadcast_planes",
    "plane_wave_mesh",
]


def rng(seed: int) -> np.random.Generator:
    """NumPy ``Generator`` over Philox4x32-10 keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(key=int(seed)))


def white_noise(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Unit-variance i.i.d. Gaussian white noise on an ``n**3`` mesh.

    Drawn in chunks of planes so that a 1024**3 field never needs a float64
    copy when ``dtype`` is float32.
    """
    g = rng(seed)
    out = np.empty((n, n, n), dtype=dtype)
    plane = n * n
    step = max(1, (1 << 24) // plane)
    for i0 in range(0, n, step):
        i1 = min(n, i0 + step)
        out[i0:i1] = g.standard_normal(size=(i1 - i0, n, n), dtype=np.float64).astype(dtype, copy=False)
    return out


def uniform_particles(n_mesh: int, n_part: int, seed: int, dtype=np.float64) -> np.ndarray:
    """``n_part`` positions uniform in the periodic box ``[0, n_mesh)^3``; shape ``[3, n_part]``."""
    g = rng(seed)
    x = g.random(size=(3, n_part), dtype=np.float64) * n_mesh
    x = x.astype(dtype)
    # float32 rounding can produce exactly n_mesh; fold it back inside the box.
    x[x >= n_mesh] = 0
    return x


def lattice_jitter_particles(n_mesh: int, seed: int, amplitude: float, dtype=np.float64) -> np.ndarray:
    """One particle per cell: the half-cell-offset lattice plus a uniform jitter
    of +-``amplitude`` cells per axis, wrapped into the box.  Lagrangian order
    (particle ``(i*N + j)*N + l`` starts near cell ``(i, j, l)``)."""
    g = rng(seed)
    n = n_mesh
    q = (np.arange(n, dtype=np.float64) + 0.5)
    qx, qy, qz = np.meshgrid(q, q, q, indexing="ij")
    x = np.stack([qx.ravel(), qy.ravel(), qz.ravel()])
    x = x + amplitude * (2.0 * g.random(size=x.shape) - 1.0)
    x = np.mod(x, n)
    x = x.astype(dtype)
    x[x >= n] = 0
    return x


def clustered_particles(n_mesh: int, n_part: int, seed: int, n_clumps: int = 16,
                        width: float = 1.5, dtype=np.float64) -> np.ndarray:
    """Half the particles uniform, half in Gaussian clumps of ``width`` cells
    around random centres (a stand-in for collapsed haloes), wrapped into the box."""
    g = rng(seed)
    n_u = n_part // 2
    n_c = n_part - n_u
    xu = g.random(size=(3, n_u)) * n_mesh
    centres = g.random(size=(3, n_clumps)) * n_mesh
    which = g.integers(0, n_clumps, size=n_c)
    xc = centres[:, which] + width * g.standard_normal(size=(3, n_c))
    x = np.concatenate([xu, xc], axis=1)
    x = np.mod(x, n_mesh).astype(dtype)
    x[x >= n_mesh] = 0
    return x


def random_real_mesh(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Gaussian random real mesh ``[n, n, n]`` (not band-limited)."""
    return rng(seed).standard_normal(size=(n, n, n)).astype(dtype)


def random_complex_mesh(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex mesh with independent standard-normal real and imaginary parts."""
    g = rng(seed)
    re = g.standard_normal(size=shape)
    im = g.standard_normal(size=shape)
    return (re + 1j * im).astype(dtype)


# ------------------------------------------------------------ full-size inputs --

QUANTUM_BITS = 13
QUANTUM = 2.0 ** -QUANTUM_BITS      # cells
_M32 = 0xFFFFFFFF


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    # x * c mod 2^32 for x in [0, 2^32), split so that no int64 product overflows
    lo = x * (c & 0xFFFF)
    hi = ((x * (c >> 16)) & 0xFFFF) << 16
    return (lo + hi) & _M32


def hash32(x: torch.Tensor) -> torch.Tensor:
    """Chris Wellons' "lowbias32" integer hash (xor-shift 16, multiply by
    0x7feb352d, xor-shift 15, multiply by 0x846ca68b, xor-shift 16, all modulo
    2^32) of an int64 tensor holding values in [0, 2^32)."""
    x = x & _M32
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    return x ^ (x >> 16)


def counter_bits(index: torch.Tensor, stream: int, seed: int) -> torch.Tensor:
    """32 random bits (int64 in [0, 2^32)) for each (seed, stream, index);
    index in [0, 2^30), stream in [0, 4)."""
    mix = int(hash32(torch.tensor([seed & _M32], dtype=torch.int64))[0])
    key = index.to(torch.int64) | (int(stream) << 30)
    return hash32(hash32(key) ^ mix)


def _signed_quanta(bits: torch.Tensor, amp_log2: int) -> torch.Tensor:
    # uniform integer in [-2^(amp_log2 + 13), 2^(amp_log2 + 13)) from the top 16 bits
    sh = 2 - amp_log2
    if not 0 <= sh <= 15:
        raise ValueError("amp_log2 must lie in [-13, 2]")
    return ((bits >> 16) - (1 << 15)) >> sh


def hashed_lattice_quanta(n: int, seed: int, amp_log2: int, axis: int, index: torch.Tensor) -> torch.Tensor:
    """Coordinate ``axis`` (in quanta, int64) of particles ``index`` of a
    half-cell-offset lattice (particle (i N + j) N + l starts in cell (i, j, l))
    displaced by a hashed uniform offset in [-2^amp_log2, 2^amp_log2) cells,
    wrapped into [0, N)."""
    index = index.to(torch.int64)
    q = (index // (n * n), (index // n) % n, index % n)[axis]
    d = _signed_quanta(counter_bits(index, axis, seed), amp_log2)
    span = n << QUANTUM_BITS
    return torch.remainder((q << QUANTUM_BITS) + (1 << (QUANTUM_BITS - 1)) + d, span)


def hashed_lattice_particles(n: int, seed: int, amp_log2: int = 1, index: torch.Tensor | None = None,
                             device=None, dtype=torch.float64) -> torch.Tensor:
    """Positions [3, len(index)] (all N^3 particles if ``index`` is None) of the
    hashed-offset lattice, built axis by axis on ``device``."""
    if n > 1024:
        raise ValueError("quanta cover meshes up to 1024 cells")
    if index is None:
        index = torch.arange(n ** 3, dtype=torch.int64, device=device)
    else:
        index = index.to(device=device, dtype=torch.int64)
    out = torch.empty((3, index.numel()), dtype=dtype, device=device)
    for a in range(3):
        out[a] = hashed_lattice_quanta(n, seed, amp_log2, a, index).to(dtype) * QUANTUM
    return out


def planar_profile(n: int, axis: int, seed: int, amp_log2: int = 1, mom_log2: int = 0):
    """A lattice whose planes normal to ``axis`` move rigidly: per plane q (its
    Lagrangian index along ``axis``) an axis coordinate, transverse offsets and a
    momentum, all in quanta (int64):

      coord [3, N]: coord[axis][q] = wrapped lattice coordinate q + 1/2 plus a
                    hashed offset in [-2^amp_log2, 2^amp_log2) cells; the two
                    transverse rows are offsets (0) added to q_b + 1/2;
      mom   [3, N]: hashed momenta in [-2^mom_log2, 2^mom_log2) cells per unit drift.
    """
    q = torch.arange(n, dtype=torch.int64)
    coord = torch.zeros((3, n), dtype=torch.int64)
    span = n << QUANTUM_BITS
    coord[axis] = torch.remainder((q << QUANTUM_BITS) + (1 << (QUANTUM_BITS - 1))
                                  + _signed_quanta(counter_bits(q, 0, seed), amp_log2), span)
    mom = torch.stack([_signed_quanta(counter_bits(q, 1 + c, seed), mom_log2) for c in range(3)])
    return coord, mom


def expand_planar(coord: torch.Tensor, mom: torch.Tensor | None, n: int, axis: int, device=None,
                  dtype=torch.float32):
    """Full particle arrays [3, N^3] (Lagrangian order) of a plane-parallel
    configuration given per plane in quanta: the particle with lattice index q
    has coordinate coord[axis][q_axis] along ``axis`` and
    wrap(q_b + 1/2 + coord[b][q_axis]) along a transverse axis b; its momentum is
    mom[:, q_axis].  Returns (pos, mom) (mom None if not given)."""
    span = n << QUANTUM_BITS
    shape = [1, 1, 1]
    shape[axis] = n
    pos = torch.empty((3, n ** 3), dtype=dtype, device=device)
    coord = coord.to(device)
    qb = torch.arange(n, dtype=torch.int64, device=device)
    for b in range(3):
        view = pos[b].view(n, n, n)
        if b == axis:
            view.copy_((coord[b].to(dtype) * QUANTUM).view(shape).expand(n, n, n))
            continue
        # table over (q_axis, q_b), broadcast along the remaining axis
        tab = torch.remainder((qb.view(1, n) << QUANTUM_BITS) + (1 << (QUANTUM_BITS - 1))
                              + coord[b].view(n, 1), span).to(dtype) * QUANTUM
        shp = [1, 1, 1]
        shp[axis] = n
        shp[b] = n
        if axis < b:
            view.copy_(tab.view(shp).expand(n, n, n))
        else:
            view.copy_(tab.t().contiguous().view(shp).expand(n, n, n))
    if mom is None:
        return pos, None
    return pos, broadcast_planes(mom.to(torch.float64) * QUANTUM, n, axis, device=device, dtype=dtype)


def broadcast_planes(values: torch.Tensor, n: int, axis: int, device=None, dtype=torch.float32) -> torch.Tensor:
    """[3, N^3] particle array (Lagrangian order) whose entry for the particle with
    lattice index q is values[:, q_axis] (``values`` [3, N], one column per plane)."""
    shape = [1, 1, 1]
    shape[axis] = n
    out = torch.empty((3, n ** 3), dtype=dtype, device=device)
    values = values.to(device)
    for c in range(3):
        out[c].view(n, n, n).copy_(values[c].to(dtype).view(shape).expand(n, n, n))
    return out


def plane_wave_mesh(n: int, waves, device=None, dtype=torch.float32) -> torch.Tensor:
    """sum_j A_j cos(2 pi (m_j . x) / N + phase_j) on the [N, N, N] node lattice,
    evaluated in float64 on ``device`` from separable factors and rounded to
    ``dtype``; ``waves`` is a list of (A, (m_x, m_y, m_z), phase)."""
    x = torch.arange(n, dtype=torch.float64, device=device)
    out = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for amp, m, ph in waves:
        ex, ey, ez = (torch.polar(torch.ones_like(x), 2.0 * np.pi * float(mi) * x / n) for mi in m)
        e = ex.view(n, 1, 1) * ey.view(1, n, 1) * complex(np.cos(ph), np.sin(ph))
        for i0 in range(0, n, 64):
            out[i0:i0 + 64] += amp * (e[i0:i0 + 64] * ez.view(1, 1, n)).real
    return out.to(dtype)
