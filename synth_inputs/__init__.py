"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only draws random numbers and lays them out in the array shapes the
library consumes.  It holds none of the particle-mesh arithmetic: no Fourier
transforms, no mass assignment, no cosmology.  Everything here is a pure
function of (shape, seed), built on NumPy's counter-based Philox generator.

Conventions shared by every caller:
  * real meshes are ``[N, N, N]`` row-major, float64 unless asked otherwise;
  * particle arrays are structure-of-arrays ``[3, Np]`` in grid units
    (a coordinate lies in ``[0, N)``).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "white_noise",
    "uniform_particles",
    "clustered_particles",
    "lattice_jitter_particles",
    "random_complex_mesh",
    "random_real_mesh",
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
