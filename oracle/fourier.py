"""DFT conventions and wavenumber grids (FP64).

Test infrastructure only (see ``oracle/__init__``).

Convention: the forward transform is unnormalised,
    dhat(n) = sum_x d(x) exp(-i k_g . x),   k_g = 2 pi n / N,
and the inverse carries 1/N^3.  The continuum Fourier amplitude of the paper's
power-spectrum and bispectrum definitions (eqs. powerspectrum, bispectre) is
(V/N^3) dhat, with V = L^3.  Integer frequencies n_d take the values
[-N/2, N/2) on the two full axes; the last axis of a real-to-complex transform
holds n_z = 0..N/2, where n_z = N/2 is the Nyquist plane (identified with -N/2).
"""
from __future__ import annotations

import math

import torch


def rfft3(d: torch.Tensor) -> torch.Tensor:
    """Real-to-complex forward DFT of an [N,N,N] mesh -> [N,N,N/2+1]."""
    return torch.fft.rfftn(d, dim=(-3, -2, -1))


def irfft3(dh: torch.Tensor, n: int) -> torch.Tensor:
    """Complex-to-real inverse DFT (with the 1/N^3 factor) -> [N,N,N]."""
    return torch.fft.irfftn(dh, s=(n, n, n), dim=(-3, -2, -1))


def int_freqs(n: int):
    """Integer frequency grids (nx, ny, nz) broadcastable to [N,N,N/2+1], int64.
    Full axes use [-N/2, N/2); the half axis uses 0..N/2."""
    full = torch.fft.fftfreq(n, d=1.0 / n).round().long()
    half = torch.arange(n // 2 + 1, dtype=torch.long)
    return full.view(n, 1, 1), full.view(1, n, 1), half.view(1, 1, n // 2 + 1)


def kgrid(n: int):
    """Grid wavenumbers k_g = 2 pi n / N for each axis, float64, broadcastable."""
    nx, ny, nz = int_freqs(n)
    s = 2.0 * math.pi / n
    return nx.double() * s, ny.double() * s, nz.double() * s


def nyquist_masks(n: int):
    """Boolean masks (broadcastable) of the Nyquist plane of each axis (|n_d| = N/2)."""
    nx, ny, nz = int_freqs(n)
    h = n // 2
    return nx.abs() == h, ny.abs() == h, nz == h


def r2c_weights(n: int) -> torch.Tensor:
    """Multiplicity of each stored r2c mode in the full cube: 1 on the n_z = 0 and
    n_z = N/2 planes (their partners -n are stored too), 2 elsewhere."""
    w = torch.full((n // 2 + 1,), 2.0, dtype=torch.float64)
    w[0] = 1.0
    w[n // 2] = 1.0
    return w.view(1, 1, n // 2 + 1)


def brute_dft3(d: torch.Tensor) -> torch.Tensor:
    """O(N^6) forward DFT written out as the definition (for pins on tiny meshes);
    returns the full [N,N,N] complex cube."""
    n = d.shape[0]
    idx = torch.arange(n, dtype=torch.float64)
    # 1-D DFT matrix exp(-2 pi i n x / N), applied once per axis is the same sum
    # factorised; to keep this an independent check we form the full 3-D phase.
    x = torch.stack(torch.meshgrid(idx, idx, idx, indexing="ij"), dim=-1).reshape(-1, 3)
    k = x.clone()   # integer frequencies 0..N-1 (aliases of [-N/2, N/2))
    phase = -2.0 * math.pi * (k @ x.T) / n
    mat = torch.complex(torch.cos(phase), torch.sin(phase))
    return (mat @ d.reshape(-1).to(torch.complex128)).reshape(n, n, n)


def plane_wave_modes(waves, n: int):
    """Stored r2c modes of sum_j A_j cos(2 pi m_j . x / N + phase_j): the DFT of a cosine
    is (N^3 A / 2) e^{+i phase} at +m and its conjugate at -m; the r2c half keeps the
    partner with n_z in (0, N/2), and both partners when n_z = 0 or N/2.  Returns
    (modes [M, 3] int64: n_x, n_y in [-N/2, N/2), n_z in [0, N/2]; values [M]
    complex128); wavevectors are reduced modulo N and coinciding modes are summed."""
    acc = {}

    def add(m, v):
        key = (((int(m[0]) + n // 2) % n) - n // 2, ((int(m[1]) + n // 2) % n) - n // 2, int(m[2]) % n)
        if key[2] > n // 2:
            return  # the conjugate partner is the stored one
        acc[key] = acc.get(key, 0j) + v

    for amp, m, ph in waves:
        v = 0.5 * amp * n ** 3 * complex(math.cos(ph), math.sin(ph))
        add(m, v)
        add(tuple(-c for c in m), v.conjugate())
    keys = sorted(acc)
    modes = torch.tensor(keys, dtype=torch.long).view(-1, 3)
    vals = torch.tensor([acc[k] for k in keys], dtype=torch.complex128)
    return modes, vals


def plane_wave_modes_full(waves, n: int):
    """Full-cube DFT of sum_j A_j cos(2 pi m_j . x / N + phase_j): (N^3 A / 2) e^{+i phase}
    at +m and its conjugate at -m, components reduced to [-N/2, N/2), coinciding
    modes summed.  Returns (modes [M, 3] int64, values [M] complex128)."""
    acc = {}
    for amp, m, ph in waves:
        v = 0.5 * amp * n ** 3 * complex(math.cos(ph), math.sin(ph))
        for sgn, val in ((1, v), (-1, v.conjugate())):
            key = tuple(((sgn * int(c) + n // 2) % n) - n // 2 for c in m)
            acc[key] = acc.get(key, 0j) + val
    keys = sorted(acc)
    return (torch.tensor(keys, dtype=torch.long).view(-1, 3),
            torch.tensor([acc[k] for k in keys], dtype=torch.complex128))


def idft_at(modes: torch.Tensor, values: torch.Tensor, n: int, points: torch.Tensor) -> torch.Tensor:
    """Inverse DFT (with 1/N^3) of a full-cube spectrum that vanishes except at
    ``modes`` ([M, 3]) with amplitudes ``values``, evaluated at ``points`` ([3, P],
    grid coordinates, not necessarily integers).  Returns complex128 [P]."""
    k = (2.0 * math.pi / n) * modes.to(torch.float64)                   # [M, 3]
    arg = k @ points.to(torch.float64)                                 # [M, P]
    e = torch.complex(torch.cos(arg), torch.sin(arg))
    return (values.view(-1, 1) * e).sum(dim=0) / n ** 3
