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
