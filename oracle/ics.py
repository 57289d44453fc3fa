"""Zel'dovich initial conditions for the Newtonian and Poisson-gauge particle sets (FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper starts all runs from the same random phases (Sec. 2 and Sec. 3),
with second-order initial conditions at z = 50 (Sec. 3).  This oracle uses the
first-order (Zel'dovich) displacement, as the benchmark configurations ask:

  * white noise w (unit variance per cell) is an input;
  * linear density: delta_L_hat(n) = DFT(w)(n) sqrt(P(k)/dx^3) D(a_i)/D(a_norm),
    with k = k_f |n|, k_f = 2 pi / L, the k = 0 mode and every Nyquist plane zeroed;
  * displacement: Psi_hat = i k_g delta_L_hat / k_g^2 (so -div Psi = delta_L),
    evaluated on the Lagrangian lattice q = (i + 1/2, j + 1/2, l + 1/2) by the
    phase factor exp(i k_g . (1/2, 1/2, 1/2));
  * Newtonian set: x = wrap(q + Psi), p = a^2 E(a) f(a) Psi  (grid units).

Poisson-gauge set (linear reading of eqs. physical_density, b1 and bgr): the
counting density of matter in Poisson gauge is, at linear order,
delta_N (1 + (3 f + (9/2) Omega_m(a)) H^2 / k^2), which is produced by the
extra displacement
    xi_lin_hat(n, a) = i k_g g(a) delta_L_hat(n) / k_g^4,
    g(a) = (3 f(a) + (9/2) Omega_m(a)) calH_g(a)^2 D(a)/D(a_i),
evaluated on the same lattice.  The relativistic set starts at
x_GR = wrap(x_N + xi_lin(a_i)), p_GR = p_N + a^2 E d xi_lin / d ln a.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import cic, cosmology as cm, fourier


@dataclass(frozen=True)
class ICParams:
    n: int                    # particles per axis = mesh cells per axis
    box: float                # L, Mpc/h
    a_init: float             # scale factor of the initial conditions
    power: cm.PowerSpec       # linear P(k) (Mpc/h)^3 at a_norm
    a_norm: float = 1.0       # scale factor at which ``power`` is the linear spectrum
    cosmo: cm.Cosmo = cm.FIDUCIAL

    @property
    def dx(self) -> float:
        return self.box / self.n


def _power_on_grid(p: ICParams) -> torch.Tensor:
    """P(k_f |n|) on the r2c grid, evaluated once per distinct |n|^2."""
    nx, ny, nz = fourier.int_freqs(p.n)
    n2 = (nx * nx + ny * ny + nz * nz)
    uniq, inv = torch.unique(n2.reshape(-1), return_inverse=True)
    kf = 2.0 * math.pi / p.box
    vals = torch.tensor([p.power(kf * math.sqrt(float(u))) for u in uniq.tolist()], dtype=torch.float64)
    return vals[inv].reshape(n2.shape)


def linear_delta_k(noise: torch.Tensor, p: ICParams) -> torch.Tensor:
    """delta_L_hat at a_init on the r2c grid (k = 0 and Nyquist planes zeroed)."""
    w_hat = fourier.rfft3(noise.to(torch.float64))
    growth = cm.growth_d(p.cosmo, p.a_init) / cm.growth_d(p.cosmo, p.a_norm)
    amp = torch.sqrt(_power_on_grid(p) / p.dx ** 3) * growth
    mx, my, mz = fourier.nyquist_masks(p.n)
    keep = ~(mx | my | mz)
    nx, ny, nz = fourier.int_freqs(p.n)
    keep = keep & ((nx != 0) | (ny != 0) | (nz != 0))
    return torch.where(keep, w_hat * amp, torch.zeros_like(w_hat))


def truncate_noise(noise: torch.Tensor, n_coarse: int) -> torch.Tensor:
    """White noise of a coarse run that shares the fine run's random phases (Secs. 2
    and 3 use the same initial phases for every simulation; reading for runs of
    different resolution): keep the fine modes with |n_i| < N_c/2 on every axis,
    scale by (N_c/N_f)^(3/2) so that the physical field (V/N^3) delta_hat is the same
    on the shared modes, drop the coarse Nyquist planes, transform back."""
    nf = noise.shape[-1]
    if nf % n_coarse != 0 or n_coarse > nf:
        raise ValueError("n_coarse must divide the fine mesh size")
    w_hat = fourier.rfft3(noise.to(torch.float64))
    out = torch.zeros((n_coarse, n_coarse, n_coarse // 2 + 1), dtype=torch.complex128)
    h = n_coarse // 2
    idx = torch.cat([torch.arange(0, h), torch.arange(nf - h + 1, nf)])          # n in (-N_c/2, N_c/2)
    cidx = torch.cat([torch.arange(0, h), torch.arange(n_coarse - h + 1, n_coarse)])
    sub = w_hat[idx][:, idx][:, :, :h]                                          # n_z in [0, N_c/2)
    out[cidx.view(-1, 1, 1), cidx.view(1, -1, 1), torch.arange(h).view(1, 1, -1)] = sub
    out *= (n_coarse / nf) ** 1.5
    return fourier.irfft3(out, n_coarse)


def fix_spectrum(w_hat: torch.Tensor, n: int) -> torch.Tensor:
    """Every mode keeps its phase and takes the expected modulus of unit white noise,
    |w_hat| = N^(3/2); modes with w_hat = 0 stay zero (no phase; reading)."""
    mag = w_hat.abs()
    return torch.where(mag > 0, w_hat / torch.where(mag > 0, mag, torch.ones_like(mag)) * n ** 1.5,
                       torch.zeros_like(w_hat))


def fixed_noise(noise: torch.Tensor, negate: bool = False) -> torch.Tensor:
    """Paired-and-fixed white noise (the pairing method cited in Sec. 4 for the
    bispectrum): the fixed spectrum of the noise, transformed back; the partner
    realisation is its negative (all phases shifted by pi)."""
    n = noise.shape[-1]
    out = fourier.irfft3(fix_spectrum(fourier.rfft3(noise.to(torch.float64)), n), n)
    return -out if negate else out


def _lattice_phase(n: int) -> torch.Tensor:
    kx, ky, kz = fourier.kgrid(n)
    ph = 0.5 * (kx + ky + kz)
    return torch.complex(torch.cos(ph), torch.sin(ph))


def _vector_field_on_lattice(scalar_hat: torch.Tensor, n: int, power_of_k2: int) -> torch.Tensor:
    """IDFT of i k_g scalar_hat / k_g^(2 p) with the half-cell lattice phase -> [3, N^3]."""
    kx, ky, kz = fourier.kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    inv = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)) ** power_of_k2,
                      torch.zeros_like(k2))
    base = scalar_hat * inv * _lattice_phase(n)
    comps = []
    for k in (kx, ky, kz):
        comps.append(fourier.irfft3(torch.complex(torch.zeros_like(k), k) * base, n).reshape(-1))
    return torch.stack(comps)


def lagrangian_lattice(n: int) -> torch.Tensor:
    """q_j = (i + 1/2, j + 1/2, l + 1/2) for particle (i N + j) N + l -> [3, N^3]."""
    q = torch.arange(n, dtype=torch.float64) + 0.5
    gx, gy, gz = torch.meshgrid(q, q, q, indexing="ij")
    return torch.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)])


def za_displacement(noise: torch.Tensor, p: ICParams) -> torch.Tensor:
    """Psi(q) at a_init, [3, N^3] in cells."""
    return _vector_field_on_lattice(linear_delta_k(noise, p), p.n, 1)


def zeldovich(noise: torch.Tensor, p: ICParams):
    """Newtonian set: (pos, mom), each [3, N^3] float64."""
    psi = za_displacement(noise, p)
    a = p.a_init
    pos = cic.wrap(lagrangian_lattice(p.n) + psi, p.n)
    mom = a * a * cm.hubble_e(p.cosmo, a) * cm.growth_f(p.cosmo, a) * psi
    return pos, mom


def gr_shift_coefficients(p: ICParams, a: float):
    """(g(a), dg/dlna) of the linear Poisson-gauge displacement at scale factor a."""
    c = p.cosmo
    calh2 = cm.conformal_hubble_grid(c, a, p.dx) ** 2
    om = cm.omega_m_of_a(c, a)
    f = cm.growth_f(c, a)
    fp = cm.growth_f_dlna(c, a)
    dratio = cm.growth_d(c, a) / cm.growth_d(c, p.a_init)
    s = 3.0 * f + 4.5 * om
    g = s * calh2 * dratio
    # d/dlna: s' = 3 f' + 4.5 Om', Om' = -3 Om (1 - Om); calH^2' = calH^2 (2 - 3 Om); D' = f D
    sp = 3.0 * fp - 13.5 * om * (1.0 - om)
    gp = calh2 * dratio * (sp + s * (2.0 - 3.0 * om + f))
    return g, gp


def xi_linear(noise: torch.Tensor, p: ICParams, a: float):
    """(xi_lin(a), d xi_lin / d ln a) on the lattice, each [3, N^3]."""
    base = _vector_field_on_lattice(linear_delta_k(noise, p), p.n, 2)
    g, gp = gr_shift_coefficients(p, a)
    return g * base, gp * base


def zeldovich_pair(noise: torch.Tensor, p: ICParams):
    """Newtonian and Poisson-gauge sets from the same noise:
    (pos_N, mom_N, pos_GR, mom_GR)."""
    pos_n, mom_n = zeldovich(noise, p)
    xi, dxi = xi_linear(noise, p, p.a_init)
    a = p.a_init
    pos_gr = cic.wrap(pos_n + xi, p.n)
    mom_gr = mom_n + a * a * cm.hubble_e(p.cosmo, a) * dxi
    return pos_n, mom_n, pos_gr, mom_gr


# ------------------------------------------------------------ second order --
#
# Sec. 3 starts the runs from second-order Lagrangian initial conditions.  The
# paper's discrete relativistic derivation is not reproducible from its text; the
# Newtonian set here is the standard continuous 2LPT (reading): with Psi1 = grad chi,
# lap chi = -delta_L (chi_hat = delta_L_hat / k^2),
#     S(q) = sum_{i<j} (chi_ii chi_jj - chi_ij^2),
#     Psi2 = c2 grad(-lap^-1 S),   Psi2_hat = c2 i k S_hat / k^2,
# c2 = -D2 / D1^2 = (3/7) Omega_m(a)^(-1/143) (the second-order growth factor
# D2 = -(3/7) D1^2 Omega_m^(-1/143)), and momenta a^2 E (f1 Psi1 + f2 Psi2) with
# f2 = dln D2 / dln a = 2 f1 + (3/143)(1 - Omega_m(a)).  S is formed from the Hessian
# sampled on the particle lattice and differentiated spectrally on the same samples
# (no de-aliasing of the product); k = 0 and the Nyquist planes of S_hat are dropped.

def lpt2_coefficients(p: ICParams):
    """(c2, f2) at a_init."""
    om = cm.omega_m_of_a(p.cosmo, p.a_init)
    c2 = (3.0 / 7.0) * om ** (-1.0 / 143.0)
    f2 = 2.0 * cm.growth_f(p.cosmo, p.a_init) + (3.0 / 143.0) * (1.0 - om)
    return c2, f2


def second_order_source(dl_hat: torch.Tensor, n: int) -> torch.Tensor:
    """S on the particle lattice, [N^3], from delta_L_hat on the r2c grid."""
    kx, ky, kz = fourier.kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    inv = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)), torch.zeros_like(k2))
    chi_hat = dl_hat * inv * _lattice_phase(n)
    k = (kx, ky, kz)
    h = {(i, j): fourier.irfft3(-k[i] * k[j] * chi_hat, n) for i in range(3) for j in range(i, 3)}
    s = (h[0, 0] * h[1, 1] + h[0, 0] * h[2, 2] + h[1, 1] * h[2, 2]
         - h[0, 1] ** 2 - h[0, 2] ** 2 - h[1, 2] ** 2)
    return s.reshape(-1)


def second_order_displacement(s: torch.Tensor, n: int, c2: float) -> torch.Tensor:
    """Psi2 = c2 IDFT(i k DFT(S) / k^2) on the same samples as S, [3, N^3]."""
    s_hat = fourier.rfft3(s.view(n, n, n))
    kx, ky, kz = fourier.kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    mx, my, mz = fourier.nyquist_masks(n)
    keep = ~(mx | my | mz) & (k2 > 0)
    inv = torch.where(keep, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)), torch.zeros_like(k2))
    base = c2 * s_hat * inv
    return torch.stack([fourier.irfft3(torch.complex(torch.zeros_like(k), k) * base, n).reshape(-1)
                        for k in (kx, ky, kz)])


def lpt2_displacement(noise: torch.Tensor, p: ICParams):
    """(Psi1, Psi2) at a_init, each [3, N^3] in cells."""
    dl = linear_delta_k(noise, p)
    c2, _ = lpt2_coefficients(p)
    return (_vector_field_on_lattice(dl, p.n, 1),
            second_order_displacement(second_order_source(dl, p.n), p.n, c2))


def lpt2(noise: torch.Tensor, p: ICParams):
    """Newtonian second-order set: (pos, mom), each [3, N^3] float64."""
    psi1, psi2 = lpt2_displacement(noise, p)
    _, f2 = lpt2_coefficients(p)
    a = p.a_init
    ae = a * a * cm.hubble_e(p.cosmo, a)
    pos = cic.wrap(lagrangian_lattice(p.n) + psi1 + psi2, p.n)
    mom = ae * (cm.growth_f(p.cosmo, a) * psi1 + f2 * psi2)
    return pos, mom


def powerlaw_for_rms_displacement(n: int, box: float, rms_cells: float, index: float = -2.0) -> cm.PowerSpec:
    """P(k) = A k^index with A chosen so that the expected 3-D rms Zel'dovich
    displacement over the discrete (non-Nyquist, n != 0) mode set is ``rms_cells``.

    By Parseval, E <|Psi|^2> = N^-3 sum_n P(k)/(dx^3 k_g^2) over the full cube, and with
    P = A k^index = A (k_g/dx)^index:  A = rms^2 dx^3 N^3 / sum_n dx^-index k_g^(index-2)."""
    dx = box / n
    f = torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64).round()
    nx, ny, nz = torch.meshgrid(f, f, f, indexing="ij")
    keep = (nx.abs() < n // 2) & (ny.abs() < n // 2) & (nz.abs() < n // 2)
    keep = keep & ((nx != 0) | (ny != 0) | (nz != 0))
    kg2 = (2.0 * math.pi / n) ** 2 * (nx * nx + ny * ny + nz * nz)
    terms = torch.where(keep, torch.where(keep, kg2, torch.ones_like(kg2)) ** ((index - 2.0) / 2.0),
                        torch.zeros_like(kg2))
    s = float(terms.sum()) * dx ** (-index)
    amp = rms_cells ** 2 * dx ** 3 * n ** 3 / s
    return cm.PowerSpec("powerlaw", amp, index)


def _linear_delta_sparse(modes: torch.Tensor, w_hat: torch.Tensor, p: ICParams) -> torch.Tensor:
    """``linear_delta_k`` at the full-cube modes ``modes`` ([M, 3], components in
    [-N/2, N/2)) of a noise spectrum that vanishes elsewhere."""
    growth = cm.growth_d(p.cosmo, p.a_init) / cm.growth_d(p.cosmo, p.a_norm)
    kf = 2.0 * math.pi / p.box
    out = torch.zeros_like(w_hat)
    for i, m in enumerate(modes.tolist()):
        if all(c == 0 for c in m) or any(c == -(p.n // 2) for c in m):
            continue   # k = 0 and the Nyquist planes carry no linear density
        amp = math.sqrt(p.power(kf * math.sqrt(sum(c * c for c in m))) / p.dx ** 3) * growth
        out[i] = w_hat[i] * amp
    return out


def zeldovich_pair_sparse(modes: torch.Tensor, w_hat: torch.Tensor, p: ICParams, q_index: torch.Tensor):
    """``zeldovich_pair`` for white noise whose full-cube spectrum vanishes except at
    ``modes`` with amplitudes ``w_hat``, evaluated for the particles with lattice
    indices q_index ([3, P]) only: (pos_N, mom_N, pos_GR, mom_GR), each [3, P]."""
    n = p.n
    dl = _linear_delta_sparse(modes, w_hat, p)
    kg = (2.0 * math.pi / n) * modes.to(torch.float64)
    k2 = (kg * kg).sum(dim=1)
    inv = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)), torch.zeros_like(k2))
    q = q_index.to(torch.float64) + 0.5           # the lattice point carries the half-cell phase
    psi = torch.stack([fourier.idft_at(modes, 1j * kg[:, d] * dl * inv, n, q).real for d in range(3)])
    base = torch.stack([fourier.idft_at(modes, 1j * kg[:, d] * dl * inv * inv, n, q).real for d in range(3)])
    a = p.a_init
    pos_n = cic.wrap(q + psi, n)
    mom_n = a * a * cm.hubble_e(p.cosmo, a) * cm.growth_f(p.cosmo, a) * psi
    g, gp = gr_shift_coefficients(p, a)
    pos_gr = cic.wrap(pos_n + g * base, n)
    mom_gr = mom_n + a * a * cm.hubble_e(p.cosmo, a) * gp * base
    return pos_n, mom_n, pos_gr, mom_gr


def xi_linear_sparse(modes: torch.Tensor, w_hat: torch.Tensor, p: ICParams, a: float, q_index: torch.Tensor):
    """``xi_linear(noise, p, a)[0]`` for white noise whose full-cube spectrum vanishes
    except at ``modes`` with amplitudes ``w_hat``, at the particles with lattice
    indices q_index ([3, P]) only.  Returns [3, P] in cells."""
    n = p.n
    dl = _linear_delta_sparse(modes, w_hat, p)
    kg = (2.0 * math.pi / n) * modes.to(torch.float64)
    k2 = (kg * kg).sum(dim=1)
    inv = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)), torch.zeros_like(k2))
    q = q_index.to(torch.float64) + 0.5
    g, _ = gr_shift_coefficients(p, a)
    return torch.stack([g * fourier.idft_at(modes, 1j * kg[:, d] * dl * inv * inv, n, q).real for d in range(3)])


def lpt2_sparse(modes: torch.Tensor, w_hat: torch.Tensor, p: ICParams, q_index: torch.Tensor):
    """``lpt2`` for white noise whose full-cube spectrum vanishes except at ``modes``
    (values ``w_hat``), at the particles with lattice indices q_index ([3, P]) only:
    (pos, mom), each [3, P].  The Hessian of chi is a sum over the modes, so S on the
    lattice is a sum over ordered mode pairs (m1, m2): its sample spectrum sits at
    m1 + m2 reduced to [-N/2, N/2) with the half-cell phase of the unreduced sum (the
    product aliases exactly as on the mesh)."""
    n = p.n
    dl = _linear_delta_sparse(modes, w_hat, p)
    kg = (2.0 * math.pi / n) * modes.to(torch.float64)
    k2 = (kg * kg).sum(dim=1)
    inv = torch.where(k2 > 0, 1.0 / torch.where(k2 > 0, k2, torch.ones_like(k2)), torch.zeros_like(k2))
    chi = dl * inv
    live = [i for i in range(modes.shape[0]) if chi[i] != 0]
    pairs = [(0, 1), (0, 2), (1, 2)]
    acc = {}
    for i1 in live:
        for i2 in live:
            k1, k2v = kg[i1], kg[i2]
            h1 = lambda a, b: -float(k1[a] * k1[b])
            h2 = lambda a, b: -float(k2v[a] * k2v[b])
            w = sum(h1(a, a) * h2(b, b) - h1(a, b) * h2(a, b) for a, b in pairs)
            if w == 0.0:
                continue
            msum = modes[i1] + modes[i2]
            ph = math.pi * float(msum.sum()) / n
            v = complex(chi[i1] * chi[i2]) * w * complex(math.cos(ph), math.sin(ph)) / n ** 3
            key = tuple(((int(c) + n // 2) % n) - n // 2 for c in msum)
            acc[key] = acc.get(key, 0j) + v
    c2, f2 = lpt2_coefficients(p)
    keys = [k for k in acc if any(c != 0 for c in k) and all(c != -(n // 2) for c in k)]
    psi2 = torch.zeros((3, q_index.shape[1]), dtype=torch.float64)
    if keys:
        sm = torch.tensor(keys, dtype=torch.long).view(-1, 3)
        sv = torch.tensor([acc[k] for k in keys], dtype=torch.complex128)
        sk = (2.0 * math.pi / n) * sm.to(torch.float64)
        sk2 = (sk * sk).sum(dim=1)
        psi2 = torch.stack([fourier.idft_at(sm, c2 * 1j * sk[:, d] * sv / sk2, n, q_index).real for d in range(3)])
    q = q_index.to(torch.float64) + 0.5
    psi1 = torch.stack([fourier.idft_at(modes, 1j * kg[:, d] * dl * inv, n, q).real for d in range(3)])
    a = p.a_init
    ae = a * a * cm.hubble_e(p.cosmo, a)
    return cic.wrap(q + psi1 + psi2, n), ae * (cm.growth_f(p.cosmo, a) * psi1 + f2 * psi2)


def truncate_noise_sparse(modes: torch.Tensor, w_hat: torch.Tensor, n_fine: int, n_coarse: int):
    """``truncate_noise`` of a fine noise spectrum that vanishes except at ``modes``:
    the coarse spectrum's non-zero modes (|n_i| < N_c/2 kept, scaled by
    (N_c/N_f)^(3/2)) as (modes [K, 3], values [K])."""
    h = n_coarse // 2
    keep = (modes.abs() < h).all(dim=1)
    return modes[keep].clone(), w_hat[keep] * (n_coarse / n_fine) ** 1.5


def zeldovich_adjoint_sparse(lam_pos_spectra, lam_mom_spectra, p: ICParams, cells: torch.Tensor) -> torch.Tensor:
    """Cotangent of the white noise at ``cells`` ([3, M] integer) for cotangents
    (lam_pos, lam_mom) of the Newtonian set of ``zeldovich``, given as sparse
    full-cube DFTs of their three components on the particle lattice (lists of
    (modes [K, 3], values [K]), components in [-N/2, N/2)).  The set is linear in the
    noise, Psi_d = IDFT(A_d DFT(w)) with A_d = i k_d T(k) e^{i k . (1/2, 1/2, 1/2)} / k^2
    (T the factor of ``linear_delta_k``, zero at k = 0 and on the Nyquist planes), pos
    = q + Psi (the wrap has unit derivative) and mom = c_m Psi; so the cotangent of the
    noise is IDFT(sum_d conj(A_d) DFT(lam_pos_d + c_m lam_mom_d)).  Returns [M]."""
    n = p.n
    a = p.a_init
    c_m = a * a * cm.hubble_e(p.cosmo, a) * cm.growth_f(p.cosmo, a)
    growth = cm.growth_d(p.cosmo, p.a_init) / cm.growth_d(p.cosmo, p.a_norm)
    kf = 2.0 * math.pi / p.box
    acc = {}
    for d in range(3):
        for (modes, vals), f in ((lam_pos_spectra[d], 1.0), (lam_mom_spectra[d], c_m)):
            for m, v in zip(modes.tolist(), vals.tolist()):
                if all(c == 0 for c in m) or any(c == -(n // 2) for c in m):
                    continue
                kg = [2.0 * math.pi * c / n for c in m]
                k2 = sum(x * x for x in kg)
                t = math.sqrt(p.power(kf * math.sqrt(sum(c * c for c in m))) / p.dx ** 3) * growth
                ph = 0.5 * sum(kg)
                amp = 1j * kg[d] * t / k2 * complex(math.cos(ph), math.sin(ph))
                key = tuple(m)
                acc[key] = acc.get(key, 0j) + amp.conjugate() * f * v
    if not acc:
        return torch.zeros(cells.shape[1], dtype=torch.float64)
    keys = sorted(acc)
    modes = torch.tensor(keys, dtype=torch.long).view(-1, 3)
    vals = torch.tensor([acc[k] for k in keys], dtype=torch.complex128)
    return fourier.idft_at(modes, vals, n, cells).real
