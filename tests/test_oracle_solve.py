"""Pins of the oracle's Newtonian and Poisson-gauge potential solves."""
import math

import pytest
import torch

import synth_inputs as si
from oracle import cic, cosmology as cm, fourier, solve

OM = cm.FIDUCIAL.omega_m


def _plane_wave(n, m, amp=0.3, phase=0.4):
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    k = [2 * math.pi * mi / n for mi in m]
    arg = k[0] * gx + k[1] * gy + k[2] * gz + phase
    return k, arg, amp


@pytest.mark.parametrize("m", [(1, 0, 0), (2, -3, 1), (0, 5, 7)])
def test_plane_wave_potential_and_force(m):
    # delta = A cos(k.x)  =>  phi = -(3/2) Om A cos(k.x)/k^2 and F = -grad phi exactly.
    n = 16
    k, arg, amp = _plane_wave(n, m)
    delta = amp * torch.cos(arg)
    k2 = sum(ki * ki for ki in k)
    phi = fourier.irfft3(solve.newton_potential_k(fourier.rfft3(delta), OM), n)
    assert torch.allclose(phi, -1.5 * OM * amp * torch.cos(arg) / k2, atol=1e-13)
    f = solve.newton_forces(delta, OM)
    for d in range(3):
        want = -1.5 * OM * amp * k[d] * torch.sin(arg) / k2
        assert torch.allclose(f[d], want, atol=1e-13)


def test_finite_difference_gradients_on_plane_wave():
    n = 16
    m = (1, 2, 0)
    k, arg, amp = _plane_wave(n, m, phase=0.0)
    delta = amp * torch.cos(arg)
    k2 = sum(ki * ki for ki in k)
    phi = -1.5 * OM * amp * torch.cos(arg) / k2
    # central difference: F_d = -(phi(x + e_d) - phi(x - e_d)) / 2
    f2 = solve.newton_forces(delta, OM, "fd2")
    f1 = solve.newton_forces(delta, OM, "fd1")
    for d in range(3):
        sh_p = torch.roll(phi, shifts=-1, dims=d)
        sh_m = torch.roll(phi, shifts=1, dims=d)
        assert torch.allclose(f2[d], -(sh_p - sh_m) / 2, atol=1e-13)
        assert torch.allclose(f1[d], -(sh_p - phi), atol=1e-13)


@pytest.mark.parametrize("grad", ["spectral", "fd2"])
def test_zero_net_self_force(grad):
    n = 16
    for seed in range(3):
        pos = torch.from_numpy(si.uniform_particles(n, 1, seed=seed))
        f = cic.gather(solve.newton_forces(cic.deposit_delta(pos, n), OM, grad), pos)
        assert float(f.abs().max()) < 1e-14
    pos = torch.from_numpy(si.clustered_particles(n, 2000, seed=7))
    f = cic.gather(solve.newton_forces(cic.deposit_delta(pos, n), OM, grad), pos)
    assert float(f.sum(dim=1).abs().max()) < 1e-10 * float(f.abs().sum())


def _gp(a, dx, c=cm.FIDUCIAL, inv_dtau=0.0, c_g=None):
    cg = cm.c_grid(dx) if c_g is None else c_g
    return solve.GaugeParams(a=a, om_a=cm.omega_m_of_a(c, a), calh=a * cm.hubble_e(c, a) / cg,
                             c_g=cg, inv_dtau=inv_dtau)


def test_gauge_solve_reduces_to_newton_for_infinite_c():
    n = 16
    delta = torch.from_numpy(si.random_real_mesh(n, 5)) * 0.1
    phi0 = torch.zeros((n, n, n // 2 + 1), dtype=torch.complex128)
    fn = solve.newton_forces(delta, OM)
    fg, _ = solve.poisson_gauge_forces(delta, phi0, _gp(0.5, 10.0, c_g=1e9, inv_dtau=1e-9))
    assert torch.allclose(fg, fn, rtol=1e-7, atol=1e-10 * float(fn.abs().max()))


@pytest.mark.parametrize("inv_dtau", [0.0, 0.05])
def test_gauge_linear_fixed_point_in_eds(inv_dtau):
    # Einstein-de Sitter (f = 1, Om = 1): the comoving-gauge potential is constant in time and
    # phi = -(3/2) H^2 delta_N / k^2.  The Poisson-gauge counting density implied by
    # eq. physical_density is delta_c = delta_N (1 + (3 f + 9/2 Om) H^2 / k^2).  Feeding that
    # delta_c and phi_old = phi must return phi unchanged, for any dtau.
    eds = cm.Cosmo(omega_c=0.95, omega_b=0.05)
    n, dx, a = 16, 2000.0, 0.3
    calh = a * cm.hubble_e(eds, a) / cm.c_grid(dx)
    dn = fourier.rfft3(torch.from_numpy(si.random_real_mesh(n, 8)))
    k2 = solve.k_squared(n)
    safe = torch.where(k2 > 0, k2, torch.ones_like(k2))
    phi_true = torch.where(k2 > 0, -1.5 * calh ** 2 * dn / safe, torch.zeros_like(dn))
    dc = torch.where(k2 > 0, dn * (1 + 7.5 * calh ** 2 / safe), torch.zeros_like(dn))
    gp = solve.GaugeParams(a=a, om_a=1.0, calh=calh, c_g=cm.c_grid(dx), inv_dtau=inv_dtau)
    got = solve.poisson_gauge_potential_k(dc, phi_true, gp)
    assert torch.allclose(got, phi_true, rtol=1e-12, atol=1e-14 * float(phi_true.abs().max()))


def test_gauge_potential_decouples_per_mode():
    # The solve is diagonal in k: a field with a single mode produces a single mode.
    n = 8
    dc = torch.zeros((n, n, n // 2 + 1), dtype=torch.complex128)
    dc[1, 2, 3] = 1.0 + 0.5j
    got = solve.poisson_gauge_potential_k(dc, torch.zeros_like(dc), _gp(0.4, 500.0, inv_dtau=0.01))
    mask = torch.ones_like(got.real, dtype=torch.bool)
    mask[1, 2, 3] = False
    assert float(got[mask].abs().max()) == 0.0
    assert abs(complex(got[1, 2, 3])) > 0
