"""Pins of the oracle's DFT conventions and CIC assignment."""
import itertools
import math

import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import cic, fourier, estimators


@pytest.mark.parametrize("n", [4, 6])
def test_rfft_equals_brute_force_dft(n):
    d = torch.from_numpy(si.random_real_mesh(n, 11 + n))
    full = fourier.brute_dft3(d)
    half = fourier.rfft3(d)
    assert torch.allclose(half, full[:, :, : n // 2 + 1], atol=1e-10 * n ** 3)


def test_parseval_and_roundtrip():
    n = 16
    d = torch.from_numpy(si.random_real_mesh(n, 3))
    dh = fourier.rfft3(d)
    w = fourier.r2c_weights(n)
    assert float((w * dh.abs() ** 2).sum()) / n ** 3 == pytest.approx(float((d * d).sum()), rel=1e-12)
    assert torch.allclose(fourier.irfft3(dh, n), d, atol=1e-12)


def test_single_mode_impulse():
    n = 8
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    m = (1, -2, 3)
    d = torch.cos(2 * math.pi * (m[0] * gx + m[1] * gy + m[2] * gz) / n)
    dh = fourier.rfft3(d)
    # cos -> N^3/2 at +m and -m; +m (nz = 3) is stored, -m is its conjugate partner.
    assert abs(complex(dh[1, n - 2, 3]) - n ** 3 / 2) < 1e-9
    dh[1, n - 2, 3] = 0
    assert float(dh.abs().max()) < 1e-9


def _tent_deposit(pos, n):
    """Brute force: rho(c) = sum_p prod_d max(0, 1 - periodic distance(x_pd, c_d))."""
    rho = np.zeros((n, n, n))
    for p in range(pos.shape[1]):
        for c in itertools.product(range(n), repeat=3):
            w = 1.0
            for d in range(3):
                dist = abs(pos[d, p] - c[d])
                dist = min(dist, n - dist)
                w *= max(0.0, 1.0 - dist)
            rho[c] += w
    return rho


def test_deposit_equals_tent_function_brute_force():
    n = 5
    pos = si.uniform_particles(n, 7, seed=5)
    pos[:, 0] = [4.75, 0.25, 4.999]            # straddles every periodic face
    got = cic.deposit_rho(torch.from_numpy(pos), n).numpy()
    assert np.allclose(got, _tent_deposit(pos, n), atol=1e-13)


def test_deposit_mass_conservation_and_contrast():
    n = 16
    pos = torch.from_numpy(si.clustered_particles(n, 5000, seed=2))
    rho = cic.deposit_rho(pos, n)
    assert float(rho.sum()) == pytest.approx(5000.0, rel=1e-14)
    d = cic.deposit_delta(pos, n)
    assert float(d.mean()) == pytest.approx(0.0, abs=1e-13)


def test_particle_on_node_goes_to_one_cell():
    n = 8
    pos = torch.tensor([[3.0], [0.0], [7.0]], dtype=torch.float64)
    rho = cic.deposit_rho(pos, n)
    assert float(rho[3, 0, 7]) == 1.0
    assert float(rho.sum()) == 1.0


def test_gather_is_transpose_of_deposit():
    n = 12
    pos = torch.from_numpy(si.uniform_particles(n, 300, seed=9))
    m = torch.from_numpy(si.rng(1).standard_normal(300))
    a = torch.from_numpy(si.random_real_mesh(n, 4))
    lhs = float((cic.deposit_rho(pos, n, m) * a).sum())
    rhs = float((m * cic.gather(a, pos)).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_gather_of_linear_field_is_exact_inside():
    n = 10
    pos = torch.from_numpy(si.uniform_particles(n, 200, seed=3))
    pos = pos.clamp(0.0, n - 1.0 - 1e-9)                 # away from the periodic seam
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    f = 2.0 * gx - 0.5 * gy + 0.25 * gz + 1.0
    got = cic.gather(f, pos)
    assert torch.allclose(got, 2.0 * pos[0] - 0.5 * pos[1] + 0.25 * pos[2] + 1.0, atol=1e-12)


def test_wrap_rule():
    n = 16
    x = torch.tensor([-0.5, 16.0, 31.5, 3.25, -16.0])
    assert torch.equal(cic.wrap(x.double(), n), torch.tensor([15.5, 0.0, 15.5, 3.25, 0.0], dtype=torch.float64))
    # a float32 value just below 0 wraps to N after rounding and must come back to 0
    y = torch.tensor([-1e-9], dtype=torch.float32)
    assert float(cic.wrap(y, n)[0]) == 0.0


@pytest.mark.slow
def test_cic_poisson_shot_noise():
    # Poisson particles: E[|dhat(n)|^2] = N^6/Np * prod_d [1 - (2/3) sin^2(pi n_d / N)]
    # (CIC aliasing sum for uncorrelated points; no deconvolution).
    n, npart, reps = 16, 4096, 40
    acc = torch.zeros((n, n, n // 2 + 1), dtype=torch.float64)
    for r in range(reps):
        pos = torch.from_numpy(si.uniform_particles(n, npart, seed=100 + r))
        acc += fourier.rfft3(cic.deposit_delta(pos, n)).abs() ** 2
    acc /= reps
    nx, ny, nz = fourier.int_freqs(n)
    pred = (n ** 6 / npart) * ((1 - 2 / 3 * torch.sin(math.pi * nx / n) ** 2)
                               * (1 - 2 / 3 * torch.sin(math.pi * ny / n) ** 2)
                               * (1 - 2 / 3 * torch.sin(math.pi * nz / n) ** 2))
    ratio = (acc / pred).reshape(-1)[1:]              # drop k = 0
    assert float(ratio.mean()) == pytest.approx(1.0, abs=0.01)
    # and per |n| shell, a few percent
    kb, pb, cnt = estimators.power_spectrum_from_k(acc.sqrt().to(torch.complex128), n, float(n), 8)
    kp, pp, _ = estimators.power_spectrum_from_k(pred.sqrt().to(torch.complex128), n, float(n), 8)
    assert torch.allclose(pb, pp, rtol=0.05)
