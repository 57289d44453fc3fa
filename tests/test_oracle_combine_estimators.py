"""Pins of the oracle's displacement combination and P(k)/B(k) estimators."""
import itertools
import math

import pytest
import torch

import synth_inputs as si
from oracle import cic, combine, estimators, fourier


# ---------------------------------------------------------------------------
# eq. xiGR / eq. combined
# ---------------------------------------------------------------------------

def test_combine_identity_at_equal_resolution():
    # N_f = N_c and x_fine = x_N  =>  x = x_N + (x_GR - x_N) = x_GR.
    n = 16
    xn = torch.from_numpy(si.uniform_particles(n, n ** 3, seed=1))
    xg = cic.wrap(xn + 0.7 * torch.from_numpy(si.rng(2).standard_normal((3, n ** 3))), n)
    out = combine.combine(xg, xn, n, xn, n)
    d = (out - xg + n / 2) % n - n / 2
    assert float(d.abs().max()) < 1e-12


def test_min_image_across_the_seam():
    n = 8
    xg = torch.tensor([[0.1], [7.9], [4.0]], dtype=torch.float64)
    xn = torch.tensor([[7.8], [0.2], [3.5]], dtype=torch.float64)
    xi = combine.xi_min_image(xg, xn, n)
    assert torch.allclose(xi[:, 0], torch.tensor([0.3, -0.3, 0.5], dtype=torch.float64), atol=1e-14)


def test_fine_to_coarse_offsets_for_ratio_four():
    i0, t = combine.fine_to_coarse_axis(4, 16)
    assert sorted(set(t.tolist())) == [0.125, 0.375, 0.625, 0.875]
    # fine particle j sits at (j + 1/2) dx_f = coarse coordinate u + 1/2 in coarse cells
    u = i0.double() + t
    j = torch.arange(16, dtype=torch.float64)
    assert torch.allclose((u + 0.5) * 4, j + 0.5)


def test_constant_shift_and_linear_field_interpolation():
    nc, nf = 8, 32
    # constant xi -> uniform shift of (N_f/N_c) xi
    xn = cic.wrap(torch.from_numpy(si.uniform_particles(nc, nc ** 3, seed=3)), nc)
    shift = torch.tensor([0.3, -0.2, 0.05], dtype=torch.float64).view(3, 1)
    xg = cic.wrap(xn + shift, nc)
    xf = torch.from_numpy(si.uniform_particles(nf, nf ** 3, seed=4))
    out = combine.combine(xg, xn, nc, xf, nf)
    d = (out - xf - 4 * shift + nf / 2) % nf - nf / 2
    assert float(d.abs().max()) < 1e-12
    # CIC reproduces a field that is linear in the Lagrangian coordinate away from the seam
    q = torch.arange(nc, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(q, q, q, indexing="ij")
    xi = torch.stack([0.01 * gx + 0.02 * gy, -0.03 * gz, 0.005 * gx * 0 + 0.1]).reshape(3, -1)
    fine = combine.interpolate_lagrangian(xi, nc, nf).view(3, nf, nf, nf)
    i0, t = combine.fine_to_coarse_axis(nc, nf)
    u = i0.double() + t
    inside = (i0 >= 0) & (i0 < nc - 1)
    ux, uy, uz = torch.meshgrid(u, u, u, indexing="ij")
    m = inside.view(-1, 1, 1) & inside.view(1, -1, 1) & inside.view(1, 1, -1)
    assert torch.allclose(fine[0][m], (0.01 * ux + 0.02 * uy)[m], atol=1e-14)
    assert torch.allclose(fine[1][m], (-0.03 * uz)[m], atol=1e-14)
    assert torch.allclose(fine[2], torch.full_like(fine[2], 0.1), atol=1e-14)


def test_add_displacement_brute_force_periodic_cic():
    # Fine particle j sits at coarse coordinate u_j = (j + 1/2) N_c/N_f - 1/2; its value
    # is sum_i xi_i prod_axes max(0, 1 - |u - i|) over the periodic coarse lattice.
    for nc, nf in ((4, 12), (3, 6), (5, 5)):
        g = si.rng(7)
        xi = torch.from_numpy(g.standard_normal((3, nc ** 3)))
        xf = torch.from_numpy(g.uniform(0, nf, (3, nf ** 3)))
        got = combine.add_displacement(xi, nc, xf, nf)
        want = torch.empty_like(xf)
        for jx, jy, jz in itertools.product(range(nf), repeat=3):
            u = [(j + 0.5) * nc / nf - 0.5 for j in (jx, jy, jz)]
            acc = [0.0, 0.0, 0.0]
            for ix, iy, iz in itertools.product(range(nc), repeat=3):
                w = 1.0
                for uu, ii in zip(u, (ix, iy, iz)):
                    d = abs(uu - ii)
                    d = min(d, nc - d)
                    w *= max(0.0, 1.0 - d)
                if w:
                    for c in range(3):
                        acc[c] += w * float(xi[c, (ix * nc + iy) * nc + iz])
            jj = (jx * nf + jy) * nf + jz
            for c in range(3):
                v = float(xf[c, jj]) + nf / nc * acc[c]
                want[c, jj] = v - nf * math.floor(v / nf)
        d = (got - want + nf / 2) % nf - nf / 2
        assert float(d.abs().max()) < 1e-12


def test_add_displacement_of_the_run_difference_is_the_combination():
    nc, nf = 8, 16
    xn = torch.from_numpy(si.lattice_jitter_particles(nc, 11, 1.3))
    xg = torch.from_numpy(si.lattice_jitter_particles(nc, 12, 1.3))
    xf = torch.from_numpy(si.lattice_jitter_particles(nf, 13, 0.8))
    got = combine.add_displacement(combine.xi_min_image(xg, xn, nc), nc, xf, nf)
    want = combine.combine(xg, xn, nc, xf, nf)
    assert float(((got - want + nf / 2) % nf - nf / 2).abs().max()) < 1e-12
    idx = torch.arange(0, nf ** 3, 5)
    j = torch.stack([idx // (nf * nf), (idx // nf) % nf, idx % nf])
    at = combine.add_displacement_at(combine.xi_min_image(xg, xn, nc), nc, xf[:, idx], j, nf)
    assert float(((at - want[:, idx] + nf / 2) % nf - nf / 2).abs().max()) < 1e-12


# ---------------------------------------------------------------------------
# eq. powerspectrum
# ---------------------------------------------------------------------------

def test_pk_of_plane_wave_closed_form():
    # delta = A cos(2 pi m.x/N): |dhat(+-m)| = A N^3/2 and all else 0, so the bin holding |m| has
    # P = (V/N^6) 2 (A N^3/2)^2 / count = V A^2 / (2 count).
    n, box, amp = 16, 300.0, 0.37
    m = (2, 1, -2)                                     # |m| = 3
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    d = amp * torch.cos(2 * math.pi * (m[0] * gx + m[1] * gy + m[2] * gz) / n)
    k, p, cnt = estimators.power_spectrum(d, box, 8)
    b = 2                                              # w = 1: bin b = [b + 1/2, b + 3/2)
    assert float(p[b]) == pytest.approx(box ** 3 * amp ** 2 / (2 * int(cnt[b])), rel=1e-12)
    assert float(p.abs().sum() - p[b].abs()) < 1e-20


@pytest.mark.parametrize("n,nb", [(8, 4), (12, 6), (16, 4)])
def test_pk_mode_counts_brute_force(n, nb):
    w = (n / 2) / nb
    cnt = [0] * nb
    f = torch.fft.fftfreq(n, d=1.0 / n).round().long().tolist()
    for a, b, c in itertools.product(f, f, f):
        r = math.sqrt(a * a + b * b + c * c)
        for i in range(nb):
            if w * (i + 0.5) <= r < w * (i + 1.5):
                cnt[i] += 1
    _, _, got = estimators.power_spectrum(torch.zeros((n, n, n), dtype=torch.float64), float(n), nb)
    assert got.tolist() == cnt


def test_pk_white_noise_expectation():
    # i.i.d. cells with variance s^2: E|dhat|^2 = N^3 s^2, so E[P] = s^2 V / N^3 = s^2 dx^3.
    n, box, s = 32, 640.0, 1.7
    ps = []
    for seed in range(4):
        d = torch.from_numpy(si.random_real_mesh(n, 70 + seed)) * s
        _, p, cnt = estimators.power_spectrum(d, box, 16)
        ps.append(p)
    pm = torch.stack(ps).mean(0)
    dx = box / n
    assert float(pm.mean()) == pytest.approx(s * s * dx ** 3, rel=0.02)


# ---------------------------------------------------------------------------
# eq. bispectre
# ---------------------------------------------------------------------------

def test_bispectrum_fft_equals_brute_force_triangles():
    n, box = 8, 100.0
    d = torch.from_numpy(si.random_real_mesh(n, 17))
    centres = [2.0, 3.0, 1.0, 2.5]
    tris = [(0, 0, 0), (1, 1, 2), (0, 1, 1), (3, 3, 0)]
    b_fft, n_fft = estimators.bispectrum(d, box, centres, 1.0, tris)
    b_bf, n_bf = estimators.brute_bispectrum(d, box, centres, 1.0, tris)
    assert torch.allclose(n_fft, n_bf, rtol=1e-10)
    assert torch.allclose(b_fft, b_bf, rtol=1e-9, atol=1e-12 * float(b_bf.abs().max()))


def test_bispectrum_of_three_plane_waves():
    # delta = sum_a A_a cos(k_a.x + t_a) with k1 + k2 + k3 = 0 in three distinct shells:
    # the only non-zero closed triangles are (k1, k2, k3) and its negative, so
    # B = (V^2/N^9) (N^9/4) A1 A2 A3 cos(t1 + t2 + t3) / N_tri = V^2 A1 A2 A3 cos(t1+t2+t3) / (4 N_tri).
    n, box = 16, 250.0
    ms = [(1, 0, 0), (0, 2, 0), (-1, -2, 0)]
    amps = [0.3, 0.2, 0.25]
    ths = [0.1, -0.4, 0.7]
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    d = sum(a * torch.cos(2 * math.pi * (m[0] * gx + m[1] * gy + m[2] * gz) / n + t)
            for a, m, t in zip(amps, ms, ths))
    centres = [1.0, 2.0, math.sqrt(5.0)]
    b, ntri = estimators.bispectrum(d, box, centres, 0.2, [(0, 1, 2)])   # disjoint shells
    want = box ** 6 * amps[0] * amps[1] * amps[2] * math.cos(sum(ths)) / (4 * float(ntri[0]))
    assert float(b[0]) == pytest.approx(want, rel=1e-9)
    assert float(ntri[0]) == pytest.approx(round(float(ntri[0])), abs=1e-6)


def test_triangle_count_brute_force():
    n = 8
    centres = [1.0, 2.0, 3.0]
    tris = [(0, 1, 1), (1, 1, 1), (1, 2, 2), (0, 2, 2)]
    _, n_fft = estimators.bispectrum(torch.zeros((n, n, n), dtype=torch.float64), 1.0, centres, 1.0, tris)
    f = torch.fft.fftfreq(n, d=1.0 / n).round().long().tolist()
    modes = list(itertools.product(f, f, f))

    def shell(m):
        r2 = 4 * (m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        return [i for i, c in enumerate(centres) if (2 * c - 1) ** 2 <= r2 < (2 * c + 1) ** 2]

    def fold(v):
        v %= n
        return v - n if v >= n // 2 else v

    want = []
    for a, b, c in tris:
        cnt = 0
        for m1 in modes:
            if a not in shell(m1):
                continue
            for m2 in modes:
                if b not in shell(m2):
                    continue
                m3 = tuple(fold(-(m1[i] + m2[i])) for i in range(3))
                if c in shell(m3):
                    cnt += 1
        want.append(cnt)
    assert n_fft.round().long().tolist() == want


# ---------------------------------------------------------------------------
# cross spectrum and scale-dependent bias fit (Sec. 5, eq. b1)
# ---------------------------------------------------------------------------

def test_cross_spectrum_special_cases():
    n, box, nb = 16, 300.0, 8
    g = si.rng(3)
    a = torch.from_numpy(g.standard_normal((n, n, n)))
    e = torch.from_numpy(g.standard_normal((n, n, n)))
    k0, p0, c0 = estimators.power_spectrum(a, box, nb)
    k1, p1, c1 = estimators.cross_power_spectrum(a, a, box, nb)
    assert torch.equal(c0, c1) and torch.allclose(k0, k1, rtol=1e-15)
    assert torch.allclose(p1, p0, rtol=1e-13)
    # bilinear: P(a, 2a + e) = 2 P(a, a) + P(a, e); symmetric; Cauchy-Schwarz per bin
    _, pab, _ = estimators.cross_power_spectrum(a, 2 * a + e, box, nb)
    _, pae, _ = estimators.cross_power_spectrum(a, e, box, nb)
    _, pea, _ = estimators.cross_power_spectrum(e, a, box, nb)
    _, pee, _ = estimators.power_spectrum(e, box, nb)
    assert torch.allclose(pab, 2 * p0 + pae, rtol=1e-12, atol=1e-12 * float(p0.abs().max()))
    assert torch.allclose(pae, pea, rtol=1e-14)
    assert bool((pae.abs() <= torch.sqrt(p0 * pee) * (1 + 1e-12)).all())
    # one plane wave in each field, same mode, phase lag phi: P_ab = (V/N^6) w |a||b| cos(phi) / count
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    arg = 2 * math.pi * (3 * gx + gy - 2 * gz) / n
    _, pc, cnt = estimators.cross_power_spectrum(torch.cos(arg), 2 * torch.cos(arg + 0.6), box, nb)
    b = int(estimators.pk_bin_index(n, nb)[3, 1, 2])
    want = box ** 3 / n ** 6 * 2 * (n ** 3 / 2) * (n ** 3) * math.cos(0.6) / float(cnt[b])
    assert float(pc[b]) == pytest.approx(want, rel=1e-12)


def test_bias_fit_recovers_exact_coefficients_and_reduces_to_the_mean():
    k = torch.linspace(0.002, 0.12, 40, dtype=torch.float64)
    cnt = torch.arange(1, 41) * 6
    calh = 3.3e-4
    ratio = 1.7 + 2.9 * calh ** 2 / k ** 2 - 15.0 * k ** 2
    b1, bgr, c2 = estimators.bias_fit(k, ratio, cnt, 0.08, calh)
    assert (b1, bgr, c2) == (pytest.approx(1.7, rel=1e-10), pytest.approx(2.9, rel=1e-8), pytest.approx(-15.0, rel=1e-8))
    # the first two bins below the cut are dropped: corrupting them changes nothing
    bad = ratio.clone()
    bad[:2] += 100.0
    assert estimators.bias_fit(k, bad, cnt, 0.08, calh) == pytest.approx((b1, bgr, c2), rel=1e-9)
    # bins at and above the cut are ignored
    bad = ratio.clone()
    bad[k >= 0.08] = -50.0
    assert estimators.bias_fit(k, bad, cnt, 0.08, calh) == pytest.approx((b1, bgr, c2), rel=1e-9)
    # a constant ratio without scale dependence: b1 is the (weighted) mean, b1_GR = 0
    noise = torch.from_numpy(si.rng(4).standard_normal(40)) * 0.01
    sel = slice(2, int((k < 0.08).sum()))
    r = 1.3 + noise
    b1, bgr, _ = estimators.bias_fit(k, r, cnt, 0.08, calh, with_k2=False)
    # normal equations: the weighted residual is orthogonal to both columns
    kk, rr, ww = k[sel], r[sel], cnt[sel].double()
    res = rr - b1 - bgr * calh ** 2 / kk ** 2
    assert abs(float((ww * res).sum())) < 1e-12
    assert abs(float((ww * res / kk ** 2).sum())) < 1e-12 * float((ww / kk ** 2).sum())
