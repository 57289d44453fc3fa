"""Pins of the oracle's forms for full-size (1024^3) parity, where the oracle
evaluates sampled outputs one by one: the node-centred CIC density, the
plane-parallel reduction of the cycle, the combination at sampled particles, the
spectrum of a sum of plane waves and the P(k) estimator of a sparse spectrum.
Each is pinned against the independent dense oracle (corner-enumerated deposit;
3-D Fourier solve, gather, kick and drift; dense combine; 3-D DFT; dense
estimator) on small meshes, where the two must agree to rounding."""
import math

import pytest
import torch

import synth_inputs as si
from oracle import cic, cosmology as ocm, integrate, planar, solve


def test_rho_at_nodes_equals_corner_deposit():
    n = 8
    x = torch.from_numpy(si.uniform_particles(n, 300, 4))
    rho = cic.deposit_rho(x, n)
    g = torch.arange(n)
    nodes = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = cic.rho_at_nodes(nodes, x, n)
    assert torch.allclose(got, rho.reshape(-1), atol=1e-12)
    assert float(got.sum()) == pytest.approx(300.0, rel=1e-13)


def test_rho_at_nodes_wraps_and_ignores_far_particles():
    n = 16
    # a particle at 15.25 along x shares its weight between nodes 15 (0.75) and 0 (0.25)
    x = torch.tensor([[15.25, 7.0], [3.0, 7.0], [4.0, 7.0]], dtype=torch.float64)
    nodes = torch.tensor([[15, 0, 14, 7], [3, 3, 3, 7], [4, 4, 4, 7]])
    got = cic.rho_at_nodes(nodes, x, n)
    assert got.tolist() == pytest.approx([0.75, 0.25, 0.0, 1.0], abs=1e-15)


def _planar_case(n, axis, seed, offset):
    coord, mom = si.planar_profile(n, axis, seed, amp_log2=1, mom_log2=-1)
    coord[(axis + 1) % 3] = offset
    c = coord.double() * si.QUANTUM
    m = mom.double() * si.QUANTUM
    pos, p3 = si.expand_planar(coord, mom, n, axis, dtype=torch.float64)
    return c, m, pos, p3


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("grad", ["spectral", "fd2", "fd1"])
def test_planar_cycle_equals_3d_oracle(axis, grad):
    n = 16
    om = ocm.FIDUCIAL.omega_m
    c, m, pos, p3 = _planar_case(n, axis, 20 + axis, 3 * 8192 + 77)
    kick, drift = 0.8, 1.7
    c1, m1, f1 = planar.cycle_line(c, m, axis, kick, drift, n, om, grad)

    meshes = solve.newton_forces(cic.deposit_delta(pos, n), om, grad)
    want = torch.zeros_like(meshes)
    shape = [1, 1, 1]
    shape[axis] = n
    want[axis] = f1.view(shape).expand(n, n, n)
    assert torch.allclose(meshes, want, atol=1e-12)

    wx, wv = integrate.force_then_kick_drift(pos, p3, kick, drift, integrate.NewtonForce(n, grad=grad), 0.0, n)
    g = torch.arange(n)
    q = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got_x = planar.particle_coords(c1, axis, n, q)
    d = torch.remainder(got_x - wx + n / 2, n) - n / 2
    assert float(d.abs().max()) < 1e-12
    assert torch.allclose(m1[:, q[axis]], wv, atol=1e-12)


def test_planar_density_is_mass_conserving_and_uniform_lattice_is_force_free():
    n = 32
    om = ocm.FIDUCIAL.omega_m
    x = torch.arange(n, dtype=torch.float64) + 0.5
    assert torch.allclose(planar.deposit_delta_line(x, n), torch.zeros(n, dtype=torch.float64), atol=1e-15)
    coord, _ = si.planar_profile(n, 0, 3)
    d = planar.deposit_delta_line(coord[0].double() * si.QUANTUM, n)
    assert abs(float(d.sum())) < 1e-12
    assert float(planar.newton_force_line(d, om).sum()) == pytest.approx(0.0, abs=1e-12)


# ------------------------------------------------------------- sampled forms --

def test_combine_at_equals_dense_combine():
    from oracle import combine as ocomb
    for nc, nf in ((8, 32), (8, 8), (4, 12)):
        xg = torch.from_numpy(si.lattice_jitter_particles(nc, 3, 1.7))
        xn = torch.from_numpy(si.lattice_jitter_particles(nc, 4, 1.7))
        xf = torch.from_numpy(si.lattice_jitter_particles(nf, 5, 0.9))
        want = ocomb.combine(xg, xn, nc, xf, nf)
        idx = torch.arange(0, nf ** 3, 7)
        j = torch.stack([idx // (nf * nf), (idx // nf) % nf, idx % nf])
        got = ocomb.combine_at(xg, xn, nc, xf[:, idx], j, nf)
        assert torch.allclose(got, want[:, idx], atol=1e-12)


def test_plane_wave_modes_equal_rfft():
    from oracle import fourier
    n = 8
    waves = [(0.3, (1, -2, 3), 0.4), (0.2, (4, 0, 0), 1.1), (0.1, (0, 3, 4), 2.0), (0.05, (-3, 1, 0), 0.3),
             (0.07, (1, 2, -3), 0.9)]
    x = torch.arange(n, dtype=torch.float64)
    g = torch.stack(torch.meshgrid(x, x, x, indexing="ij"))
    d = sum(a * torch.cos(2 * math.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n + ph) for a, m, ph in waves)
    dh = fourier.rfft3(d)
    modes, vals = fourier.plane_wave_modes(waves, n)
    want = torch.zeros_like(dh)
    for (mx, my, mz), v in zip(modes.tolist(), vals.tolist()):
        want[mx % n, my % n, mz] += v
    assert torch.allclose(dh, want, atol=1e-9)


@pytest.mark.parametrize("n,nb", [(16, 8), (32, 16), (24, 5)])
def test_power_spectrum_sparse_equals_dense(n, nb):
    from oracle import estimators, fourier
    g = torch.Generator().manual_seed(n)
    dh = torch.zeros((n, n, n // 2 + 1), dtype=torch.complex128)
    pick = torch.randint(0, n * n * (n // 2 + 1), (40,), generator=g)
    vals = torch.randn(40, generator=g, dtype=torch.float64) + 1j * torch.randn(40, generator=g, dtype=torch.float64)
    dh.view(-1)[pick] = vals
    nxf, nyf, nzf = fourier.int_freqs(n)
    flat = torch.nonzero(dh.abs().reshape(-1) > 0).view(-1)
    ix, iy, iz = flat // (n * (n // 2 + 1)), (flat // (n // 2 + 1)) % n, flat % (n // 2 + 1)
    modes = torch.stack([nxf.view(-1)[ix], nyf.view(-1)[iy], nzf.view(-1)[iz]], 1)
    km, pk, cnt = estimators.power_spectrum_sparse(modes, dh.reshape(-1)[flat], n, 700.0, nb)
    wkm, wpk, wcnt = estimators.power_spectrum_from_k(dh, n, 700.0, nb)
    assert torch.equal(cnt, wcnt)
    assert torch.allclose(km, wkm, rtol=1e-12)
    assert torch.allclose(pk, wpk, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,nb", [(16, 8), (32, 5)])
def test_cross_spectrum_sparse_equals_dense(n, nb):
    from oracle import estimators, fourier
    wa = [(0.3, (1, 0, 0), 0.1), (0.2, (0, 5, 0), 1.0), (0.15, (3, -7, 2), 2.0), (0.1, (n // 2 - 1, 1, 3), 0.5)]
    wb = [(0.7 * a, m, ph + 0.3 * i) for i, (a, m, ph) in enumerate(wa)]
    ma, va = fourier.plane_wave_modes(wa, n)
    mb, vb = fourier.plane_wave_modes(wb, n)
    assert torch.equal(ma, mb)
    km, pk, cnt = estimators.power_spectrum_sparse(ma, va, n, 700.0, nb, values_b=vb)
    wkm, wpk, wcnt = estimators.cross_power_spectrum(_cosine_mesh(wa, n), _cosine_mesh(wb, n), 700.0, nb)
    assert torch.equal(cnt, wcnt)
    assert torch.allclose(km, wkm, rtol=1e-12)
    assert torch.allclose(pk, wpk, rtol=1e-10, atol=1e-12 * float(wpk.abs().max()))
    assert float(wpk.abs().max()) > 0


def test_sparse_bispectrum_pieces_equal_dense_estimator():
    from oracle import estimators, fourier
    n, box = 16, 300.0
    waves = [(0.3, (3, 0, 0), 0.2), (0.25, (-1, 3, 0), 0.9), (0.2, (-2, -3, 0), 1.7), (0.1, (7, 1, -1), 0.4),
             (0.1, (-7, 6, 1), 2.2), (0.05, (0, -7, 0), 0.0),
             # closes only modulo N: (7,0,0) + (7,1,0) + (2,-1,0) = (16,0,0)
             (0.1, (7, 0, 0), 0.5), (0.12, (7, 1, 0), 1.3), (0.08, (2, -1, 0), 2.9)]
    x = torch.arange(n, dtype=torch.float64)
    g = torch.stack(torch.meshgrid(x, x, x, indexing="ij"))
    d = sum(a * torch.cos(2 * math.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n + ph) for a, m, ph in waves)
    centres, width = [3.0, 7.0, 5.0], 2.0
    tris = [(0, 0, 0), (1, 1, 1), (0, 0, 2), (1, 1, 0), (2, 1, 1)]
    wb, wn = estimators.bispectrum(d, box, centres, width, tris)
    modes, vals = fourier.plane_wave_modes_full(waves, n)
    full = torch.fft.fftn(d.to(torch.complex128))
    got_full = torch.zeros_like(full)
    for (a, b, c), v in zip(modes.tolist(), vals.tolist()):
        got_full[a % n, b % n, c % n] += v
    assert torch.allclose(full, got_full, atol=1e-9)
    nonzero = 0
    for t, tri in enumerate(tris):
        cnt = estimators.triangle_count(n, centres, width, tri)
        assert cnt == pytest.approx(float(wn[t]), abs=1e-6)
        num = estimators.bispectrum_numerator_sparse(modes, vals, n, centres, width, tri)
        want = box ** 6 / n ** 9 * num.real / cnt if cnt else 0.0
        assert want == pytest.approx(float(wb[t]), rel=1e-9, abs=1e-9 * float(wb.abs().max()))
        nonzero += abs(num) > 0
    assert nonzero >= 2   # the direct triangle in shell 0 and the aliased one in (1, 1, 0)


@pytest.mark.parametrize("axis", [0, 2])
def test_planar_vjp_equals_3d_oracle_vjp(axis):
    from oracle import adjoint as oadj
    n = 16
    om = ocm.FIDUCIAL.omega_m
    c, m, pos, p3 = _planar_case(n, axis, 50 + axis, 2 * 8192 + 5)
    g = torch.Generator().manual_seed(7 + axis)
    lc = torch.randn((3, n), generator=g, dtype=torch.float64)
    lm = torch.randn((3, n), generator=g, dtype=torch.float64)
    kick, drift = 0.37, 0.55
    gc, gm = planar.cycle_line_vjp(c, m, axis, kick, drift, n, om, lc, lm)
    lx3 = si.broadcast_planes(lc, n, axis, dtype=torch.float64)
    lp3 = si.broadcast_planes(lm, n, axis, dtype=torch.float64)
    wx, wp = oadj.step_vjp(pos, p3, kick, drift, n, ocm.FIDUCIAL, lx3, lp3)
    assert torch.allclose(si.broadcast_planes(gc, n, axis, dtype=torch.float64), wx, atol=1e-11)
    assert torch.allclose(si.broadcast_planes(gm, n, axis, dtype=torch.float64), wp, atol=1e-11)
    assert float((gc[axis] - lc[axis]).abs().max()) > 1e-3   # the force term contributes


NOISE_WAVES = [(0.02, (1, 0, 0), 0.3), (0.05, (2, -3, 1), 1.2), (0.3, (5, 5, -7), 2.2), (0.4, (-7, 2, 3), 0.7),
               (0.2, (8, 1, 0), 0.1)]


def _cosine_mesh(waves, n):
    x = torch.arange(n, dtype=torch.float64)
    g = torch.stack(torch.meshgrid(x, x, x, indexing="ij"))
    return sum(a * torch.cos(2 * math.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n + ph) for a, m, ph in waves)


def test_idft_at_equals_inverse_fft():
    from oracle import fourier
    n = 8
    modes, vals = fourier.plane_wave_modes_full(NOISE_WAVES, n)
    g = torch.arange(n)
    pts = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = fourier.idft_at(modes, vals, n, pts).real
    assert torch.allclose(got, _cosine_mesh(NOISE_WAVES, n).reshape(-1), atol=1e-12)


@pytest.mark.parametrize("kind", ["powerlaw", "eh98"])
def test_zeldovich_pair_sparse_equals_dense(kind):
    from oracle import fourier, ics as oics
    n, box = 16, 500.0
    c = ocm.Cosmo(n_s=0.965)
    power = oics.powerlaw_for_rms_displacement(n, box, 0.5) if kind == "powerlaw" else ocm.eh98_normalised(c, 0.965, 0.81)
    p = oics.ICParams(n=n, box=box, a_init=0.05, power=power, a_norm=1.0, cosmo=c)
    noise = _cosine_mesh(NOISE_WAVES, n)
    want = oics.zeldovich_pair(noise, p)
    modes, vals = fourier.plane_wave_modes_full(NOISE_WAVES, n)
    g = torch.arange(n)
    q = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = oics.zeldovich_pair_sparse(modes, vals, p, q)
    for a, b in zip(got, want):
        assert float(torch.remainder(a - b + n / 2, n).sub(n / 2).abs().max()) < 1e-11
    disp = torch.remainder(want[0] - (q + 0.5) + n / 2, n) - n / 2
    assert float(disp.abs().max()) > 1e-3   # a displacement that is not trivially zero


@pytest.mark.parametrize("a", [0.05, 0.5, 1.0])
def test_xi_linear_sparse_equals_dense(a):
    from oracle import fourier, ics as oics
    n, box = 16, 500.0
    c = ocm.Cosmo(n_s=0.965)
    p = oics.ICParams(n=n, box=box, a_init=0.05, power=ocm.eh98_normalised(c, 0.965, 0.81), a_norm=1.0, cosmo=c)
    want, _ = oics.xi_linear(_cosine_mesh(NOISE_WAVES, n), p, a)
    modes, vals = fourier.plane_wave_modes_full(NOISE_WAVES, n)
    g = torch.arange(n)
    q = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = oics.xi_linear_sparse(modes, vals, p, a, q)
    scale = float(want.abs().max())
    assert scale > 1e-5   # about 1e-4 cells on this coarse 31 Mpc/h mesh
    assert float((got - want).abs().max()) < 1e-12 * scale


@pytest.mark.parametrize("n", [16, 12])
def test_lpt2_sparse_equals_dense(n):
    # includes mode pairs whose sum wraps past the Nyquist frequency (aliasing, with
    # the sign the half-cell lattice phase gives it)
    from oracle import fourier, ics as oics
    box = 500.0
    c = ocm.Cosmo(n_s=0.965)
    p = oics.ICParams(n=n, box=box, a_init=0.05, power=ocm.eh98_normalised(c, 0.965, 0.81), a_norm=1.0, cosmo=c)
    waves = [(0.5, (1, 0, 2), 0.3), (1.0, (3, -2, 5), 1.2), (0.8, (-4, 5, 1), 2.2), (0.3, (2, 2, -5), 0.9)]
    noise = _cosine_mesh(waves, n)
    want = oics.lpt2(noise, p)
    psi2 = oics.lpt2_displacement(noise, p)[1]
    modes, vals = fourier.plane_wave_modes_full(waves, n)
    g = torch.arange(n)
    q = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = oics.lpt2_sparse(modes, vals, p, q)
    assert float(psi2.abs().max()) > 1e-3 * float((want[0] - q - 0.5).abs().max())
    assert float(torch.remainder(got[0] - want[0] + n / 2, n).sub(n / 2).abs().max()) < 1e-11
    assert float((got[1] - want[1]).abs().max()) < 1e-11 * float(want[1].abs().max())


def test_truncate_noise_sparse_equals_dense():
    from oracle import fourier, ics as oics
    nf, nc = 16, 8
    noise = _cosine_mesh(NOISE_WAVES, nf)
    want = oics.truncate_noise(noise, nc)
    modes, vals = fourier.plane_wave_modes_full(NOISE_WAVES, nf)
    cm_, cv = oics.truncate_noise_sparse(modes, vals, nf, nc)
    g = torch.arange(nc)
    pts = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = fourier.idft_at(cm_, cv, nc, pts).real
    assert torch.allclose(got, want.reshape(-1), atol=1e-12)
    assert float(want.abs().max()) > 0.1


@pytest.mark.parametrize("axis", [0, 2])
def test_planar_power_spectrum_and_vjp_equal_3d_oracle(axis):
    from oracle import adjoint as oadj, estimators
    n, box, nb = 16, 300.0, 8
    c, m, pos, _ = _planar_case(n, axis, 60 + axis, 0)
    _, pk3, cnt = estimators.power_spectrum(cic.deposit_delta(pos, n), box, nb)
    _, _, cnt_sparse = estimators.power_spectrum_sparse(torch.zeros((0, 3), dtype=torch.long),
                                                        torch.zeros(0, dtype=torch.complex128), n, box, nb)
    assert torch.equal(cnt, cnt_sparse)
    pk1 = planar.power_spectrum_line(c[axis], n, box, nb, cnt)
    assert torch.allclose(pk1, pk3, rtol=1e-10, atol=1e-10 * float(pk3.abs().max()))
    dpk = torch.randn(nb, generator=torch.Generator().manual_seed(3), dtype=torch.float64)
    (want,) = oadj.vjp(lambda x: estimators.power_spectrum(cic.deposit_delta(x, n), box, nb)[1], (pos,), dpk)
    g = planar.power_spectrum_line_vjp(c[axis], n, box, nb, cnt, dpk)
    full = torch.zeros((3, n), dtype=torch.float64)
    full[axis] = g
    got = si.broadcast_planes(full, n, axis, dtype=torch.float64)
    assert torch.allclose(got, want, atol=1e-10 * float(want.abs().max()))
    assert float(g.abs().max()) > 0


def test_zeldovich_adjoint_sparse_equals_autograd():
    from oracle import adjoint as oadj, fourier, ics as oics
    n, box = 16, 500.0
    c = ocm.Cosmo(n_s=0.965)
    p = oics.ICParams(n=n, box=box, a_init=0.05, power=ocm.eh98_normalised(c, 0.965, 0.81), a_norm=1.0, cosmo=c)
    pos_waves = [[(0.7, (1, 2, -3), 0.2), (0.2, (8, 1, 0), 0.5)], [(0.5, (0, 3, 1), 1.0)],
                 [(0.3, (-5, 2, 7), 2.0), (0.4, (2, 2, 2), 0.1)]]
    mom_waves = [[(1.1, (3, -1, 0), 0.4)], [(0.9, (1, 2, -3), 2.5), (0.2, (0, 0, 8), 0.0)], [(0.6, (4, 0, 1), 1.4)]]
    lx = torch.stack([_cosine_mesh(w, n).reshape(-1) for w in pos_waves])
    lp = torch.stack([_cosine_mesh(w, n).reshape(-1) for w in mom_waves])
    noise = _cosine_mesh(NOISE_WAVES, n)

    def fwd(w):
        x, m = oics.zeldovich(w, p)
        return torch.cat([x.reshape(-1), m.reshape(-1)])

    (want,) = oadj.vjp(fwd, (noise,), torch.cat([lx.reshape(-1), lp.reshape(-1)]))
    g = torch.arange(n)
    cells = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = oics.zeldovich_adjoint_sparse([fourier.plane_wave_modes_full(w, n) for w in pos_waves],
                                        [fourier.plane_wave_modes_full(w, n) for w in mom_waves], p, cells)
    assert torch.allclose(got, want.reshape(-1), atol=1e-10 * float(want.abs().max()))
    assert float(want.abs().max()) > 1e-3
