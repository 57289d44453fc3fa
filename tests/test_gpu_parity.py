"""Parity of every C-ABI entry point against the FP64 oracle on identical inputs.

Bar: FP64 plans agree to ~1e-10 relative L2 (rounding order only); FP32 plans agree
to 1e-5 relative L2 on fields; integer decisions (cell and shell assignment, mode
counts) are bit-exact.  Sizes span several workgroups and ragged tails.
"""
import math

import numpy as np
import pytest
import torch

import synth_inputs as si
from oracle import cic, combine as ocomb, cosmology as ocm, estimators, ics as oics, integrate, solve as osolve

gpu = pytest.mark.gpu
pytestmark = gpu

pm = pytest.importorskip("paper_2404_02783_amd")

F32_TOL = 1e-5
F64_TOL = 1e-10


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def _tol(dt):
    return F32_TOL if dt == torch.float32 else F64_TOL


def rel_l2(a, b):
    a = torch.as_tensor(a).double().cpu()
    b = torch.as_tensor(b).double().cpu()
    return float(torch.linalg.norm((a - b).reshape(-1)) / max(float(torch.linalg.norm(b.reshape(-1))), 1e-300))


def min_image(d, n):
    return (d + n / 2) % n - n / 2


DTYPES = [torch.float32, torch.float64]


# ----------------------------------------------------------------- deposit --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,np_,kind", [(32, 32 ** 3, "lattice"), (64, 100003, "clustered"), (16, 777, "uniform"),
                                         (128, 128 ** 3, "lattice"), (128, 128 ** 3, "lattice_far"),
                                         (128, 128 ** 3, "lattice_vfar"), (256, 256 ** 3, "lattice")])
def test_deposit(dt, n, np_, kind):
    # FP32 N^3 lattice runs at N >= 64 take the tiled path: each Lagrangian tile sums its
    # particles in an LDS window (32-bit fixed point, scale 2^21) that is flushed with one
    # global float atomic per non-empty cell.  "lattice_far" moves particles up to 5
    # cells, so windows outgrow the LDS capacity and shrink to fit_box's box, and the
    # particles outside it take global atomics; "lattice_vfar" moves them up to 20 cells.
    dev = _dev()
    if kind == "lattice":
        x = si.lattice_jitter_particles(n, 3, 0.7, dtype=np.float64)
    elif kind == "lattice_far":
        x = si.lattice_jitter_particles(n, 4, 5.0, dtype=np.float64)
    elif kind == "lattice_vfar":
        x = si.lattice_jitter_particles(n, 6, 20.0, dtype=np.float64)
    elif kind == "clustered":
        x = si.clustered_particles(n, np_, 4)
    else:
        x = si.uniform_particles(n, np_, 5)
    pos = torch.from_numpy(x).to(dt)
    pos[pos >= n] = 0          # a coordinate just below N can round up to N in float32
    pos = pos.to(dev).contiguous()
    plan = pm.Plan(n, 100.0, dt)
    d = pm.pm_deposit(plan, pos)
    torch.cuda.synchronize()
    want = cic.deposit_delta(pos.double().cpu(), n)
    assert rel_l2(d, want) < _tol(dt)
    pm.pm_check(plan)


def test_deposit_batched_boxes():
    """A batch of three 128^3 lattice boxes (tiled LDS-window path, box index in the grid)
    against the oracle per box."""
    dev = _dev()
    n = 128
    xs = [si.lattice_jitter_particles(n, 40 + b, 0.7 + 3 * b, dtype=np.float64) for b in range(3)]
    pos = torch.from_numpy(np.stack(xs)).to(torch.float32)
    pos[pos >= n] = 0
    plan = pm.Plan(n, 100.0, torch.float32, dev, batch=3)
    d = pm.pm_deposit(plan, pos.to(dev).contiguous())
    torch.cuda.synchronize()
    for b in range(3):
        assert rel_l2(d[b], cic.deposit_delta(pos[b].double(), n)) < F32_TOL


@pytest.mark.parametrize("dt", DTYPES)
def test_deposit_assignment_bit_exact_on_nodes(dt):
    # particles exactly on nodes put all their weight in one cell: the integer assignment
    # decides the result, which must match the oracle exactly.
    dev = _dev()
    n = 16
    g = si.rng(8)
    x = g.integers(0, n, size=(3, 5000)).astype(np.float64)
    x[:, :3] = [[0, 15, 7], [15, 0, 7], [0, 15, 7]]
    pos = torch.from_numpy(x).to(dt).to(dev)
    plan = pm.Plan(n, 100.0, dt)
    d = pm.pm_deposit(plan, pos).double().cpu()
    want = cic.deposit_delta(torch.from_numpy(x), n)
    # counts are integers times N^3/Np: compare the counts exactly
    scale = 5000 / n ** 3
    assert torch.equal(torch.round((d + 1) * scale), torch.round((want + 1) * scale))


def test_deposit_empty_and_guards():
    dev = _dev()
    n = 8
    plan = pm.Plan(n, 10.0, torch.float32)
    d = pm.pm_deposit(plan, torch.empty((3, 0), dtype=torch.float32, device=dev))
    assert torch.all(d == -1)
    pm.pm_check(plan)
    pos = torch.tensor([[1.5, float("nan"), 9.5], [1.5, 2.0, 1.0], [1.5, 2.0, 1.0]], device=dev)
    pm.pm_deposit(plan, pos)
    with pytest.raises(pm.PMError) as e:
        pm.pm_check(plan)
    assert e.value.code == -5
    pm.pm_check(plan)   # counters were cleared


# ------------------------------------------------------------------- solve --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 192])
def test_newton_solve_random_field(dt, n):
    dev = _dev()
    delta = torch.from_numpy(si.random_real_mesh(n, 100 + n))
    plan = pm.Plan(n, 500.0, dt)
    f = pm.pm_solve(plan, delta.to(dt).to(dev), pm.newton_params())
    torch.cuda.synchronize()
    want = osolve.newton_forces(delta.to(dt).double(), ocm.FIDUCIAL.omega_m)
    assert rel_l2(f, want) < _tol(dt)


@pytest.mark.parametrize("grad", [pm.PM_GRAD_FD2, pm.PM_GRAD_FD1])
def test_newton_solve_fd_gradients(grad):
    dev = _dev()
    n = 32
    delta = torch.from_numpy(si.random_real_mesh(n, 7))
    plan = pm.Plan(n, 500.0, torch.float64)
    f = pm.pm_solve(plan, delta.to(dev), pm.newton_params(grad=grad))
    want = osolve.newton_forces(delta, ocm.FIDUCIAL.omega_m, {1: "fd2", 2: "fd1"}[grad])
    assert rel_l2(f, want) < F64_TOL


@pytest.mark.parametrize("dt", DTYPES)
def test_plane_wave_force_closed_form(dt):
    dev = _dev()
    n = 64
    x = torch.arange(n, dtype=torch.float64)
    gx, gy, gz = torch.meshgrid(x, x, x, indexing="ij")
    m = (3, -5, 7)
    k = [2 * math.pi * v / n for v in m]
    arg = k[0] * gx + k[1] * gy + k[2] * gz
    delta = 0.2 * torch.cos(arg)
    plan = pm.Plan(n, 500.0, dt)
    f = pm.pm_solve(plan, delta.to(dt).to(dev), pm.newton_params()).double().cpu()
    k2 = sum(v * v for v in k)
    for d in range(3):
        want = -1.5 * ocm.FIDUCIAL.omega_m * 0.2 * k[d] * torch.sin(arg) / k2
        assert rel_l2(f[d], want) < _tol(dt)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [16, 64])
def test_poisson_gauge_solve(dt, n):
    dev = _dev()
    box = 8000.0
    delta = torch.from_numpy(si.random_real_mesh(n, 300 + n)) * 0.05
    # the carried potential is the spectrum of a real field (Hermitian on the n_z = 0, N/2 planes)
    phi0 = torch.fft.rfftn(torch.from_numpy(si.random_real_mesh(n, 301)) * 1e-6)
    phi0[0, 0, 0] = 0
    sp = pm.gauge_params(box, n, 0.4, 0.35)
    plan = pm.Plan(n, box, dt)
    cd = torch.complex64 if dt == torch.float32 else torch.complex128
    phi = phi0.to(cd).to(dev).clone().contiguous()
    f = pm.pm_solve(plan, delta.to(dt).to(dev), sp, phi_state=phi)
    torch.cuda.synchronize()
    gp = osolve.GaugeParams(a=sp.a, om_a=sp.om_a, calh=sp.calh, c_g=sp.c_g, inv_dtau=sp.inv_dtau)
    wf, wphi = osolve.poisson_gauge_forces(delta.to(dt).double(), phi0.to(cd).to(torch.complex128), gp)
    assert rel_l2(f, wf) < _tol(dt)
    got_phi = phi.cpu().to(torch.complex128)
    assert rel_l2(torch.view_as_real(got_phi), torch.view_as_real(wphi)) < _tol(dt)


# ------------------------------------------------------------------ gather --

@pytest.mark.parametrize("dt", DTYPES)
def test_gather(dt):
    dev = _dev()
    n = 32
    force = torch.from_numpy(np.stack([si.random_real_mesh(n, s) for s in (1, 2, 3)]))
    x = torch.from_numpy(si.clustered_particles(n, 50001, 6))
    plan = pm.Plan(n, 100.0, dt)
    xd = x.to(dt).to(dev).contiguous()
    acc = pm.pm_gather(plan, force.to(dt).to(dev).contiguous(), xd)
    want = cic.gather(force.to(dt).double(), xd.double().cpu())
    assert rel_l2(acc, want) < _tol(dt)


# -------------------------------------------------------------------- step --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,amp", [(32, 0.8), (128, 0.4), (128, 0.8), (128, 6.0)])
def test_step_matches_force_kick_drift(dt, n, amp):
    # FP32 N^3 lattice runs at N >= 64 stage forces through LDS windows: whole at
    # amp = 0.4, only the touched cells at 0.8 (boxes past the sparse threshold); amp = 6
    # pushes tiles past the window capacity so the direct-read fallback runs too.
    dev = _dev()
    x = torch.from_numpy(si.lattice_jitter_particles(n, 9, amp))
    v = torch.from_numpy(si.rng(10).standard_normal((3, n ** 3))) * 0.05
    plan = pm.Plan(n, 200.0, dt)
    pos, mom = x.to(dt).to(dev).contiguous(), v.to(dt).to(dev).contiguous()
    pos0, mom0 = pos.double().cpu().clone(), mom.double().cpu().clone()
    st = pm.StepParams(kick=0.7, drift=1.3, solve=pm.newton_params())
    force = plan.mesh(3)
    pm.pm_step(plan, pos, mom, st, force)
    torch.cuda.synchronize()
    f = integrate.NewtonForce(n)
    wx, wv = integrate.force_then_kick_drift(pos0, mom0, 0.7, 1.3, f, 0.0, n)
    assert rel_l2(mom, wv) < _tol(dt)
    d = min_image(pos.double().cpu() - wx, n)
    assert float(torch.linalg.norm(d)) / float(torch.linalg.norm(wx)) < _tol(dt)


# ----------------------------------------------------------------- combine --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("nc,nf", [(8, 32), (16, 16), (16, 32), (32, 288)])
def test_displacement_combine(dt, nc, nf):
    dev = _dev()
    xn = torch.from_numpy(si.lattice_jitter_particles(nc, 11, 0.9))
    xg = cic.wrap(xn + 0.3 * torch.from_numpy(si.rng(12).standard_normal((3, nc ** 3))), nc)
    xf = torch.from_numpy(si.lattice_jitter_particles(nf, 13, 0.9))
    a, b, c = (t.to(dt).to(dev).contiguous() for t in (xg, xn, xf))
    out = pm.displacement_combine(a, b, nc, c, nf)
    want = ocomb.combine(a.double().cpu(), b.double().cpu(), nc, c.double().cpu(), nf)
    d = min_image(out.double().cpu() - want, nf)
    tol = 1e-6 if dt == torch.float32 else 1e-12
    assert float(d.abs().max()) < tol * nf


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("nc,nf", [(8, 32), (16, 16), (32, 288)])
def test_displacement_add(dt, nc, nf):
    dev = _dev()
    xi = 0.6 * torch.from_numpy(si.rng(21).standard_normal((3, nc ** 3)))
    xf = torch.from_numpy(si.lattice_jitter_particles(nf, 22, 0.9))
    a, c = (t.to(dt).to(dev).contiguous() for t in (xi, xf))
    want = ocomb.add_displacement(a.double().cpu(), nc, c.double().cpu(), nf)
    out = pm.displacement_add(a, nc, c, nf)
    pm.displacement_add(a, nc, c, nf, x_out=c)          # in place
    tol = 1e-6 if dt == torch.float32 else 1e-12
    for got in (out, c):
        assert float(min_image(got.double().cpu() - want, nf).abs().max()) < tol * nf


def test_displacement_add_rejects_bad_sizes():
    dev = _dev()
    x = torch.zeros((3, 8 ** 3), device=dev)
    with pytest.raises(pm.PMError, match="multiple"):
        pm.displacement_add(torch.zeros((3, 27), device=dev), 3, x, 8)


# ------------------------------------------------------------------- P(k) --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,nb", [(32, 16), (64, 32), (64, 13), (192, 96)])
def test_pk_estimate(dt, n, nb):
    dev = _dev()
    delta = torch.from_numpy(si.random_real_mesh(n, 40 + nb))
    plan = pm.Plan(n, 1000.0, dt)
    k, p, c = pm.pk_estimate(plan, delta.to(dt).to(dev), nb)
    wk, wp, wc = estimators.power_spectrum(delta.to(dt).double(), 1000.0, nb)
    assert torch.equal(c.cpu(), wc)
    assert rel_l2(p, wp) < _tol(dt)
    assert rel_l2(k, wk) < 1e-12


# ------------------------------------------------------------------- B(k) --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,nb,batch", [(32, 16, 1), (64, 13, 1), (192, 96, 1), (32, 16, 2)])
def test_pk_cross_estimate(dt, n, nb, batch):
    dev = _dev()
    box = 800.0
    g = si.rng(40 + n)
    a = torch.from_numpy(g.standard_normal((batch, n, n, n)))
    b = 0.5 * a + torch.from_numpy(g.standard_normal((batch, n, n, n)))
    plan = pm.Plan(n, box, dt, batch=batch)
    ad, bd = a.to(dt).to(dev).squeeze(0).contiguous(), b.to(dt).to(dev).squeeze(0).contiguous()
    k, p, c = pm.pk_cross_estimate(plan, ad, bd, nb)
    torch.cuda.synchronize()
    k, p, c = (t.reshape(batch, nb).cpu() for t in (k, p, c))
    for i in range(batch):
        wk, wp, wc = estimators.cross_power_spectrum(a[i].to(dt).double(), b[i].to(dt).double(), box, nb)
        assert torch.equal(c[i], wc)
        assert rel_l2(k[i], wk) < 1e-12
        assert rel_l2(p[i], wp) < _tol(dt)
    # the auto case equals pk_estimate
    _, pa, _ = pm.pk_cross_estimate(plan, ad, ad, nb)
    _, pp, _ = pm.pk_estimate(plan, ad, nb)
    torch.cuda.synchronize()
    assert rel_l2(pa, pp) < 1e-12


def test_bias_fit_matches_oracle_and_rejects_short_input():
    _dev()
    g = si.rng(44)
    k = torch.linspace(0.003, 0.15, 50, dtype=torch.float64)
    cnt = torch.from_numpy(g.integers(1, 500, 50))
    ratio = 1.2 + 3.0 * (4e-4 / k) ** 2 + 5.0 * k * k + torch.from_numpy(g.standard_normal(50)) * 0.02
    for with_k2 in (True, False):
        got = pm.bias_fit(k.tolist(), ratio.tolist(), cnt.tolist(), 0.08, 4e-4, 2, with_k2)
        want = estimators.bias_fit(k, ratio, cnt, 0.08, 4e-4, 2, with_k2)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-12)
    with pytest.raises(pm.PMError, match="bins"):
        pm.bias_fit([0.01, 0.02, 0.03, 0.04], [1.0] * 4, [1] * 4, 0.08, 4e-4, 2, True)


def test_bias_of_the_poisson_gauge_counting_density():
    """Matter proxy of the scale-dependent bias fit: the Poisson-gauge counting density
    of the partner set, against the Newtonian set, is biased by b1 = 1 and b1_GR =
    3f + (9/2) Omega_m at linear order (eqs. physical_density and b1).  Noise made of
    plane waves with one |n| per P(k) bin makes each bin's ratio exactly
    1 + b1_GR calH^2/k^2 at that |n| (the bin's mean k averages over all its modes,
    so the fit is given the waves' k), and the fit must return these values."""
    dev = _dev()
    n, box, a_i = 64, 30000.0, 0.1
    nb = n // 2
    waves = [(1.0, (1, 0, 0), 0.2), (1.0, (0, 2, 0), 0.4), (1.0, (3, 0, 0), 1.0), (1.0, (0, 4, 0), 2.0),
             (1.0, (0, 0, 5), 0.3), (1.0, (3, 4, 0), 1.3), (1.0, (6, 0, 0), 0.8), (1.0, (2, 3, 6), 2.5),
             (1.0, (0, 8, 0), 0.1), (1.0, (0, 0, 10), 1.7), (1.0, (6, 8, 0), 0.6), (1.0, (12, 0, 0), 2.9),
             (1.0, (0, 0, 16), 1.4), (1.0, (20, 0, 0), 0.5)]
    noise = si.plane_wave_mesh(n, waves, device=dev, dtype=torch.float64)
    plan = pm.Plan(n, box, torch.float64)
    icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 1e-7), index=-2.0,
                      a_init=a_i, a_norm=a_i, cosmo=pm.FIDUCIAL)
    disp = plan.mesh(3)
    pos, mom, pg, mg = (plan.particles() for _ in range(4))
    pm.pm_ic_zeldovich(plan, noise, icp, disp, pos, mom)
    pm.pm_ic_gauge(plan, noise, icp, disp, pos, mom, pg, mg)
    dn, dg = pm.pm_deposit(plan, pos), pm.pm_deposit(plan, pg)
    k, pnn, cnt = pm.pk_estimate(plan, dn, nb)
    _, pgn, _ = pm.pk_cross_estimate(plan, dg, dn, nb)
    torch.cuda.synchronize()
    k, pnn, pgn, cnt = (t.cpu() for t in (k, pnn, pgn, cnt))
    sel = pnn > 1e-6 * float(pnn.max())
    # bin of each wave: (2b+1)^2 <= 4|n|^2 < (2b+3)^2 for n_bins = N/2
    k_wave = {}
    for _, m, _ in waves:
        n2 = sum(v * v for v in m)
        b = next(b for b in range(nb) if (2 * b + 1) ** 2 <= 4 * n2 < (2 * b + 3) ** 2)
        k_wave[b] = math.sqrt(n2) * 2.0 * math.pi / box
    bins = [b for b in range(nb) if bool(sel[b])]
    assert bins == sorted(k_wave)
    calh = a_i * pm.cosmo_hubble_e(a_i) / 2997.92458
    ratio = pgn[sel] / pnn[sel]
    kk = [k_wave[b] for b in bins]
    b1, bgr, c2 = pm.bias_fit(kk, ratio.tolist(), cnt[sel].tolist(), 0.08, calh, 2, True)
    c = ocm.Cosmo(n_s=0.965)
    want = 3.0 * ocm.growth_f(c, a_i) + 4.5 * ocm.omega_m_of_a(c, a_i)
    assert b1 == pytest.approx(1.0, abs=1e-4)
    assert bgr == pytest.approx(want, rel=1e-4)
    assert abs(c2) * max(kk) ** 2 < 1e-4
    assert float(ratio[0]) > 10.0     # a strong large-scale effect in this horizon-size box


@pytest.mark.parametrize("dt", DTYPES)
def test_bk_estimate(dt):
    dev = _dev()
    n = 32
    pos = torch.from_numpy(si.clustered_particles(n, 40000, 14, n_clumps=40, width=1.0))
    delta = cic.deposit_delta(pos, n)
    centres = [float(m) for m in range(1, 9)] + [4.0]
    tris = [(i, i, i) for i in range(8)] + [(i, i, 8) for i in range(2, 8)] + [(1, 2, 2), (2, 3, 4)]
    plan = pm.Plan(n, 500.0, dt)
    bk, ntri = pm.bk_estimate(plan, delta.to(dt).to(dev), centres, 1.0, tris)
    wb, wn = estimators.bispectrum(delta.to(dt).double(), 500.0, centres, 1.0, tris)
    assert rel_l2(ntri, wn) < _tol(dt)
    assert rel_l2(bk, wb) < _tol(dt)
    # cached indicator counts reproduce the same result
    bk2, ntri2 = pm.bk_estimate(plan, delta.to(dt).to(dev), centres, 1.0, tris, ntri_known=ntri)
    assert torch.allclose(bk2, bk, rtol=1e-12, atol=0)
    assert torch.equal(ntri2, ntri)
    # with room for only three shell fields, shells are evicted and recomputed between batches
    ws3 = torch.empty((3, n, n, n), dtype=dt, device=dev)
    bk3, ntri3 = pm.bk_estimate(plan, delta.to(dt).to(dev), centres, 1.0, tris, shell_ws=ws3)
    assert rel_l2(ntri3, wn) < _tol(dt)
    assert rel_l2(bk3, wb) < _tol(dt)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,slots,seed", [(32, 3, 1), (32, 4, 2), (64, 8, 3), (128, 5, 4), (192, 3, 5)])
def test_bk_estimate_triangle_lists(dt, n, slots, seed):
    """Random shell sets (thin and wide shells, from the centre to the corner of the
    cube) and random triangle lists with repeated shells, evaluated with few resident
    shell fields so that fields are evicted and recomputed, against the oracle."""
    dev = _dev()
    g = si.rng(700 + seed)
    n_shells = 10
    centres = [float(c) for c in g.uniform(0.5, 0.8 * n, size=n_shells)]
    centres[0], centres[1] = 1.0, 0.5 * math.sqrt(3.0) * n   # the first mode shell and the cube's corner
    width = float(g.choice([1.0, 2.0, 3.5]))
    tris = [tuple(int(v) for v in g.integers(0, n_shells, size=3)) for _ in range(13)]
    tris += [(2, 2, 2), (3, 3, 0), (0, 0, 0)]
    delta = torch.from_numpy(si.random_real_mesh(n, 710 + seed))
    box = 40.0 * n
    plan = pm.Plan(n, box, dt)
    ws = torch.empty((slots, n, n, n), dtype=dt, device=dev)
    bk, ntri = pm.bk_estimate(plan, delta.to(dt).to(dev), centres, width, tris, shell_ws=ws)
    torch.cuda.synchronize()
    wb, wn = estimators.bispectrum(delta.to(dt).double(), box, centres, width, tris)
    if dt == torch.float64:
        assert torch.equal(torch.round(ntri.cpu()), torch.round(wn))     # integer triangle counts
    assert rel_l2(ntri, wn) < _tol(dt)
    nz = wn > 0.5          # triangles that close (B of an empty triangle set is undefined)
    assert rel_l2(bk.cpu()[nz], wb[nz]) < _tol(dt)
    # counts of empty triangle sets: 0 up to the rounding of the indicator fields
    assert torch.all(ntri.cpu()[~nz].abs() < (0.5 if dt == torch.float64 else F32_TOL * float(wn.max())))


# ---------------------------------------------------------------- ICs ------

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("kind", ["powerlaw", "eh98"])
def test_initial_conditions(dt, kind):
    dev = _dev()
    n, box, a_i = 32, 1000.0, 0.02
    c = ocm.Cosmo(n_s=0.965)
    if kind == "powerlaw":
        power = oics.powerlaw_for_rms_displacement(n, box, 0.2)
        a_norm = a_i
        icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 0.2), index=-2.0,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    else:
        power = ocm.eh98_normalised(c, 0.965, 0.81)
        a_norm = 1.0
        icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    noise = torch.from_numpy(si.white_noise(n, 77))
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=power, a_norm=a_norm, cosmo=c)
    wpn, wmn, wpg, wmg = oics.zeldovich_pair(noise.to(dt).double(), p)
    plan = pm.Plan(n, box, dt)
    disp = plan.mesh(3)
    pos = torch.empty((3, n ** 3), dtype=dt, device=dev)
    mom = torch.empty_like(pos)
    pm.pm_ic_zeldovich(plan, noise.to(dt).to(dev), icp, disp, pos, mom)
    psi = disp.reshape(3, -1).double().cpu().clone()
    pg = torch.empty_like(pos)
    mg = torch.empty_like(pos)
    pm.pm_ic_gauge(plan, noise.to(dt).to(dev), icp, disp, pos, mom, pg, mg)
    torch.cuda.synchronize()
    xi = disp.reshape(3, -1).double().cpu()
    tol = _tol(dt)
    # fields: displacement and shift meshes, momenta
    assert rel_l2(psi, oics.za_displacement(noise.to(dt).double(), p)) < tol
    assert rel_l2(xi, oics.xi_linear(noise.to(dt).double(), p, a_i)[0]) < tol
    assert rel_l2(mom, wmn) < tol
    # positions: q + Psi rounded to the plan's precision (a displacement of 1e-3 cells is
    # only resolved to ulp(N)/1e-3 in float32), so they are compared in ulps of N
    ulp = float(torch.finfo(dt).eps) * n
    assert float(min_image(pos.double().cpu() - wpn, n).abs().max()) < 4 * ulp
    assert float(min_image(pg.double().cpu() - wpg, n).abs().max()) < 8 * ulp
    assert float((mg.double().cpu() - wmg).abs().max()) < 10 * tol * float(wmn.abs().max())


def _eh98(n, box, a_i):
    c = ocm.Cosmo(n_s=0.965)
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965,
                      a_init=a_i, a_norm=1.0, cosmo=pm.FIDUCIAL)
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=ocm.eh98_normalised(c, 0.965, 0.81), a_norm=1.0, cosmo=c)
    return icp, p


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("a", [0.02, 0.3, 1.0])
def test_xi_linear(dt, a):
    dev = _dev()
    n, box = 32, 1000.0
    icp, p = _eh98(n, box, 0.02)
    noise = torch.from_numpy(si.white_noise(n, 78)).to(dt)
    plan = pm.Plan(n, box, dt)
    xi = pm.pm_xi_linear(plan, noise.to(dev), icp, a)
    torch.cuda.synchronize()
    want, _ = oics.xi_linear(noise.double(), p, a)
    assert rel_l2(xi.reshape(3, -1), want) < _tol(dt)
    if a == 0.02:   # at a_init it is the shift that the Poisson-gauge ICs add
        disp = plan.mesh(3)
        pos, mom, pg, mg = (plan.particles() for _ in range(4))
        pm.pm_ic_gauge(plan, noise.to(dev), icp, disp, pos, mom, pg, mg)
        torch.cuda.synchronize()
        assert torch.equal(disp, xi)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("nf,nc", [(64, 16), (32, 32)])
def test_combined_linear_shift(dt, nf, nc):
    """A Newtonian Zel'dovich set at N_f plus the linear Poisson-gauge shift at a = 1
    of the noise truncated to N_c: the combination with linear theory."""
    dev = _dev()
    box = 1000.0
    icp, pf = _eh98(nf, box, 0.02)
    _, pc = _eh98(nc, box, 0.02)
    noise = torch.from_numpy(si.white_noise(nf, 79)).to(dt)
    fine = pm.Plan(nf, box, dt)
    coarse = pm.Plan(nc, box, dt)
    pos, mom = fine.particles(), fine.particles()
    pm.pm_ic_zeldovich(fine, noise.to(dev), icp, fine.mesh(3), pos, mom)
    xi = pm.pm_xi_linear(coarse, pm.pm_noise_truncate(fine, noise.to(dev), coarse), icp, 1.0)
    out = pm.displacement_add(xi, nc, pos, nf)
    torch.cuda.synchronize()
    nd = noise.double()
    want = ocomb.add_displacement(oics.xi_linear(oics.truncate_noise(nd, nc), pc, 1.0)[0], nc,
                                  oics.zeldovich(nd, pf)[0], nf)
    ulp = float(torch.finfo(dt).eps) * nf
    assert float(min_image(out.double().cpu() - want, nf).abs().max()) < 8 * ulp
    shift = min_image(want - oics.zeldovich(nd, pf)[0], nf)
    assert float(shift.abs().max()) > 100 * ulp   # the shift (1e-3 cells here) is resolved


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,kind", [(32, "eh98"), (64, "powerlaw"), (192, "eh98")])
def test_initial_conditions_2lpt(dt, n, kind):
    """Second-order Newtonian set, and the Poisson-gauge partner built on it."""
    dev = _dev()
    box, a_i = 1000.0, 0.02
    c = ocm.Cosmo(n_s=0.965)
    if kind == "powerlaw":
        power, a_norm = oics.powerlaw_for_rms_displacement(n, box, 0.4), a_i
        icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 0.4), index=-2.0,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    else:
        power, a_norm = ocm.eh98_normalised(c, 0.965, 0.81), 1.0
        icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=power, a_norm=a_norm, cosmo=c)
    noise = torch.from_numpy(si.white_noise(n, 91)).to(dt)
    plan = pm.Plan(n, box, dt)
    disp = plan.mesh(3)
    pos, mom, pg, mg = (plan.particles() for _ in range(4))
    pm.pm_ic_2lpt(plan, noise.to(dev), icp, disp, pos, mom)
    torch.cuda.synchronize()
    psi1 = disp.reshape(3, -1).double().cpu().clone()
    pm.pm_ic_gauge(plan, noise.to(dev), icp, disp, pos, mom, pg, mg)
    torch.cuda.synchronize()
    nd = noise.double()
    wpos, wmom = oics.lpt2(nd, p)
    w1, w2 = oics.lpt2_displacement(nd, p)
    tol = _tol(dt)
    assert rel_l2(psi1, w1) < tol
    ulp = float(torch.finfo(dt).eps) * n
    assert float(min_image(pos.double().cpu() - wpos, n).abs().max()) < 8 * ulp
    assert rel_l2(mom, wmom) < tol
    # the second-order part itself: from the positions where it is well above their
    # rounding (the power-law case: 0.03 cell; EH98 at a = 0.02 on 31 Mpc/h cells gives
    # 5e-5 cell), and from the FP64 momenta, mom = a^2 E (f Psi1 + f2 Psi2)
    if kind == "powerlaw":
        got2 = min_image(pos.double().cpu() - (oics.lagrangian_lattice(n) + w1), n)
        assert float(w2.abs().max()) > 100 * ulp
        assert float((got2 - w2).abs().max()) < 8 * ulp + tol * float(w2.abs().max())
    ae = a_i * a_i * ocm.hubble_e(c, a_i)
    if dt == torch.float64:
        _, f2 = oics.lpt2_coefficients(p)
        psi2 = (mom.cpu() - ae * ocm.growth_f(c, a_i) * psi1) / (ae * f2)
        assert rel_l2(psi2, w2) < 1e-6
    xi, dxi = oics.xi_linear(nd, p, a_i)
    assert float(min_image(pg.double().cpu() - cic.wrap(wpos + xi, n), n).abs().max()) < 8 * ulp
    assert rel_l2(mg, wmom + ae * dxi) < 10 * tol


def test_2lpt_rejects_shared_buffers_and_batches():
    dev = _dev()
    n = 16
    plan = pm.Plan(n, 100.0, torch.float32)
    icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=1.0, index=-2.0, a_init=0.02, a_norm=0.02, cosmo=pm.FIDUCIAL)
    noise = plan.mesh().normal_()
    disp, pos = plan.mesh(3), plan.particles()
    with pytest.raises(pm.PMError, match="distinct"):
        pm.pm_ic_2lpt(plan, noise, icp, disp, pos, pos)
    bplan = pm.Plan(n, 100.0, torch.float32, batch=2)
    with pytest.raises(pm.PMError, match="single-box"):
        pm.pm_ic_2lpt(bplan, bplan.mesh(), icp, bplan.mesh(3), bplan.particles(), bplan.particles())


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [32, 192])
def test_noise_fix(dt, n):
    dev = _dev()
    plan = pm.Plan(n, 1000.0, dt)
    noise = torch.from_numpy(si.white_noise(n, 93)).to(dt)
    want = oics.fixed_noise(noise.double())
    for mode, sign in ((0, 1.0), (1, -1.0)):
        got = pm.pm_noise_fix(plan, noise.to(dev), mode)
        torch.cuda.synchronize()
        assert rel_l2(got, sign * want) < _tol(dt)
    inplace = noise.to(dev)
    pm.pm_noise_fix(plan, inplace, 0, out=inplace)
    torch.cuda.synchronize()
    assert rel_l2(inplace, want) < _tol(dt)


def test_noise_fix_pairs_in_a_batch():
    dev = _dev()
    n = 32
    plan = pm.Plan(n, 1000.0, torch.float64, batch=4)
    a, b = (torch.from_numpy(si.white_noise(n, s)) for s in (94, 95))
    got = pm.pm_noise_fix(plan, torch.stack([a, a, b, b]).to(dev), 2)
    torch.cuda.synchronize()
    for i, want in enumerate((oics.fixed_noise(a), -oics.fixed_noise(a), oics.fixed_noise(b), -oics.fixed_noise(b))):
        assert rel_l2(got[i], want) < F64_TOL
    with pytest.raises(pm.PMError, match="even"):
        pm.pm_noise_fix(pm.Plan(n, 1000.0, torch.float64, batch=3), torch.zeros((3, n, n, n), device=dev,
                                                                                dtype=torch.float64), 2)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("nf,nc", [(64, 16), (32, 32), (128, 32)])
def test_noise_truncate(dt, nf, nc):
    dev = _dev()
    w = torch.from_numpy(si.white_noise(nf, 5 + nf))
    fine, coarse = pm.Plan(nf, 1000.0, dt), pm.Plan(nc, 1000.0, dt)
    got = pm.pm_noise_truncate(fine, w.to(dt).to(dev).contiguous(), coarse)
    torch.cuda.synchronize()
    assert rel_l2(got, oics.truncate_noise(w.to(dt).double(), nc)) < _tol(dt)


# ------------------------------------------------------- end-to-end FP64 ----

@pytest.mark.slow
def test_paired_run_32_fp64():
    """32^3 particles, L = 1000 Mpc/h, power law with rms displacement 0.2 cell at a = 0.02,
    10 log steps to a = 0.1, Newtonian and Poisson-gauge sets, P(k) in 16 bins."""
    dev = _dev()
    n, box, a_i, a_f, steps = 32, 1000.0, 0.02, 0.1, 10
    power = oics.powerlaw_for_rms_displacement(n, box, 0.2)
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=power, a_norm=a_i)
    noise = torch.from_numpy(si.white_noise(n, 1))
    wpn, wmn, wpg, wmg = oics.zeldovich_pair(noise, p)
    a_s = ocm.log_steps(a_i, a_f, steps)
    xn, vn = integrate.run_kdk(wpn, wmn, a_s, integrate.NewtonForce(n), n)
    xg, vg = integrate.run_kdk(wpg, wmg, a_s, integrate.GaugeForce(n, box / n), n)

    plan = pm.Plan(n, box, torch.float64)
    icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 0.2), index=-2.0,
                      a_init=a_i, a_norm=a_i, cosmo=pm.FIDUCIAL)
    disp = plan.mesh(3)
    pos = torch.empty((3, n ** 3), dtype=torch.float64, device=dev)
    mom = torch.empty_like(pos)
    pm.pm_ic_zeldovich(plan, noise.to(dev), icp, disp, pos, mom)
    pg, mg = torch.empty_like(pos), torch.empty_like(pos)
    pm.pm_ic_gauge(plan, noise.to(dev), icp, disp, pos, mom, pg, mg)
    rn = pm.sim.Run(plan, pos, mom)
    rn.leapfrog(pm.sim.log_steps(a_i, a_f, steps))
    rg = pm.sim.Run(plan, pg, mg, gauge=True)
    rg.leapfrog(pm.sim.log_steps(a_i, a_f, steps))
    torch.cuda.synchronize()
    for got, want in ((pos, xn), (pg, xg)):
        d = min_image(got.cpu() - want, n)
        assert float(d.abs().max()) < 1e-9
    assert rel_l2(mom, vn) < 1e-10
    assert rel_l2(mg, vg) < 1e-10
    for x in (pos, pg):
        _, pk, cnt = pm.pk_estimate(plan, pm.pm_deposit(plan, x), 16)
        _, wpk, wcnt = estimators.power_spectrum(cic.deposit_delta(x.cpu(), n), box, 16)
        assert torch.equal(cnt.cpu(), wcnt)
        assert rel_l2(pk, wpk) < 1e-10


def test_combined_pm_and_combined_linear_shift_agree_in_the_linear_regime():
    """Combination through a Poisson-gauge/Newtonian run pair against combination with
    the linear shift xi_lin(a = 1): a 32^3 pair in a horizon-size box (L = 30000 Mpc/h,
    rms Zel'dovich displacement 1e-5 cell at a = 0.1, 40 log steps).  In the linear
    regime the run pair's xi^GR follows xi_lin (the oracle's runs agree to 0.2 % in
    relative L2), and the P(k) of the two combinations agree on the largest scales,
    where the gauge raises the power some fortyfold over the Newtonian run."""
    dev = _dev()
    n, box, a_i = 32, 30000.0, 0.1
    plan = pm.Plan(n, box, torch.float64)
    icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 1e-5), index=-2.0,
                      a_init=a_i, a_norm=a_i, cosmo=pm.FIDUCIAL)
    noise = torch.from_numpy(si.white_noise(n, 31)).to(dev)
    pos, mom, pg, mg = (plan.particles() for _ in range(4))
    disp = plan.mesh(3)
    pm.pm_ic_zeldovich(plan, noise, icp, disp, pos, mom)
    pm.pm_ic_gauge(plan, noise, icp, disp, pos, mom, pg, mg)
    a_s = pm.sim.log_steps(a_i, 1.0, 40)
    pm.sim.Run(plan, pos, mom).leapfrog(a_s)
    pm.sim.Run(plan, pg, mg, gauge=True).leapfrog(a_s)
    xi = pm.pm_xi_linear(plan, noise, icp, 1.0).reshape(3, -1)
    comb_lin = pm.displacement_add(xi, n, pos, n)
    comb_pm = pm.displacement_combine(pg, pos, n, pos, n)
    torch.cuda.synchronize()
    xi_pm = min_image(pg.cpu() - pos.cpu(), n)
    assert rel_l2(xi_pm, xi) < 0.01
    pks = [pm.pk_estimate(plan, pm.pm_deposit(plan, x), 16)[1].cpu() for x in (comb_pm, comb_lin, pos)]
    assert float((pks[0][:2] / pks[1][:2] - 1.0).abs().max()) < 0.01
    assert float(pks[2][0]) < 0.05 * float(pks[0][0])


def test_combination_recovers_the_relativistic_run_at_several_redshifts():
    """The paper's power-spectrum comparison (Sec. 4.1) in miniature: a fine 128^3
    Newtonian run plus xi of a 64^3 relativistic/Newtonian pair sharing its phases
    (eq. combined) against a fine 128^3 Poisson-gauge run, L = 4000 Mpc/h, EH98 2LPT
    ICs at a = 0.02, 50 log steps, at a = 0.17, 0.36, 0.49 and 1.  The gauge raises the
    fundamental bin by 6-31 % over the Newtonian run; the combination reproduces the
    relativistic run to 0.4 % in every bin (measured 0.33 % at most)."""
    dev = _dev()
    box, nf, nc = 4000.0, 128, 64
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965, a_init=0.02,
                      a_norm=1.0, cosmo=pm.FIDUCIAL)
    fine, coarse = pm.Plan(nf, box, torch.float32), pm.Plan(nc, box, torch.float32)
    noise_f = torch.from_numpy(si.white_noise(nf, 71, dtype=np.float32)).to(dev)
    noise_c = pm.pm_noise_truncate(fine, noise_f, coarse)
    a_s = pm.sim.log_steps(0.02, 1.0, 50)
    snap = [26, 36, 40, 49]

    def run(plan, noise, gauge):
        disp = plan.mesh(3)
        pos, mom, pg, mg = (plan.particles() for _ in range(4))
        pm.pm_ic_2lpt(plan, noise, icp, disp, pos, mom)
        if gauge:
            pm.pm_ic_gauge(plan, noise, icp, disp, pos, mom, pg, mg)
            pos, mom = pg, mg
        out = {}
        pm.sim.Run(plan, pos, mom, gauge=gauge).leapfrog(
            a_s, close=False, on_cycle=lambda j: out.__setitem__(j, pos.clone()) if j in snap else None)
        return out
    fn, fg, cn, cg = run(fine, noise_f, False), run(fine, noise_f, True), run(coarse, noise_c, False), \
        run(coarse, noise_c, True)
    nb = nf // 4
    for j in snap:
        comb = pm.displacement_combine(cg[j], cn[j], nc, fn[j], nf)
        p_n, p_g, p_c = (pm.pk_estimate(fine, pm.pm_deposit(fine, x), nb)[1].cpu() for x in (fn[j], fg[j], comb))
        gauge_effect = float(p_g[0] / p_n[0] - 1.0)
        assert gauge_effect > 0.05, (a_s[j + 1], gauge_effect)
        assert float((p_c / p_g - 1.0).abs().max()) < 0.004, a_s[j + 1]
        assert abs(float(p_c[0] / p_g[0] - 1.0)) < 0.05 * gauge_effect


def _gradient_variant_runs(n, box, steps, nb):
    """P(k) of the Newtonian and Poisson-gauge runs with each gradient symbol, and of
    the spectral Newtonian run combined with each variant's xi (eq. combined)."""
    dev = _dev()
    plan = pm.Plan(n, box, torch.float32)
    noise = torch.from_numpy(si.white_noise(n, 11, dtype=np.float32)).to(dev)
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965, a_init=0.02,
                      a_norm=1.0, cosmo=pm.FIDUCIAL)
    disp = plan.mesh(3)
    a_s = pm.sim.log_steps(0.02, 1.0, steps)
    pk, runs = {}, {}
    for name, g in (("spectral", pm.PM_GRAD_SPECTRAL), ("fd2", pm.PM_GRAD_FD2), ("fd1", pm.PM_GRAD_FD1)):
        pos, mom, pg, mg = (plan.particles() for _ in range(4))
        pm.pm_ic_zeldovich(plan, noise, icp, disp, pos, mom)
        pm.pm_ic_gauge(plan, noise, icp, disp, pos, mom, pg, mg)
        pm.sim.Run(plan, pos, mom, grad=g).leapfrog(a_s)
        pm.sim.Run(plan, pg, mg, gauge=True, grad=g).leapfrog(a_s)
        runs[name] = (pos, pg)
        for tag, x in (("N", pos), ("GR", pg)):
            k, p, _ = pm.pk_estimate(plan, pm.pm_deposit(plan, x), nb)
            pk[name, tag] = p.cpu()
    for name in ("fd2", "fd1"):
        xn, xg = runs[name]
        _, p, _ = pm.pk_estimate(plan, pm.pm_deposit(plan, pm.displacement_combine(xg, xn, n, runs["spectral"][0], n)), nb)
        pk[name, "comb"] = p.cpu()
    torch.cuda.synchronize()
    return k.cpu(), pk


def test_gradient_order_study():
    """Finite-difference gradients (first-order one-sided, second-order central) lose
    power against the spectral gradient, little on the largest scales and more towards
    the mesh scale (Sec. 4.1 discusses the loss with gevolution's gradients).  The same
    loss hits the relativistic and the Newtonian run, so it cancels in xi: the spectral
    Newtonian run plus xi from either finite-difference pair reproduces the spectral
    relativistic run far better than that pair's relativistic run does."""
    k, pk = _gradient_variant_runs(128, 8000.0, 50, 64)
    ref_n, ref_gr = pk["spectral", "N"], pk["spectral", "GR"]
    for name in ("fd1", "fd2"):
        d_n = pk[name, "N"] / ref_n - 1.0
        d_gr = pk[name, "GR"] / ref_gr - 1.0
        d_comb = pk[name, "comb"] / ref_gr - 1.0
        assert float(d_n[:3].abs().max()) < 0.02          # largest scales barely affected
        assert float(d_n[16:48].max()) < -0.1               # towards the mesh scale: a clear deficit
        assert float(d_gr.abs().max()) > 0.2
        assert float(d_comb.abs().max()) < 0.01             # the loss cancels in xi
        assert float(d_comb.abs().max()) < 0.05 * float(d_gr.abs().max())
    # the gauge itself is a large-scale effect here (L = 8000 Mpc/h): tens of per cent in the first bin
    assert float(ref_gr[0] / ref_n[0]) > 1.3


# ------------------------------------------- density handed to the next cycle --

@pytest.mark.parametrize("dt,n,amp", [(torch.float32, 128, 0.8), (torch.float32, 64, 6.0), (torch.float64, 32, 0.8)])
def test_step_density_handoff_matches_plain_cycles(dt, n, amp):
    """Cycles that leave the drifted positions' density for the next cycle (fused into
    the gather for full FP32 lattices, a separate deposit otherwise) reproduce plain
    cycles."""
    dev = _dev()
    x0 = torch.from_numpy(si.lattice_jitter_particles(n, 81, amp)).to(dt)
    x0[x0 >= n] = 0
    p0 = (0.2 * torch.from_numpy(si.rng(82).standard_normal((3, n ** 3)))).to(dt)
    plan = pm.Plan(n, 300.0, dt)
    force = plan.mesh(3)
    res = []
    for fused in (False, True):
        x, p = x0.clone().to(dev).contiguous(), p0.clone().to(dev).contiguous()
        for j in range(3):
            fl = 0
            if fused:
                fl = (pm.PM_STEP_DENSITY_READY if j > 0 else 0) | (pm.PM_STEP_DEPOSIT_NEXT if j < 2 else 0)
            pm.pm_step(plan, x, p, pm.StepParams(kick=0.3, drift=0.4, solve=pm.newton_params(), flags=fl), force)
        torch.cuda.synchronize()
        pm.pm_check(plan)
        res.append((x.double().cpu(), p.double().cpu()))
    tol = 1e-6 if dt == torch.float32 else 1e-12
    assert float(min_image(res[1][0] - res[0][0], n).abs().max()) < tol * n
    assert rel_l2(res[1][1], res[0][1]) < tol


def test_step_density_ready_is_checked():
    dev = _dev()
    n = 64
    plan = pm.Plan(n, 300.0, torch.float32)
    x = torch.from_numpy(si.lattice_jitter_particles(n, 83, 0.5)).to(torch.float32).to(dev).contiguous()
    p = torch.zeros_like(x)
    force = plan.mesh(3)
    sp = pm.newton_params()
    ready, nxt = pm.PM_STEP_DENSITY_READY, pm.PM_STEP_DEPOSIT_NEXT
    with pytest.raises(pm.PMError) as e:            # nothing deposited yet
        pm.pm_step(plan, x, p, pm.StepParams(kick=0.1, drift=0.1, solve=sp, flags=ready), force)
    assert e.value.code == -5
    pm.pm_step(plan, x, p, pm.StepParams(kick=0.1, drift=0.1, solve=sp, flags=nxt), force)
    pm.pm_deposit(plan, x)                          # any other call discards the density
    with pytest.raises(pm.PMError):
        pm.pm_step(plan, x, p, pm.StepParams(kick=0.1, drift=0.1, solve=sp, flags=ready), force)
    pm.pm_step(plan, x, p, pm.StepParams(kick=0.1, drift=0.1, solve=sp, flags=nxt), force)
    with pytest.raises(pm.PMError):                 # other positions
        pm.pm_step(plan, x.clone(), p, pm.StepParams(kick=0.1, drift=0.1, solve=sp, flags=ready), force)
    torch.cuda.synchronize()


def test_step_fused_deposit_counts_non_finite_positions():
    dev = _dev()
    n = 64
    plan = pm.Plan(n, 300.0, torch.float32)
    x = torch.from_numpy(si.lattice_jitter_particles(n, 84, 0.5)).to(torch.float32).to(dev).contiguous()
    p = torch.zeros_like(x)
    p[0, 5] = float("nan")
    st = pm.StepParams(kick=0.1, drift=0.1, solve=pm.newton_params(), flags=pm.PM_STEP_DEPOSIT_NEXT)
    pm.pm_step(plan, x, p, st, plan.mesh(3))
    with pytest.raises(pm.PMError) as e:
        pm.pm_check(plan)
    assert e.value.code == -5


def test_poisson_gauge_run_with_density_handoff_matches_plain_cycles():
    """The Poisson-gauge set (potential carried between evaluations) run through the
    leapfrog host loop, which hands each cycle's density to the next, against plain
    cycles issued one by one."""
    dev = _dev()
    n, box = 32, 2000.0
    x0 = torch.from_numpy(si.lattice_jitter_particles(n, 85, 0.6))
    p0 = 0.1 * torch.from_numpy(si.rng(86).standard_normal((3, n ** 3)))
    a_s = ocm.log_steps(0.05, 0.1, 3)
    plan = pm.Plan(n, box, torch.float64)
    # host loop (density handoff between cycles)
    x, p = x0.clone().to(dev), p0.clone().to(dev)
    pm.sim.Run(plan, x, p, gauge=True).leapfrog(a_s)
    # plain cycles
    xr, pr = x0.clone().to(dev), p0.clone().to(dev)
    force, phi = plan.mesh(3), plan.spectrum()
    k2_prev, a_prev = 0.0, 0.0
    sched = [(a_s[j], *pm.kdk_factors(a_s[j], a_s[j + 1])) for j in range(len(a_s) - 1)]
    for a, k1, dr, k2 in sched:
        sp = pm.gauge_params(box, n, a, a_prev)
        pm.pm_step(plan, xr, pr, pm.StepParams(kick=k2_prev + k1, drift=dr, solve=sp), force, phi)
        k2_prev, a_prev = k2, a
    sp = pm.gauge_params(box, n, a_s[-1], a_prev)
    pm.pm_step(plan, xr, pr, pm.StepParams(kick=k2_prev, drift=0.0, solve=sp), force, phi)
    torch.cuda.synchronize()
    assert float(min_image(x.double().cpu() - xr.double().cpu(), n).abs().max()) < 1e-12 * n
    assert rel_l2(p, pr) < 1e-12


def test_entry_points_of_the_extensions_reject_bad_arguments():
    """Argument errors of the combined-1LPT, 2LPT, pairing, cross-spectrum, bias-fit
    and tuning entry points are reported synchronously, before any launch."""
    dev = _dev()
    n = 16
    plan = pm.Plan(n, 100.0, torch.float32)
    icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=1.0, index=-2.0, a_init=0.02, a_norm=0.02, cosmo=pm.FIDUCIAL)
    noise = plan.mesh().normal_()
    with pytest.raises(pm.PMError, match="scale factor"):
        pm.pm_xi_linear(plan, noise, icp, 0.0)
    bplan = pm.Plan(n, 100.0, torch.float32, batch=2)
    with pytest.raises(pm.PMError, match="single-box"):
        pm.pm_xi_linear(bplan, bplan.mesh(), icp, 1.0)
    with pytest.raises(pm.PMError, match="pair_mode"):
        pm.pm_noise_fix(plan, noise, 3)
    with pytest.raises(pm.PMError, match="n_bins|null"):   # zero bins: empty output buffers
        pm.pk_cross_estimate(plan, noise, noise, 0)
    with pytest.raises(pm.PMError, match="n_bins"):
        pm.pk_cross_estimate(plan, noise, noise, 4 * n + 1)
    with pytest.raises(pm.PMError, match="singular"):
        pm.bias_fit([0.01] * 6, [1.0] * 6, [5] * 6, 0.08, 1e-3, 0, True)   # one k: columns collinear
    with pytest.raises(pm.PMError, match="reps"):
        pm.pm_plan_autotune(plan, reps=0)
    with pytest.raises(pm.PMError):
        pm.pm_plan_tuning_candidates(plan, 4)
    x = torch.zeros((3, 8 ** 3), device=dev)
    with pytest.raises(pm.PMError, match="multiple"):
        pm.displacement_add(torch.zeros((3, 16 ** 3), device=dev), 16, x, 8)
