"""Pins of the oracle's reference gradient (central finite differences)."""
import pytest
import torch

import synth_inputs as si
from oracle import adjoint, cic, cosmology as cm, ics


def _setup(n=8, box=200.0):
    p = ics.ICParams(n=n, box=box, a_init=0.05, power=ics.powerlaw_for_rms_displacement(n, box, 0.3), a_norm=0.05)
    a_steps = cm.log_steps(0.05, 0.3, 3)
    noise = torch.from_numpy(si.white_noise(n, 5))
    _, target, _ = adjoint.forward_pk(torch.from_numpy(si.white_noise(n, 6)), p, a_steps, 4)
    return p, a_steps, noise, target


def test_gradient_matches_central_differences():
    p, a_steps, noise, target = _setup()
    val, g = adjoint.loss_and_grad(noise, p, a_steps, 4, target)
    assert val > 0
    idx = si.rng(7).choice(noise.numel(), size=8, replace=False)
    h = 1e-5
    checked = 0
    for j in idx:
        e = torch.zeros_like(noise).reshape(-1)
        e[j] = h
        e = e.reshape(noise.shape)
        lp = float(adjoint.loss(noise + e, p, a_steps, 4, target))
        lm = float(adjoint.loss(noise - e, p, a_steps, 4, target))
        fd = (lp - lm) / (2 * h)
        ad = float(g.reshape(-1)[j])
        assert abs(fd - ad) <= 1e-5 * max(abs(ad), 1e-3 * float(g.abs().max())), (j, fd, ad)
        checked += 1
    assert checked == 8


@pytest.mark.parametrize("lpt_order", [1, 2])
def test_gradient_by_cycles_equals_whole_run_reverse_mode(lpt_order):
    """The memory-bounded reverse pass (cycle by cycle) gives the whole-run gradient."""
    n, box = 16, 300.0
    p = ics.ICParams(n=n, box=box, a_init=0.05, power=ics.powerlaw_for_rms_displacement(n, box, 0.5), a_norm=0.05)
    a_steps = cm.log_steps(0.05, 0.5, 5)
    noise = torch.from_numpy(si.white_noise(n, 15))
    _, target, _ = adjoint.forward_pk(torch.from_numpy(si.white_noise(n, 16)), p, a_steps, 8, lpt_order=lpt_order)
    val, g = adjoint.loss_and_grad(noise, p, a_steps, 8, target, lpt_order=lpt_order)
    val2, g2 = adjoint.loss_and_grad_by_cycles(noise, p, a_steps, 8, target, lpt_order=lpt_order)
    assert val2 == pytest.approx(val, rel=1e-12)
    assert float((g2 - g).norm() / g.norm()) < 1e-11
    assert float(g.norm()) > 0


def test_deposit_gather_dot_product():
    n = 8
    pos = torch.from_numpy(si.uniform_particles(n, 100, seed=3))
    mass = torch.from_numpy(si.rng(4).standard_normal(100))
    mesh = torch.from_numpy(si.random_real_mesh(n, 8))
    # <deposit(m), A> = <m, gather(A)>: the mesh cotangent of a deposit is a gather.
    (gm,) = adjoint.vjp(lambda m: cic.deposit_rho(pos, n, m), (mass,), mesh)
    assert torch.allclose(gm, cic.gather(mesh, pos), atol=1e-13)


def test_lpt2_vjp_equals_central_differences():
    # The 2LPT set is quadratic in the noise, so a central difference along v is exact
    # up to rounding: <lam, (F(w + e v) - F(w - e v)) / 2e> = <VJP(lam), v>.
    import math
    from oracle import adjoint as oadj, cosmology as cm, ics
    n, box = 16, 500.0
    c = cm.Cosmo(n_s=0.965)
    p = ics.ICParams(n=n, box=box, a_init=0.05, power=ics.powerlaw_for_rms_displacement(n, box, 0.8), a_norm=0.05,
                     cosmo=c)
    g = si.rng(9)
    w = torch.from_numpy(g.standard_normal((n, n, n)))
    v = torch.from_numpy(g.standard_normal((n, n, n)))
    lp = torch.from_numpy(g.standard_normal((3, n ** 3)))
    lm = torch.from_numpy(g.standard_normal((3, n ** 3)))
    got = float((oadj.lpt2_vjp(w, p, lp, lm) * v).sum())
    e = 1e-3
    (pp, mp), (pm_, mm) = ics.lpt2(w + e * v, p), ics.lpt2(w - e * v, p)
    dpos = torch.remainder(pp - pm_ + n / 2, n) - n / 2
    want = float(((lp * dpos).sum() + (lm * (mp - mm)).sum()) / (2 * e))
    assert got == pytest.approx(want, rel=1e-8)
    # the second-order part matters: the Zel'dovich VJP alone differs
    (pz, mz), (pz2, mz2) = ics.zeldovich(w + e * v, p), ics.zeldovich(w - e * v, p)
    wz = float(((lp * (torch.remainder(pz - pz2 + n / 2, n) - n / 2)).sum() + (lm * (mz - mz2)).sum()) / (2 * e))
    assert abs(wz - want) > 1e-4 * abs(want)
    assert math.isfinite(got)
