"""Parity of the hand-written adjoint entry points against the FP64 oracle's
reverse-mode derivatives (the oracle's gradient is itself pinned by central finite
differences in test_oracle_adjoint.py).

Bar: FP64 plans agree with the oracle's vector-Jacobian products to ~1e-9 relative L2
(summation order of atomics and FFTs only); FP32 plans to 1e-5 per operator on
identical inputs, and the end-to-end FP32 gradient to 1e-3 relative L2 against the
FP64 reference gradient (the FP32 forward trajectory itself differs at ~1e-6).
"""
import math

import pytest
import torch

import synth_inputs as si
from oracle import adjoint as oadj, cic, cosmology as ocm, estimators, ics as oics, integrate

pytestmark = pytest.mark.gpu

pm = pytest.importorskip("paper_2404_02783_amd")
from paper_2404_02783_amd import diff  # noqa: E402

DTYPES = [torch.float64, torch.float32]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def rel_l2(a, b):
    a = torch.as_tensor(a).double().cpu()
    b = torch.as_tensor(b).double().cpu()
    return float(torch.linalg.norm((a - b).reshape(-1)) / max(float(torch.linalg.norm(b.reshape(-1))), 1e-300))


def _randn(shape, seed):
    return torch.from_numpy(si.rng(seed).standard_normal(shape))


# ------------------------------------------------------------ one PM cycle --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,amp", [(16, 0.8), (32, 3.0)])
@pytest.mark.parametrize("cached_force", [True, False])
def test_step_adjoint_matches_oracle_vjp(dt, n, amp, cached_force):
    _step_adjoint_case(dt, n, amp, cached_force)


@pytest.mark.parametrize("amp", [0.4, 0.8, 6.0, 20.0])
def test_step_adjoint_lattice_tiles(amp):
    """A full 128^3 FP32 lattice takes the tiled adjoint gather with its fixed-point
    deposit of v: at amplitude 0.4 every box is staged whole, at 0.8 sparsely (only the
    cells the particles touch); amplitudes 6 and 20 overflow the LDS windows, so the
    fallback boxes and the direct global paths run too."""
    _step_adjoint_case(torch.float32, 128, amp, True)


def _step_adjoint_case(dt, n, amp, cached_force):
    dev = _dev()
    kick, drift = 0.37, 0.55
    pos0 = torch.from_numpy(si.lattice_jitter_particles(n, 11, amp))
    mom0 = 0.3 * _randn((3, n ** 3), 12)
    lx = _randn((3, n ** 3), 13)
    lp = _randn((3, n ** 3), 14)
    pos = pos0.to(dt)
    want_x, want_p = oadj.step_vjp(pos.double(), mom0.to(dt).double(), kick, drift, n, ocm.FIDUCIAL, lx, lp)
    plan = pm.Plan(n, 100.0, dt)
    st = pm.StepParams(kick=kick, drift=drift, solve=pm.newton_params())
    gpos = pos.to(dev).contiguous()
    force = None
    if cached_force:
        x1 = gpos.clone()
        m1 = mom0.to(dt).to(dev).contiguous()
        force = plan.mesh(3)
        pm.pm_step(plan, x1, m1, st, force)
    glx = lx.to(dt).to(dev).contiguous()
    glp = lp.to(dt).to(dev).contiguous()
    pm.pm_step_adjoint(plan, gpos, st, glx, glp, force=force)
    torch.cuda.synchronize()
    tol = 1e-9 if dt == torch.float64 else 1e-5
    assert rel_l2(glp, want_p) < tol
    assert rel_l2(glx, want_x) < tol


def test_step_adjoint_rejects_poisson_gauge():
    dev = _dev()
    n = 16
    plan = pm.Plan(n, 100.0, torch.float64)
    sp = pm.gauge_params(100.0, n, 0.1)
    st = pm.StepParams(kick=0.1, drift=0.1, solve=sp)
    x = torch.zeros((3, n ** 3), dtype=torch.float64, device=dev)
    with pytest.raises(pm.PMError):
        pm.pm_step_adjoint(plan, x, st, x.clone(), x.clone())


def test_step_adjoint_no_particles():
    dev = _dev()
    n = 16
    plan = pm.Plan(n, 100.0, torch.float32)
    st = pm.StepParams(kick=0.1, drift=0.1, solve=pm.newton_params())
    x = torch.zeros((3, 0), dtype=torch.float32, device=dev)
    pm.pm_step_adjoint(plan, x, st, x.clone(), x.clone())
    torch.cuda.synchronize()


# ------------------------------------------------------------- P(k) adjoint --

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n,nb", [(16, 8), (32, 16), (64, 32)])
def test_pk_adjoint_matches_oracle_vjp(dt, n, nb):
    dev = _dev()
    box = 300.0
    pos = torch.from_numpy(si.lattice_jitter_particles(n, 21, 1.5)).to(dt)
    dpk = _randn(nb, 22)

    def fwd(x):
        return estimators.power_spectrum(cic.deposit_delta(x, n), box, nb)[1]

    (want,) = oadj.vjp(fwd, (pos.double(),), dpk)
    plan = pm.Plan(n, box, dt)
    got = pm.pk_adjoint(plan, pos.to(dev).contiguous(), nb, dpk.to(dev))
    torch.cuda.synchronize()
    tol = 1e-9 if dt == torch.float64 else 1e-5
    assert rel_l2(got, want) < tol


# ------------------------------------------------------------- IC adjoint ----

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("kind", ["powerlaw", "eh98"])
def test_ic_adjoint_matches_oracle_vjp(dt, kind):
    dev = _dev()
    n, box, a_i = 32, 1000.0, 0.02
    c = ocm.Cosmo(n_s=0.965)
    if kind == "powerlaw":
        power, a_norm = oics.powerlaw_for_rms_displacement(n, box, 0.2), a_i
        icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 0.2), index=-2.0,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    else:
        power, a_norm = ocm.eh98_normalised(c, 0.965, 0.81), 1.0
        icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=power, a_norm=a_norm, cosmo=c)
    noise = torch.from_numpy(si.white_noise(n, 31))
    lx = _randn((3, n ** 3), 32)
    lp = _randn((3, n ** 3), 33)

    def fwd(w):
        x, m = oics.zeldovich(w, p)
        return torch.cat([x.reshape(-1), m.reshape(-1)])

    (want,) = oadj.vjp(fwd, (noise,), torch.cat([lx.reshape(-1), lp.reshape(-1)]))
    plan = pm.Plan(n, box, dt)
    got = pm.pm_ic_zeldovich_adjoint(plan, icp, lx.to(dt).to(dev).contiguous(), lp.to(dt).to(dev).contiguous())
    torch.cuda.synchronize()
    tol = 1e-9 if dt == torch.float64 else 1e-5
    assert rel_l2(got, want) < tol


# -------------------------------------------------------- whole gradient -----

def _model(n, box, a_i, a_f, steps, seed):
    power = oics.powerlaw_for_rms_displacement(n, box, 0.3)
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=power, a_norm=a_i)
    icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 0.3), index=-2.0,
                      a_init=a_i, a_norm=a_i, cosmo=pm.FIDUCIAL)
    a_steps = ocm.log_steps(a_i, a_f, steps)
    noise = torch.from_numpy(si.white_noise(n, seed))
    return p, icp, a_steps, noise


@pytest.mark.parametrize("dt", DTYPES)
def test_loss_gradient_matches_oracle(dt):
    """Gradient of L = sum_b ((P_b - T_b)/T_b)^2 with respect to the noise through ICs,
    6 leapfrog cycles and P(k), with checkpoints every 4 cycles."""
    dev = _dev()
    n, box, nb = 32, 500.0, 16
    p, icp, a_steps, noise = _model(n, box, 0.05, 0.5, 6, 41)
    _, target, _ = oadj.forward_pk(torch.from_numpy(si.white_noise(n, 42)), p, a_steps, nb)
    val, want = oadj.loss_and_grad(noise.to(dt).double(), p, a_steps, nb, target)

    plan = pm.Plan(n, box, dt)
    w = noise.to(dt).to(dev).requires_grad_(True)
    pk = diff.power_spectrum_model(w, plan, icp, diff.Schedule(a_steps), nb, 4)
    t = target.to(dev)
    loss = (((pk - t) / t) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    if dt == torch.float64:
        assert float(loss) == pytest.approx(val, rel=1e-9)
        assert rel_l2(w.grad, want) < 1e-8
    else:
        assert float(loss) == pytest.approx(val, rel=1e-3)
        assert rel_l2(w.grad, want) < 1e-3


@pytest.mark.parametrize("graphed", [False, True])
def test_loss_gradient_with_2lpt_start_matches_oracle(graphed):
    """The same loss and gradient from second-order ICs (FP64), through the autograd
    function and through the graph-captured model."""
    dev = _dev()
    n, box, nb = 32, 500.0, 16
    p, icp, a_steps, noise = _model(n, box, 0.05, 0.5, 6, 43)
    _, target, _ = oadj.forward_pk(torch.from_numpy(si.white_noise(n, 44)), p, a_steps, nb, lpt_order=2)
    val, want = oadj.loss_and_grad(noise, p, a_steps, nb, target, lpt_order=2)
    _, want_za = oadj.loss_and_grad(noise, p, a_steps, nb, target)
    plan = pm.Plan(n, box, torch.float64)
    sched = diff.Schedule(a_steps, lpt_order=2)
    t = target.to(dev)
    if graphed:
        model = diff.GraphedModel(plan, icp, sched, nb, 4).capture()
        pk = model.forward(noise.to(dev))
        dpk = 2.0 * (pk - t) / t ** 2
        got_val = float((((pk - t) / t) ** 2).sum())
        got = model.backward(dpk).clone()
    else:
        w = noise.to(dev).requires_grad_(True)
        pk = diff.power_spectrum_model(w, plan, icp, sched, nb, 4)
        loss = (((pk - t) / t) ** 2).sum()
        loss.backward()
        got_val, got = float(loss), w.grad
    torch.cuda.synchronize()
    assert got_val == pytest.approx(val, rel=1e-9)
    assert rel_l2(got, want) < 1e-8
    assert rel_l2(want_za, want) > 1e-6   # the second-order start changes the gradient


def test_checkpoint_interval_does_not_change_gradient():
    dev = _dev()
    n, box, nb = 16, 300.0, 8
    _, icp, a_steps, noise = _model(n, box, 0.05, 0.4, 5, 51)
    plan = pm.Plan(n, box, torch.float64)
    dpk = _randn(nb, 52).to(dev)
    grads = []
    for ck in (1, 2, 5):
        (_, pk, _), tape = diff.forward(plan, noise.to(dev), icp, diff.Schedule(a_steps), nb, ck)
        grads.append(diff.backward(tape, dpk).cpu())
    torch.cuda.synchronize()
    assert rel_l2(grads[1], grads[0]) < 1e-11
    assert rel_l2(grads[2], grads[0]) < 1e-11


def test_gradient_matches_central_differences_fp64():
    """GPU FP64 gradient against central differences of the GPU forward model on
    a few noise entries (h = 1e-5); entries whose perturbation moves a particle
    across a cell edge within +-h would be kinks, and the loss is smooth here
    (no entry changes a particle's cell)."""
    dev = _dev()
    n, box, nb = 16, 300.0, 8
    p, icp, a_steps, noise = _model(n, box, 0.05, 0.3, 3, 61)
    _, target, _ = oadj.forward_pk(torch.from_numpy(si.white_noise(n, 62)), p, a_steps, nb)
    plan = pm.Plan(n, box, torch.float64)
    sched = diff.Schedule(a_steps)
    t = target.to(dev)

    def loss_of(wv):
        (_, pk, _), _ = diff.forward(plan, wv, icp, sched, nb, 2)
        return float((((pk - t) / t) ** 2).sum())

    w = noise.to(dev).requires_grad_(True)
    pk = diff.power_spectrum_model(w, plan, icp, sched, nb, 2)
    ((((pk - t) / t) ** 2).sum()).backward()
    g = w.grad.detach().reshape(-1).cpu()
    idx = si.rng(63).choice(n ** 3, size=12, replace=False)
    h = 1e-5
    gmax = float(g.abs().max())
    for j in idx:
        e = torch.zeros(n ** 3, dtype=torch.float64)
        e[j] = h
        e = e.reshape(noise.shape).to(dev)
        fd = (loss_of(noise.to(dev) + e) - loss_of(noise.to(dev) - e)) / (2 * h)
        assert abs(fd - float(g[j])) <= 1e-5 * max(abs(float(g[j])), 1e-3 * gmax), (int(j), fd, float(g[j]))


def test_graphed_model_matches_eager():
    """Forward and reverse passes captured as graphs: three replays with different
    noise fields (and eager work in between) each reproduce the eager model."""
    dev = _dev()
    n, box, nb = 64, 400.0, 16
    _, icp, a_steps, _ = _model(n, box, 0.05, 0.5, 6, 71)
    plan = pm.Plan(n, box, torch.float32)
    sched = diff.Schedule(a_steps)
    gm = diff.GraphedModel(plan, icp, sched, nb, 4).capture()
    dpk = _randn(nb, 72).to(dev)
    for r in range(3):
        noise = torch.from_numpy(si.white_noise(n, 73 + r)).to(torch.float32).to(dev)
        pk_g = gm.forward(noise).clone()
        g_g = gm.backward(dpk).clone()
        torch.cuda.synchronize()
        (_, pk_e, _), tape = diff.forward(plan, noise, icp, sched, nb, 4)
        g_e = diff.backward(tape, dpk)
        torch.cuda.synchronize()
        assert rel_l2(pk_g, pk_e) < 1e-6
        assert rel_l2(g_g, g_e) < 1e-5
        float(torch.randn(1 << 20, device=dev).sum())



@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
@pytest.mark.parametrize("n,kind", [(32, "powerlaw"), (64, "eh98")])
def test_2lpt_ic_adjoint_matches_oracle(dt, tol, n, kind):
    """Adjoint of the second-order ICs against the oracle's reverse-mode VJP."""
    dev = _dev()
    box, a_i = 500.0, 0.05
    c = ocm.Cosmo(n_s=0.965)
    if kind == "powerlaw":
        power, a_norm = oics.powerlaw_for_rms_displacement(n, box, 0.6), a_i
        icp = pm.ICParams(pk_kind=pm.PM_PK_POWERLAW, amp=pm.power_law_amplitude(n, box, 0.6), index=-2.0,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    else:
        power, a_norm = ocm.eh98_normalised(c, 0.965, 0.81), 1.0
        icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965,
                          a_init=a_i, a_norm=a_norm, cosmo=pm.FIDUCIAL)
    p = oics.ICParams(n=n, box=box, a_init=a_i, power=power, a_norm=a_norm, cosmo=c)
    g = si.rng(70 + n)
    w = torch.from_numpy(g.standard_normal((n, n, n))).to(dt)
    lp = torch.from_numpy(g.standard_normal((3, n ** 3))).to(dt)
    lm = torch.from_numpy(g.standard_normal((3, n ** 3))).to(dt)
    plan = pm.Plan(n, box, dt)
    got = pm.pm_ic_2lpt_adjoint(plan, w.to(dev), icp, lp.to(dev), lm.to(dev))
    torch.cuda.synchronize()
    want = oadj.lpt2_vjp(w.double(), p, lp.double(), lm.double())
    assert rel_l2(got.reshape(-1), want.reshape(-1)) < tol
    # the second-order part is a visible share of the answer
    za = pm.pm_ic_zeldovich_adjoint(plan, icp, lp.to(dev), lm.to(dev))
    torch.cuda.synchronize()
    assert rel_l2(za.reshape(-1), want.reshape(-1)) > 100 * tol


# ------------------------------------------ the differentiable configuration --

def _config5():
    """128^3 particles on a 128^3 mesh, L = 1000 Mpc/h, EH98 no-wiggle LCDM ICs
    (n_s = 0.965, sigma8 = 0.81), 20 log steps a = 0.05 -> 1, P(k) in 64 bins, target
    spectrum from seed 6, noise from seed 5."""
    n, box, nb = 128, 1000.0, 64
    c = ocm.Cosmo(n_s=0.965)
    p = oics.ICParams(n=n, box=box, a_init=0.05, power=ocm.eh98_normalised(c, 0.965, 0.81), a_norm=1.0, cosmo=c)
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965, a_init=0.05,
                      a_norm=1.0, cosmo=pm.FIDUCIAL)
    a_steps = ocm.log_steps(0.05, 1.0, 20)
    noise = torch.from_numpy(si.white_noise(n, 5)).float()
    _, target, _ = oadj.forward_pk(torch.from_numpy(si.white_noise(n, 6)), p, a_steps, nb)
    return n, box, nb, p, icp, a_steps, noise, target


@pytest.mark.timeout(900)
def test_differentiable_configuration_gradient_matches_oracle():
    """The differentiable configuration at its own size, checkpoints every 5 cycles:
    FP32 and FP64 gradients of L = sum_b ((P_b - T_b)/T_b)^2 with respect to the noise
    against the oracle's FP64 reverse-mode gradient (taken cycle by cycle)."""
    dev = _dev()
    n, box, nb, p, icp, a_steps, noise, target = _config5()
    val, want = oadj.loss_and_grad_by_cycles(noise.double(), p, a_steps, nb, target)
    t = target.to(dev)
    for dt, tol_val, tol in ((torch.float64, 1e-9, 1e-8), (torch.float32, 1e-3, 1e-3)):
        plan = pm.Plan(n, box, dt)
        w = noise.to(dt).to(dev).requires_grad_(True)
        pk = diff.power_spectrum_model(w, plan, icp, diff.Schedule(a_steps), nb, 5)
        loss = (((pk - t) / t) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        assert float(loss.detach()) == pytest.approx(val, rel=tol_val), dt
        assert rel_l2(w.grad, want) < tol, dt
        del plan, w, pk, loss


def test_differentiable_configuration_central_differences_fp64():
    """32 noise entries of the differentiable configuration: the FP64 gradient (reverse
    pass with checkpoints every 5 cycles) against central differences of the FP64
    forward model, h = 1e-4.  A perturbation moves every particle by ~1e-7 cells, so
    the few particles it pushes across a cell edge (a kink of the CIC weights) change
    the difference by far less than the bar."""
    dev = _dev()
    n, box, nb, p, icp, a_steps, noise, target = _config5()
    plan = pm.Plan(n, box, torch.float64)
    sched = diff.Schedule(a_steps)
    t = target.to(dev)
    w0 = noise.double().to(dev)

    def loss_of(wv):
        (_, pk, _), _ = diff.forward(plan, wv, icp, sched, nb, 5)
        return float((((pk - t) / t) ** 2).sum())

    w = w0.clone().requires_grad_(True)
    pk = diff.power_spectrum_model(w, plan, icp, sched, nb, 5)
    ((((pk - t) / t) ** 2).sum()).backward()
    g = w.grad.detach().reshape(-1).cpu()
    gmax = float(g.abs().max())
    idx = si.rng(65).choice(n ** 3, size=32, replace=False)
    h = 1e-4
    for j in idx:
        e = torch.zeros(n ** 3, dtype=torch.float64)
        e[j] = h
        e = e.reshape(w0.shape).to(dev)
        fd = (loss_of(w0 + e) - loss_of(w0 - e)) / (2 * h)
        assert abs(fd - float(g[j])) <= 1e-4 * max(abs(float(g[j])), 1e-2 * gmax), (int(j), fd, float(g[j]))
