"""Pins of the oracle's reference gradient (central finite differences)."""
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


def test_deposit_gather_dot_product():
    n = 8
    pos = torch.from_numpy(si.uniform_particles(n, 100, seed=3))
    mass = torch.from_numpy(si.rng(4).standard_normal(100))
    mesh = torch.from_numpy(si.random_real_mesh(n, 8))
    # <deposit(m), A> = <m, gather(A)>: the mesh cotangent of a deposit is a gather.
    (gm,) = adjoint.vjp(lambda m: cic.deposit_rho(pos, n, m), (mass,), mesh)
    assert torch.allclose(gm, cic.gather(mesh, pos), atol=1e-13)
