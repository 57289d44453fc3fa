"""Reference gradients of the differentiable PM forward model (FP64).

Test infrastructure only (see ``oracle/__init__``).

Not part of the paper: the forward map white noise -> Zel'dovich ICs -> leapfrog
PM steps -> CIC counting density -> P(k) -> loss is differentiated exactly by
reverse-mode automatic differentiation of the oracle's own plain operations
(``torch.autograd``).  At a CIC kink (a particle exactly on a cell edge) the
derivative of floor() is taken as zero, i.e. the right derivative of the
weights, consistently with the assignment.

Loss (reading): L = sum_b (P_b - T_b)^2 / T_b^2 over the bins with T_b > 0.
"""
from __future__ import annotations

import torch

from . import cic, estimators, ics, integrate, cosmology as cm


def pk_loss(pk: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    sel = target > 0
    return (((pk[sel] - target[sel]) / target[sel]) ** 2).sum()


def forward_pk(noise: torch.Tensor, p: ics.ICParams, a_steps, n_bins: int, grad: str = "spectral",
               lpt_order: int = 1):
    """Final-time P(k) of a Newtonian run started from ``noise`` (Zel'dovich ICs, or
    the second-order set for lpt_order = 2)."""
    pos, mom = ics.zeldovich(noise, p) if lpt_order == 1 else ics.lpt2(noise, p)
    force = integrate.NewtonForce(p.n, p.cosmo, grad)
    pos, mom = integrate.run_kdk(pos, mom, a_steps, force, p.n, p.cosmo)
    delta = cic.deposit_delta(pos, p.n)
    return estimators.power_spectrum(delta, p.box, n_bins)


def loss(noise: torch.Tensor, p: ics.ICParams, a_steps, n_bins: int, target: torch.Tensor,
         grad: str = "spectral", lpt_order: int = 1) -> torch.Tensor:
    _, pk, _ = forward_pk(noise, p, a_steps, n_bins, grad, lpt_order)
    return pk_loss(pk, target)


def loss_and_grad(noise: torch.Tensor, p: ics.ICParams, a_steps, n_bins: int, target: torch.Tensor,
                  grad: str = "spectral", lpt_order: int = 1):
    """(L, dL/dnoise) by reverse-mode differentiation of the FP64 forward model."""
    w = noise.detach().to(torch.float64).clone().requires_grad_(True)
    val = loss(w, p, a_steps, n_bins, target, grad, lpt_order)
    (g,) = torch.autograd.grad(val, w)
    return float(val.detach()), g


def loss_and_grad_by_cycles(noise: torch.Tensor, p: ics.ICParams, a_steps, n_bins: int, target: torch.Tensor,
                            grad: str = "spectral", lpt_order: int = 1):
    """(L, dL/dnoise) as ``loss_and_grad``, with memory bounded by one cycle.

    The leapfrog is written as its chain of force-kick-drift cycles (cycle j: force
    at x_j, kick K2(j-1) + K1(j), drift Dr(a_j, a_j+1); the closing half-kick does not
    move the particles, so P(k) does not see it).  The forward keeps every cycle's
    input (x, p); the reverse pass takes the cotangent of the final positions from
    the P(k) loss, pulls it back through the cycles from the last to the first with
    ``step_vjp`` (autograd of one cycle), and through the ICs.  Mathematically the
    same derivative as reverse mode over the whole run; for meshes whose whole-run
    graph does not fit in host memory."""
    w = noise.detach().to(torch.float64)
    ic = (lambda w_: ics.zeldovich(w_, p)) if lpt_order == 1 else (lambda w_: ics.lpt2(w_, p))
    pos, mom = ic(w)
    force = integrate.NewtonForce(p.n, p.cosmo, grad)
    cycles = []
    k2_prev = 0.0
    for a0, a1 in zip(a_steps[:-1], a_steps[1:]):
        k1, dr, k2 = integrate.kdk_factors(p.cosmo, a0, a1)
        cycles.append((k2_prev + k1, dr))
        k2_prev = k2
    states = []
    for kick, drift in cycles:
        states.append((pos, mom))
        pos, mom = integrate.force_then_kick_drift(pos, mom, kick, drift, force, 0.0, p.n)
    xf = pos.clone().requires_grad_(True)
    _, pk, _ = estimators.power_spectrum(cic.deposit_delta(xf, p.n), p.box, n_bins)
    val = pk_loss(pk, target)
    (lam_x,) = torch.autograd.grad(val, xf)
    lam_p = torch.zeros_like(lam_x)
    for (x, v), (kick, drift) in zip(reversed(states), reversed(cycles)):
        lam_x, lam_p = step_vjp(x, v, kick, drift, p.n, p.cosmo, lam_x, lam_p, grad)
    (g,) = vjp(ic, (w,), (lam_x, lam_p))
    return float(val.detach()), g


def vjp(fn, primals, cotangent):
    """Vector-Jacobian product of ``fn`` at ``primals`` (a tuple of tensors)."""
    xs = tuple(t.detach().clone().requires_grad_(True) for t in primals)
    out = fn(*xs)
    gs = torch.autograd.grad(out, xs, grad_outputs=cotangent, allow_unused=True)
    return tuple(torch.zeros_like(x) if g is None else g for x, g in zip(xs, gs))


def step_vjp(pos, mom, kick: float, drift: float, n: int, cosmo: cm.Cosmo, lam_pos, lam_mom, grad="spectral"):
    """Cotangents (lam_pos_in, lam_mom_in) of one force-kick-drift cycle."""
    force = integrate.NewtonForce(n, cosmo, grad)

    def cycle(x, p):
        x1, p1 = integrate.force_then_kick_drift(x, p, kick, drift, force, 0.0, n)
        return torch.cat([x1.reshape(-1), p1.reshape(-1)])

    ct = torch.cat([lam_pos.reshape(-1), lam_mom.reshape(-1)])
    return vjp(cycle, (pos, mom), ct)


def lpt2_vjp(noise: torch.Tensor, p: ics.ICParams, lam_pos: torch.Tensor, lam_mom: torch.Tensor) -> torch.Tensor:
    """Cotangent of the white noise for cotangents (lam_pos, lam_mom) of the second-
    order Newtonian set ``ics.lpt2`` (the wrap has unit derivative)."""
    (g,) = vjp(lambda w: ics.lpt2(w, p), (noise.to(torch.float64),), (lam_pos, lam_mom))
    return g
