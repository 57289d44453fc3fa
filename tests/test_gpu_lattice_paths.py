"""Oracle parity of the tiled FP32 particle kernels on the lattice paths that the
benchmark's ensembles and late clustered steps take (Sec. 2's PM cycle):

* N = 192, a mesh size that is not a power of two, so the kernels wrap, fold and take
  minimum images with divisions instead of masks (deposit, plain cycle, the cycle
  fused with the next cycle's deposit, the adjoint cycle);
* jitters of 0.4, 0.8 and 6 cells: at 0.4 every gather tile's box is the undisplaced
  one and is staged whole; at 0.8 the boxes are larger than the sparse threshold, so
  only the cells the particles touch are staged; at 6 every tile outgrows its window,
  so the windows shrink to fit_box's box and the particles outside take the direct
  global paths (global atomics for the deposit, direct force loads for the gather).
  A host count of the window volumes asserts which case each input is.

Each cycle is checked against the oracle's force-kick-drift cycle on the positions and
momenta the GPU cycle started from (promoted exactly to FP64), so the density handed
from one fused cycle to the next is checked against the oracle's own deposit.
"""
import pytest
import torch

import synth_inputs as si
from oracle import adjoint as oadj, cic, cosmology as ocm, integrate

pytestmark = pytest.mark.gpu

pm = pytest.importorskip("paper_2404_02783_amd")

F32_TOL = 1e-5

# Tile shapes and LDS window capacities (cells) of the tiled kernels: the deposit
# tile is 8 x 8 x 32 particles (8192 cells); the gather tile 4 x 8 x 32 (4096 cells);
# the fused gather-deposit merges two x-adjacent gather tiles into one deposit
# window (12288 cells).
DEPOSIT_TILE, DEPOSIT_CAP = (8, 8, 32), 8192
GATHER_TILE, GATHER_CAP = (4, 8, 32), 4096
FUSED_TILE, FUSED_CAP = (8, 8, 32), 12288
# gather boxes of more cells than this are staged sparsely (marked cells only)
GATHER_SPARSE = 2048


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def rel_l2(a, b):
    a = torch.as_tensor(a).double().cpu()
    b = torch.as_tensor(b).double().cpu()
    return float(torch.linalg.norm((a - b).reshape(-1)) / max(float(torch.linalg.norm(b.reshape(-1))), 1e-300))


def min_image(d, n):
    return (d + n / 2) % n - n / 2


def window_volumes(pos: torch.Tensor, n: int, tile) -> torch.Tensor:
    """Cells of each Lagrangian tile's CIC bounding box (base cells floor(x) as minimum
    images relative to the tile origin, widened by one cell)."""
    tx, ty, tz = tile
    base = torch.floor(pos.double()).long().reshape(3, n, n, n)
    vol = torch.ones((n // tx, n // ty, n // tz), dtype=torch.int64)
    for d, t in enumerate((tx, ty, tz)):
        org = torch.arange(n).reshape([n if k == d else 1 for k in range(3)])
        org = (org // t) * t
        r = ((base[d] - org + n // 2) % n) - n // 2
        r = r.reshape(n // tx, tx, n // ty, ty, n // tz, tz)
        lo = r.amin(dim=(1, 3, 5))
        hi = r.amax(dim=(1, 3, 5))
        vol = vol * (hi - lo + 2)
    return vol


def overflow_fraction(pos: torch.Tensor, n: int, tile, cap: int) -> float:
    """Fraction of Lagrangian tiles whose box exceeds `cap` cells: the tiles whose
    windows fit_box shrinks."""
    return float((window_volumes(pos, n, tile) > cap).double().mean())


def _lattice(n, seed, amp, dt=torch.float32):
    x = torch.from_numpy(si.lattice_jitter_particles(n, seed, amp)).to(dt)
    x[x >= n] = 0          # a coordinate just below N can round up to N in float32
    return x


def _case_windows(x, n, amp):
    """Asserts that the input takes the intended window case in every tiled kernel."""
    fractions = [overflow_fraction(x, n, t, c) for t, c in
                 ((DEPOSIT_TILE, DEPOSIT_CAP), (GATHER_TILE, GATHER_CAP), (FUSED_TILE, FUSED_CAP))]
    if amp < 1:
        assert max(fractions) == 0.0, fractions
        vol = window_volumes(x, n, GATHER_TILE)
        if amp < 0.5:
            assert int(vol.max()) <= GATHER_SPARSE, int(vol.max())
        else:
            assert int(vol.min()) > GATHER_SPARSE, int(vol.min())
    else:
        assert min(fractions) == 1.0, fractions
    return fractions


@pytest.mark.parametrize("amp", [0.8, 6.0])
def test_deposit_192(amp):
    dev = _dev()
    n = 192
    x = _lattice(n, 91, amp)
    _case_windows(x, n, amp)
    plan = pm.Plan(n, 1500.0, torch.float32)
    d = pm.pm_deposit(plan, x.to(dev).contiguous())
    torch.cuda.synchronize()
    pm.pm_check(plan)
    want = cic.deposit_delta(x.double(), n)
    assert rel_l2(d, want) < F32_TOL
    # mass conservation of the device sum (one particle per cell: sum(delta) = 0)
    assert abs(float(d.double().sum())) < 1e-3 * n ** 1.5


@pytest.mark.parametrize("amp", [0.4, 0.8, 6.0])
def test_plain_step_192(amp):
    dev = _dev()
    n = 192
    x = _lattice(n, 92, amp)
    v = (0.05 * torch.from_numpy(si.rng(93).standard_normal((3, n ** 3)))).float()
    _case_windows(x, n, amp)
    plan = pm.Plan(n, 1500.0, torch.float32)
    pos, mom = x.to(dev).contiguous(), v.to(dev).contiguous()
    force = plan.mesh(3)
    pm.pm_step(plan, pos, mom, pm.StepParams(kick=0.7, drift=1.3, solve=pm.newton_params()), force)
    torch.cuda.synchronize()
    pm.pm_check(plan)
    wx, wv = integrate.force_then_kick_drift(x.double(), v.double(), 0.7, 1.3, integrate.NewtonForce(n), 0.0, n)
    assert rel_l2(mom, wv) < F32_TOL
    d = min_image(pos.double().cpu() - wx, n)
    assert float(torch.linalg.norm(d)) / float(torch.linalg.norm(wx)) < F32_TOL


def _handed_over_cycles(n, amp, seed, box):
    """Three cycles on one plan: the first two leave the drifted positions' density
    for the next cycle (the fused gather-kick-drift-deposit kernel), the second and
    third start from that density.  Each cycle against the oracle's cycle from the
    GPU state it started from."""
    dev = _dev()
    x0 = _lattice(n, seed, amp)
    p0 = (0.2 * torch.from_numpy(si.rng(seed + 1).standard_normal((3, n ** 3)))).float()
    plan = pm.Plan(n, box, torch.float32)
    force = plan.mesh(3)
    x, p = x0.clone().to(dev).contiguous(), p0.clone().to(dev).contiguous()
    flags = [pm.PM_STEP_DEPOSIT_NEXT, pm.PM_STEP_DENSITY_READY | pm.PM_STEP_DEPOSIT_NEXT, pm.PM_STEP_DENSITY_READY]
    kicks, drifts = (0.3, 0.45, 0.2), (0.4, 0.5, 0.0)
    oracle_force = integrate.NewtonForce(n)
    _case_windows(x0, n, amp)
    for j, fl in enumerate(flags):
        xin, pin = x.double().cpu(), p.double().cpu()
        if j > 0 and amp >= 1:   # the previous cycle's fused deposit saw these positions
            assert overflow_fraction(xin, n, FUSED_TILE, FUSED_CAP) == 1.0
        pm.pm_step(plan, x, p, pm.StepParams(kick=kicks[j], drift=drifts[j], solve=pm.newton_params(), flags=fl),
                   force)
        torch.cuda.synchronize()
        pm.pm_check(plan)
        wx, wv = integrate.force_then_kick_drift(xin, pin, kicks[j], drifts[j], oracle_force, 0.0, n)
        assert rel_l2(p.double().cpu() - pin, wv - pin) < F32_TOL, j   # the kick itself
        assert rel_l2(p, wv) < F32_TOL, j
        d = min_image(x.double().cpu() - wx, n)
        assert float(torch.linalg.norm(d)) / float(torch.linalg.norm(wx)) < F32_TOL, j


@pytest.mark.parametrize("amp", [0.4, 0.8, 6.0])
def test_density_handed_over_cycles_192(amp):
    _handed_over_cycles(192, amp, 94, 1500.0)


@pytest.mark.parametrize("amp", [0.4, 0.8])
def test_density_handed_over_cycles_128(amp):
    """Power-of-two mesh (mask arithmetic) with whole and sparsely staged gather boxes."""
    _handed_over_cycles(128, amp, 95, 1000.0)


def test_density_handed_over_cycles_fit_box_128():
    """Clustered-like tiles on a power-of-two mesh: every gather and fused deposit
    window is shrunk by fit_box and particles outside it take the global paths."""
    _handed_over_cycles(128, 6.0, 96, 1000.0)


@pytest.mark.parametrize("n", [128, 192])
def test_cycle_from_unwrapped_positions(n):
    """Positions handed over outside [0, N) (about 5 % of the coordinates shifted by
    +N, 5 % by -N, some exactly N): the tiled kernels wrap them on load (a wave whose
    coordinates all lie inside skips the wrap, the others take it), so a deposit and a
    cycle fused with the next deposit match the oracle's, which reads the same values
    periodically.  The shifts are exact in FP32, so both sides see the same positions.
    The deposit counts the particles it wrapped back in and pm_check reports them."""
    dev = _dev()
    x = _lattice(n, 97, 0.4)
    r = torch.from_numpy(si.rng(98).random((3, n ** 3)))
    xu = torch.where(r < 0.05, x + n, torch.where(r > 0.95, x - n, x)).float()
    xu[0, 1000:1010] = float(n)
    assert bool(((xu < 0) | (xu >= n)).any())
    p0 = (0.2 * torch.from_numpy(si.rng(99).standard_normal((3, n ** 3)))).float()
    box = 1000.0 * n / 128
    plan = pm.Plan(n, box, torch.float32)
    outside = int(((xu < 0) | (xu >= n)).any(dim=0).sum())
    d = pm.pm_deposit(plan, xu.to(dev).contiguous())
    torch.cuda.synchronize()
    with pytest.raises(pm.PMError, match=f" {outside} positions outside"):
        pm.pm_check(plan)
    assert rel_l2(d, cic.deposit_delta(xu.double(), n)) < F32_TOL
    force = plan.mesh(3)
    pos, mom = xu.clone().to(dev).contiguous(), p0.clone().to(dev).contiguous()
    oracle_force = integrate.NewtonForce(n)
    xin, pin = xu.double(), p0.double()
    for j, fl in enumerate([pm.PM_STEP_DEPOSIT_NEXT, pm.PM_STEP_DENSITY_READY]):
        pm.pm_step(plan, pos, mom, pm.StepParams(kick=0.3, drift=0.4, solve=pm.newton_params(), flags=fl), force)
        torch.cuda.synchronize()
        if j == 0:   # this cycle's own deposit read the unwrapped positions
            with pytest.raises(pm.PMError, match=f" {outside} positions outside"):
                pm.pm_check(plan)
        else:        # the handed-over density came from wrapped positions
            pm.pm_check(plan)
        wx, wv = integrate.force_then_kick_drift(xin, pin, 0.3, 0.4, oracle_force, 0.0, n)
        assert rel_l2(mom, wv) < F32_TOL, j
        px = pos.double().cpu()
        assert bool(((px >= 0) & (px < n)).all()), j   # written back wrapped
        dd = min_image(px - wx, n)
        assert float(torch.linalg.norm(dd)) / float(torch.linalg.norm(wx)) < F32_TOL, j
        xin, pin = px, mom.double().cpu()


@pytest.mark.parametrize("amp", [0.4, 0.8, 6.0])
def test_step_adjoint_192(amp):
    """Tiled adjoint gather and fixed-point vector deposit at N = 192 against the
    oracle's vector-Jacobian product of the cycle."""
    dev = _dev()
    n = 192
    kick, drift = 0.37, 0.55
    x = _lattice(n, 97, amp)
    _case_windows(x, n, amp)
    mom0 = (0.3 * torch.from_numpy(si.rng(98).standard_normal((3, n ** 3)))).float()
    lx = torch.from_numpy(si.rng(99).standard_normal((3, n ** 3)))
    lp = torch.from_numpy(si.rng(100).standard_normal((3, n ** 3)))
    want_x, want_p = oadj.step_vjp(x.double(), mom0.double(), kick, drift, n, ocm.FIDUCIAL, lx, lp)
    plan = pm.Plan(n, 1500.0, torch.float32)
    st = pm.StepParams(kick=kick, drift=drift, solve=pm.newton_params())
    gpos = x.to(dev).contiguous()
    force = plan.mesh(3)
    pm.pm_step(plan, gpos.clone(), mom0.to(dev).contiguous(), st, force)
    glx, glp = lx.float().to(dev).contiguous(), lp.float().to(dev).contiguous()
    pm.pm_step_adjoint(plan, gpos, st, glx, glp, force=force)
    torch.cuda.synchronize()
    assert rel_l2(glp, want_p) < F32_TOL
    assert rel_l2(glx, want_x) < F32_TOL
