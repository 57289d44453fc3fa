"""FFT launch-shape tuning: every allowed shape computes the same numbers (bit for
bit), the autotuner picks allowed shapes and caches them per process, the JSON cache
round-trips, and an autotuned ensemble reproduces the untuned one."""
import os

import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu

pm = pytest.importorskip("paper_2404_02783_amd")
from paper_2404_02783_amd import ensemble, tuning  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def _outputs(plan, delta, phi):
    """Newtonian and Poisson-gauge forces, P(k): every FFT pass kind runs."""
    f1 = pm.pm_solve(plan, delta, pm.newton_params()).clone()
    ph = phi.clone()
    f2 = pm.pm_solve(plan, delta, pm.gauge_params(plan.box, plan.n, 0.5, 0.45), ph).clone()
    _, p, _ = pm.pk_estimate(plan, delta, plan.n // 2)
    torch.cuda.synchronize()
    return f1, f2, ph, p.clone()


def _same(got, ref, what):
    # transforms are deterministic: bit-identical forces and potentials; P(k) sums its
    # bins with double atomics in no fixed order, so it agrees to rounding
    for a, b in zip(got[:3], ref[:3]):
        assert torch.equal(a, b), what
    assert float((got[3] - ref[3]).abs().max()) <= 1e-13 * float(ref[3].abs().max()), what


@pytest.mark.parametrize("n,dt,batch", [(64, torch.float32, 1), (192, torch.float64, 1), (32, torch.float32, 3),
                                        (128, torch.float32, 1)])
def test_every_launch_shape_gives_identical_results(n, dt, batch):
    dev = _dev()
    plan = pm.Plan(n, 500.0, dt, batch=batch)
    g = si.rng(60 + n)
    delta = torch.from_numpy(g.standard_normal((batch, n, n, n))).to(dt).to(dev).squeeze(0).contiguous()
    phi = torch.zeros((batch, n, n, n // 2 + 1), dtype=torch.complex64 if dt == torch.float32 else torch.complex128,
                      device=dev).squeeze(0).contiguous()
    default = pm.pm_plan_get_tuning(plan)
    ref = _outputs(plan, delta, phi)
    tried = 0
    for slot in range(4):
        cands = pm.pm_plan_tuning_candidates(plan, slot)
        assert default[slot] in cands and cands == sorted(cands) and len(cands) >= 2
        for c in cands:
            shapes = [0, 0, 0, 0]
            shapes[slot] = c
            pm.pm_plan_set_tuning(plan, shapes)
            assert pm.pm_plan_get_tuning(plan)[slot] == c
            _same(_outputs(plan, delta, phi), ref, (slot, c))
            tried += 1
    assert tried >= 8


def test_set_tuning_rejects_shapes_outside_the_limits():
    _dev()
    plan = pm.Plan(64, 500.0, torch.float32)
    before = pm.pm_plan_get_tuning(plan)
    for bad in ([3, 0, 0, 0], [0, 512, 0, 0], [0, 0, 1024, 0], [0, 0, 0, -2]):
        with pytest.raises(pm.PMError, match="launch shape"):
            pm.pm_plan_set_tuning(plan, bad)
        assert pm.pm_plan_get_tuning(plan) == before


def test_autotune_picks_allowed_shapes_and_caches_them():
    dev = _dev()
    n = 128
    plan = pm.Plan(n, 500.0, torch.float32)
    delta = torch.from_numpy(si.white_noise(n, 61)).float().to(dev)
    phi = torch.zeros((n, n, n // 2 + 1), dtype=torch.complex64, device=dev)
    ref = _outputs(plan, delta, phi)
    shapes, ms = pm.pm_plan_autotune(plan, reps=2, use_cache=False)
    for slot in range(4):
        assert shapes[slot] in pm.pm_plan_tuning_candidates(plan, slot)
        assert ms[slot] > 0
    _same(_outputs(plan, delta, phi), ref, "autotuned")
    other = pm.Plan(n, 900.0, torch.float32)   # same device, N, dtype and batch: cached
    shapes2, ms2 = pm.pm_plan_autotune(other, reps=2, use_cache=True)
    assert shapes2 == shapes and all(m < 0 for m in ms2)


def test_tuning_file_round_trip(tmp_path):
    dev = _dev()
    path = os.path.join(tmp_path, "fft_tuning.json")
    plan = pm.Plan(64, 500.0, torch.float64, batch=2)
    shapes, src = tuning.tune(plan, path, reps=1)
    assert src in ("measured", "process") and os.path.exists(path)
    again = pm.Plan(64, 100.0, torch.float64, batch=2)
    pm.pm_plan_set_tuning(again, [0, 0, 0, 0])
    shapes2, src2 = tuning.tune(again, path)
    assert src2 == "file" and shapes2 == shapes == pm.pm_plan_get_tuning(again)
    del dev


def test_autotuned_ensemble_matches_untuned():
    dev = _dev()
    groups = [ensemble.Group(32, 250.0, [3, 4, 5]), ensemble.Group(64, 500.0, [6, 7])]
    noise = lambda n, s: si.white_noise(n, s)
    runs = []
    for tuned in (False, True):
        ens = ensemble.Ensemble(groups, noise, 0.02, 0.05, 3, torch.float64, dev, autotune=tuned)
        ens.run()
        torch.cuda.synchronize()
        runs.append([p.cpu() for _, p, _ in ens.power_spectra()])
        if tuned:
            assert all(st.tuning is not None for st in ens.states)
    for a, b in zip(*runs):
        assert float((a - b).abs().max()) <= 1e-12 * float(b.abs().max())
