"""CPU-side checks of the C ABI: the library loads, exports every declared entry point,
and its host-side cosmology agrees with the oracle (no GPU calls here)."""
import math
import os
import re

import pytest

import paper_2404_02783_amd as pm
from oracle import cosmology as ocm, ics as oics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmhip.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", txt, flags=re.M)
    return sorted({n for n in names if n not in ("if", "while", "for", "sizeof")})


def test_library_loads_and_exports_every_declared_symbol():
    l = pm.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(l, n), n


def test_error_message_is_thread_local_string():
    import ctypes
    h = ctypes.c_void_p()
    rc = pm.lib().pm_plan_create(ctypes.byref(h), 100, 1.0, 0, None, 0)    # unsupported N: no device work
    assert rc == -2
    assert b"unsupported" in pm.lib().pm_last_error()
    assert pm.lib().pm_plan_workspace_bytes(100, 0) == 0
    assert pm.lib().pm_plan_workspace_bytes(64, 0) >= 3 * 64 * 64 * 33 * 8


C = ocm.FIDUCIAL


@pytest.mark.parametrize("a", [0.02, 0.1, 0.5, 1.0])
def test_host_background_matches_oracle(a):
    assert pm.cosmo_hubble_e(a) == pytest.approx(ocm.hubble_e(C, a), rel=1e-14)
    assert pm.cosmo_omega_m_a(a) == pytest.approx(ocm.omega_m_of_a(C, a), rel=1e-13)
    assert pm.cosmo_growth(a) == pytest.approx(ocm.growth_d(C, a), rel=1e-12)
    assert pm.cosmo_growth_rate(a) == pytest.approx(ocm.growth_f(C, a), rel=1e-11)


@pytest.mark.parametrize("a0,a1", [(0.02, 0.03), (0.05, 0.2), (0.5, 1.0)])
def test_host_kick_drift_match_oracle(a0, a1):
    k1, dr, k2 = pm.kdk_factors(a0, a1)
    o1, odr, o2 = (ocm.kick_factor(C, a0, math.sqrt(a0 * a1)), ocm.drift_factor(C, a0, a1),
                   ocm.kick_factor(C, math.sqrt(a0 * a1), a1))
    assert (k1, dr, k2) == pytest.approx((o1, odr, o2), rel=1e-12)


def test_library_is_built_from_this_tree():
    """The build record compiled into the library names the digest of the sources in
    the tree (a stale libpmhip.so fails here: rebuild with __graft_entry__.build())."""
    info = pm.build_info()
    assert info.startswith("pmhip gfx950 sources "), info
    assert pm.build_is_current(), info


def test_plan_rejects_misaligned_workspace():
    """A caller workspace must be 256-byte aligned; the check precedes any device work."""
    import ctypes
    h = ctypes.c_void_p()
    need = pm.lib().pm_plan_workspace_bytes(64, 0)
    rc = pm.lib().pm_plan_create(ctypes.byref(h), 64, 100.0, 0, ctypes.c_void_p(0x10000010), need)
    assert rc == -1 and not h.value
    assert b"aligned" in pm.lib().pm_last_error()


def test_host_log_steps_match_oracle():
    got = pm.log_steps(0.02, 1.0, 50)
    want = ocm.log_steps(0.02, 1.0, 50)
    assert len(got) == 51
    assert got == pytest.approx(want, rel=1e-15)
    assert got[0] == pytest.approx(0.02, rel=1e-15) and got[-1] == pytest.approx(1.0, rel=1e-15)


def test_host_leapfrog_chain_matches_oracle_steps():
    """The cycle chain equals the oracle's kick-drift-kick step by step: kick_j =
    K(a_{j-1/2}, a_j) + K(a_j, a_{j+1/2}), drift_j = Dr(a_j, a_{j+1}), closing kick
    K(a_{n-1/2}, a_n) with no drift; the kicks add up to K(a_0, a_n)."""
    a = ocm.log_steps(0.05, 1.0, 20)
    kick, drift = pm.leapfrog_factors(a)
    n = len(a) - 1
    assert len(kick) == len(drift) == n + 1
    for j in range(n + 1):
        k_in = ocm.kick_factor(C, math.sqrt(a[j - 1] * a[j]), a[j]) if j > 0 else 0.0
        k_out = ocm.kick_factor(C, a[j], math.sqrt(a[j] * a[j + 1])) if j < n else 0.0
        assert kick[j] == pytest.approx(k_in + k_out, rel=1e-12), j
        assert drift[j] == (pytest.approx(ocm.drift_factor(C, a[j], a[j + 1]), rel=1e-12) if j < n else 0.0), j
    assert sum(kick) == pytest.approx(ocm.kick_factor(C, a[0], a[-1]), rel=1e-12)
    assert sum(drift) == pytest.approx(ocm.drift_factor(C, a[0], a[-1]), rel=1e-12)


@pytest.mark.parametrize("bad", [[0.1], [0.2, 0.1], [0.0, 0.5], [0.1, 0.1]])
def test_host_leapfrog_factors_reject_bad_schedules(bad):
    with pytest.raises(pm.PMError):
        pm.leapfrog_factors(bad)


def test_host_gauge_params_match_oracle():
    box, n, a, ap = 4000.0, 256, 0.3, 0.28
    sp = pm.gauge_params(box, n, a, ap)
    dx = box / n
    cg = ocm.c_grid(dx)
    assert sp.kind == pm.PM_POISSON_GAUGE
    assert sp.c_g == pytest.approx(cg, rel=1e-14)
    assert sp.calh == pytest.approx(ocm.conformal_hubble_grid(C, a, dx), rel=1e-13)
    assert sp.om_a == pytest.approx(ocm.omega_m_of_a(C, a), rel=1e-13)
    assert sp.inv_dtau == pytest.approx(1.0 / (cg * ocm.kick_factor(C, ap, a)), rel=1e-12)
    assert pm.gauge_params(box, n, a, 0.0).inv_dtau == 0.0


def test_host_power_amplitudes_match_oracle():
    c65 = ocm.Cosmo(n_s=0.965)
    amp = pm.power_eh98_amplitude(0.965, 0.81)
    assert amp == pytest.approx(ocm.eh98_normalised(c65, 0.965, 0.81).amp, rel=1e-8)
    a_pl = pm.power_law_amplitude(16, 1000.0, 0.2, -2.0)
    assert a_pl == pytest.approx(oics.powerlaw_for_rms_displacement(16, 1000.0, 0.2).amp, rel=1e-12)


def test_every_entry_point_has_a_binding_of_the_same_name():
    # plan lifetime and the error string are covered by Plan and PMError
    by_class = {"pm_plan_create", "pm_plan_create_batch", "pm_plan_destroy", "pm_plan_workspace_bytes",
                "pm_plan_workspace_bytes_batch", "pm_last_error",
                # batch lifetime and groups are covered by Batch
                "pm_batch_create", "pm_batch_destroy", "pm_batch_num_groups", "pm_batch_group"}
    missing = []
    for n in _declared():
        if n in by_class:
            continue
        cands = (n, n.replace("pm_cosmo_", "cosmo_"), n.replace("pm_power_", "power_"), n.replace("pm_", "", 1))
        if not any(callable(getattr(pm, c, None)) for c in cands):
            missing.append(n)
    assert missing == []
    assert callable(pm.Plan) and callable(pm.Batch) and issubclass(pm.PMError, RuntimeError)
