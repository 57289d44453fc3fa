"""Pins of the oracle's background cosmology against closed forms and paper values."""
import json
import math
import os

import pytest

from oracle import cosmology as cm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
EDS = cm.Cosmo(omega_c=0.95, omega_b=0.05)          # Omega_m = 1: Einstein-de Sitter


def test_fiducial_matches_paper_setup():
    g = GOLD["cosmology"]
    assert cm.FIDUCIAL.omega_c == g["omega_c"]
    assert cm.FIDUCIAL.omega_b == g["omega_b"]
    assert cm.FIDUCIAL.h == pytest.approx(g["H0"] / 100.0)
    assert cm.FIDUCIAL.omega_l == pytest.approx(1.0 - g["omega_c"] - g["omega_b"])


def test_box_of_paper_from_fundamental_mode():
    b = GOLD["box"]
    box = 2.0 * math.pi / b["k_f_h_per_mpc"]                 # Mpc/h
    gpc = box / cm.FIDUCIAL.h / 1000.0
    assert gpc == pytest.approx(b["box_gpc_approx"], abs=0.06)
    k_nyq = b["k_f_h_per_mpc"] * b["grid"] / 2
    assert k_nyq == pytest.approx(b["nyquist_h_per_mpc_approx"], abs=0.006)
    s = GOLD["squeezed"]
    assert s["k3_over_kf"] * b["k_f_h_per_mpc"] == pytest.approx(s["k3_h_per_mpc"])


@pytest.mark.parametrize("a", [0.02, 0.1, 0.5, 1.0])
def test_einstein_de_sitter_closed_forms(a):
    # Omega_m = 1: D = a, f = 1, E = a^-3/2.
    assert cm.hubble_e(EDS, a) == pytest.approx(a ** -1.5, rel=1e-14)
    assert cm.growth_d(EDS, a) == pytest.approx(a, rel=1e-10)
    assert cm.growth_f(EDS, a) == pytest.approx(1.0, rel=1e-9)
    assert cm.growth_f_dlna(EDS, a) == pytest.approx(0.0, abs=1e-8)


def test_eds_kick_drift_closed_forms():
    a0, a1 = 0.03, 0.7
    # K = int a^-2 a^{3/2} da = 2 (sqrt a1 - sqrt a0);  Dr = int a^-3/2 da = 2 (a0^-1/2 - a1^-1/2)
    assert cm.kick_factor(EDS, a0, a1) == pytest.approx(2 * (math.sqrt(a1) - math.sqrt(a0)), rel=1e-12)
    assert cm.drift_factor(EDS, a0, a1) == pytest.approx(2 * (a0 ** -0.5 - a1 ** -0.5), rel=1e-12)


@pytest.mark.parametrize("a", [0.05, 0.3, 0.8, 1.0])
def test_growth_rate_is_log_derivative(a):
    c = cm.FIDUCIAL
    h = 1e-4
    num = (math.log(cm.growth_d(c, a * math.exp(h))) - math.log(cm.growth_d(c, a * math.exp(-h)))) / (2 * h)
    assert cm.growth_f(c, a) == pytest.approx(num, rel=1e-7)
    fnum = (cm.growth_f(c, a * math.exp(h)) - cm.growth_f(c, a * math.exp(-h))) / (2 * h)
    assert cm.growth_f_dlna(c, a) == pytest.approx(fnum, rel=1e-5, abs=1e-8)


@pytest.mark.parametrize("a", [0.1, 0.6, 1.0])
def test_growth_solves_linear_growth_ode(a):
    # D'' + (2 + dlnE/dlna) D' - (3/2) Om(a) D = 0 in ln a, checked by finite differences.
    c = cm.FIDUCIAL
    h = 1e-3
    d = [cm.growth_d(c, a * math.exp(s * h)) for s in (-1, 0, 1)]
    d1 = (d[2] - d[0]) / (2 * h)
    d2 = (d[2] - 2 * d[1] + d[0]) / (h * h)
    om = cm.omega_m_of_a(c, a)
    res = d2 + (2 - 1.5 * om) * d1 - 1.5 * om * d[1]
    assert abs(res) < 1e-5 * d[1]


def test_early_time_growth_is_matter_dominated():
    c = cm.FIDUCIAL
    assert cm.growth_d(c, 1e-3) == pytest.approx(1e-3, rel=1e-4)
    assert cm.growth_f(c, 1e-3) == pytest.approx(1.0, abs=1e-6)


def test_relativistic_bias_consistent_with_table1():
    # eq. bgr: b1^GR = 3 (f + 3/2 Omega_m(z)) (1 - b1).  With the combined b1 of Table 1 and
    # this background, the theory lies within 1.5 sigma of the measured b1^GR at z <= 0.5.
    t = GOLD["table1_combined"]
    c = cm.FIDUCIAL
    for z, b1, bgr, err in zip(t["z"], t["b1"], t["b1gr"], t["b1gr_err"]):
        if z > 0.5:
            continue
        a = 1.0 / (1.0 + z)
        th = 3.0 * (cm.growth_f(c, a) + 1.5 * cm.omega_m_of_a(c, a)) * (1.0 - b1)
        assert abs(th - bgr) < 1.5 * err, (z, th, bgr)


def test_eh98_limits():
    # Parity unpinned for the fitting constants themselves; only the limits are checked.
    c = cm.Cosmo(n_s=0.965)
    assert cm.eh98_nowiggle_transfer(c, 1e-6) == pytest.approx(1.0, abs=1e-4)
    ks = [10 ** (x / 10) for x in range(-40, 10)]
    ts = [cm.eh98_nowiggle_transfer(c, k) for k in ks]
    assert all(t1 < t0 for t0, t1 in zip(ts, ts[1:]))
    # deep in the small-scale regime T ~ ln(q)/q^2: log slope tends to -2 from above
    s = math.log(ts[-1] / ts[-2]) / math.log(ks[-1] / ks[-2])
    assert -2.0 < s < -1.5


def test_sigma8_normalisation_integral():
    c = cm.Cosmo(n_s=0.965)
    ps = cm.eh98_normalised(c, 0.965, 0.81)
    s2 = cm.sigma_r_sq_unnormalised(c, 8.0, 0.965) * ps.amp
    assert math.sqrt(s2) == pytest.approx(0.81, rel=1e-10)
