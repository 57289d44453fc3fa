"""Background cosmology, linear growth and time-integration factors (FP64).

Test infrastructure only (see ``oracle/__init__``).

Units ("grid units"): comoving positions in cells of size dx = L/N (Mpc/h),
time variable the scale factor a, momenta p = a^2 (dx/dt) / H0 in cells.  With
these units the equations of motion are

    dx/da = p / (a^3 E(a)),      dp/da = F / (a^2 E(a)),     F = -grad phi,
    laplacian(phi) = (3/2) Omega_m delta                      (cells^-2),

so a kick over [a0, a1] multiplies the force by K = int da / (a^2 E) and a drift
multiplies the momentum by Dr = int da / (a^3 E).  Conformal time in units of
1/H0 is the same integral as the kick factor, so a conformal-time interval in
cells is c_g * K with c_g = (c/H0)/dx.

The fiducial parameters are those of the paper's simulation setup (Sec. 3):
Omega_c = 0.263771, Omega_b = 0.0482754, H0 = 67.556, no radiation, and
Omega_Lambda = 1 - Omega_c - Omega_b.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from scipy import integrate as _int

C_KMS = 299792.458                 # speed of light, km/s
HUBBLE_DISTANCE = C_KMS / 100.0    # c / H0 in Mpc/h

_QUAD = dict(epsabs=0.0, epsrel=1e-13, limit=200)


@dataclass(frozen=True)
class Cosmo:
    """Flat LCDM without radiation (paper Sec. 3)."""
    omega_c: float = 0.263771
    omega_b: float = 0.0482754
    h: float = 0.67556
    n_s: float = 0.9619
    t_cmb: float = 2.7255

    @property
    def omega_m(self) -> float:
        return self.omega_c + self.omega_b

    @property
    def omega_l(self) -> float:
        return 1.0 - self.omega_m


FIDUCIAL = Cosmo()


def hubble_e(c: Cosmo, a: float) -> float:
    """E(a) = H(a)/H0 = sqrt(Omega_m a^-3 + Omega_Lambda)."""
    return math.sqrt(c.omega_m / a ** 3 + c.omega_l)


def omega_m_of_a(c: Cosmo, a: float) -> float:
    """Matter fraction Omega_m(a) = Omega_m a^-3 / E(a)^2."""
    return c.omega_m / a ** 3 / hubble_e(c, a) ** 2


def _growth_integral(c: Cosmo, a: float) -> float:
    """I(a) = int_0^a da' / (a' E(a'))^3 (finite: the integrand ~ a'^{3/2} near 0)."""
    val, _ = _int.quad(lambda x: 1.0 / (x * hubble_e(c, x)) ** 3, 0.0, a, **_QUAD)
    return val


def growth_d(c: Cosmo, a: float) -> float:
    """Linear growing mode D(a) = (5 Omega_m / 2) E(a) I(a) (Heath integral; exact for
    a pressureless matter + Lambda background).  D(a) -> a for a -> 0."""
    return 2.5 * c.omega_m * hubble_e(c, a) * _growth_integral(c, a)


def growth_f(c: Cosmo, a: float) -> float:
    """Growth rate f = dlnD/dlna.  Differentiating the Heath form gives
    f = dlnE/dlna + 1/(a^2 E^3 I) with dlnE/dlna = -(3/2) Omega_m(a)."""
    return -1.5 * omega_m_of_a(c, a) + 1.0 / (a * a * hubble_e(c, a) ** 3 * _growth_integral(c, a))


def growth_f_dlna(c: Cosmo, a: float) -> float:
    """df/dlna from the growth equation
    f' + f^2 + (2 + dlnE/dlna) f = (3/2) Omega_m(a)."""
    om = omega_m_of_a(c, a)
    f = growth_f(c, a)
    return 1.5 * om - f * f - (2.0 - 1.5 * om) * f


def kick_factor(c: Cosmo, a0: float, a1: float) -> float:
    """K(a0, a1) = int_{a0}^{a1} da / (a^2 E(a))."""
    val, _ = _int.quad(lambda x: 1.0 / (x * x * hubble_e(c, x)), a0, a1, **_QUAD)
    return val


def drift_factor(c: Cosmo, a0: float, a1: float) -> float:
    """Dr(a0, a1) = int_{a0}^{a1} da / (a^3 E(a))."""
    val, _ = _int.quad(lambda x: 1.0 / (x ** 3 * hubble_e(c, x)), a0, a1, **_QUAD)
    return val


def c_grid(dx: float) -> float:
    """Speed of light in cells per (1/H0): c_g = (c/H0) / dx."""
    return HUBBLE_DISTANCE / dx


def conformal_hubble_grid(c: Cosmo, a: float, dx: float) -> float:
    """Conformal Hubble rate in inverse cells: calH_g = a E(a) / c_g."""
    return a * hubble_e(c, a) / c_grid(dx)


def log_steps(a_start: float, a_end: float, n_steps: int) -> list[float]:
    """n_steps+1 scale factors equally spaced in ln a (step spacing reading)."""
    la, lb = math.log(a_start), math.log(a_end)
    return [math.exp(la + (lb - la) * j / n_steps) for j in range(n_steps + 1)]


# ---------------------------------------------------------------------------
# Linear power spectra (inputs to the initial conditions)
# ---------------------------------------------------------------------------

def eh98_nowiggle_transfer(c: Cosmo, k_h: float) -> float:
    """Eisenstein & Hu (1998) zero-baryon-oscillation transfer function
    (their sound-horizon fit, alpha_Gamma, effective shape Gamma and T0(q)).
    ``k_h`` in h/Mpc.  The constants are recalled from that paper."""
    h = c.h
    om_h2 = c.omega_m * h * h
    ob_h2 = c.omega_b * h * h
    fb = c.omega_b / c.omega_m
    theta = c.t_cmb / 2.7
    s = 44.5 * math.log(9.83 / om_h2) / math.sqrt(1.0 + 10.0 * ob_h2 ** 0.75)   # Mpc
    alpha = 1.0 - 0.328 * math.log(431.0 * om_h2) * fb + 0.38 * math.log(22.3 * om_h2) * fb * fb
    k_mpc = k_h * h
    gamma = c.omega_m * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k_mpc * s) ** 4))
    q = k_h * theta * theta / gamma
    l0 = math.log(2.0 * math.e + 1.8 * q)
    c0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return l0 / (l0 + c0 * q * q)


def tophat_window(x: float) -> float:
    """Fourier transform of a unit-volume spherical top hat, W(x) = 3 (sin x - x cos x)/x^3."""
    if x < 1e-4:
        return 1.0 - x * x / 10.0
    return 3.0 * (math.sin(x) - x * math.cos(x)) / x ** 3


def sigma_r_sq_unnormalised(c: Cosmo, r: float, n_s: float) -> float:
    """sigma^2(R) for P(k) = k^n_s T(k)^2 (unit amplitude):
    (1/2 pi^2) int P(k) W(kR)^2 k^2 dk, integrated in ln k."""
    def integrand(lnk):
        k = math.exp(lnk)
        t = eh98_nowiggle_transfer(c, k)
        w = tophat_window(k * r)
        return k ** (3.0 + n_s) * t * t * w * w / (2.0 * math.pi ** 2)
    val, _ = _int.quad(integrand, math.log(1e-6), math.log(1e3), epsabs=0.0, epsrel=1e-11, limit=2000)
    return val


@dataclass(frozen=True)
class PowerSpec:
    """Linear matter power spectrum at a = 1: P(k) = amp * k^index * T(k)^2 with
    T = 1 ("power law") or the EH98 no-wiggle transfer ("eh98")."""
    kind: str            # "powerlaw" | "eh98"
    amp: float
    index: float
    cosmo: Cosmo = FIDUCIAL

    def __call__(self, k_h: float) -> float:
        if k_h <= 0.0:
            return 0.0
        p = self.amp * k_h ** self.index
        if self.kind == "eh98":
            t = eh98_nowiggle_transfer(self.cosmo, k_h)
            p *= t * t
        return p


def eh98_normalised(c: Cosmo, n_s: float, sigma8: float) -> PowerSpec:
    """EH98 no-wiggle spectrum with amplitude fixed by sigma(8 Mpc/h) = sigma8 at a = 1."""
    s2 = sigma_r_sq_unnormalised(c, 8.0, n_s)
    return PowerSpec("eh98", sigma8 * sigma8 / s2, n_s, c)
