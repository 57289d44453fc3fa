// Host-side background cosmology (double precision) and the initial-condition entry
// points.  Quadratures use composite Gauss-Legendre rules whose nodes are found by
// Newton iteration on the Legendre polynomial (Golub-Welsch-free textbook method).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "pm_common.h"
#include "pm_plan.h"

namespace {

constexpr double kC_over_H0 = 2997.92458;  // Mpc/h

struct GaussLegendre {
  std::vector<double> x, w;  // on [-1, 1]
  explicit GaussLegendre(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(pm::kPi * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

const GaussLegendre& gl16() {
  static const GaussLegendre g(16);
  return g;
}

template <typename F>
double integrate(F f, double a, double b, int panels) {
  const GaussLegendre& g = gl16();
  const double h = (b - a) / panels;
  double sum = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double lo = a + p * h;
    double s = 0.0;
    for (size_t i = 0; i < g.x.size(); ++i) s += g.w[i] * f(lo + 0.5 * h * (g.x[i] + 1.0));
    sum += 0.5 * h * s;
  }
  return sum;
}

double omega_l(const pm_cosmology* c) { return 1.0 - c->omega_m; }

double hubble(const pm_cosmology* c, double a) { return std::sqrt(c->omega_m / (a * a * a) + omega_l(c)); }

// I(a) = int_0^a dx / (x E(x))^3, with x = u^2 (smooth integrand 2u / (u^2 E)^3).
double growth_integral(const pm_cosmology* c, double a) {
  auto f = [c](double u) {
    if (u <= 0.0) return 0.0;
    const double x = u * u;
    const double xe = x * hubble(c, x);
    return 2.0 * u / (xe * xe * xe);
  };
  return integrate(f, 0.0, std::sqrt(a), 64);
}

double eh98_t(const pm_cosmology* c, double k) {
  const double h = c->h, om = c->omega_m, ob = c->omega_b;
  const double omh2 = om * h * h, obh2 = ob * h * h, fb = ob / om, th = c->t_cmb / 2.7;
  const double s = 44.5 * std::log(9.83 / omh2) / std::sqrt(1.0 + 10.0 * std::pow(obh2, 0.75));
  const double al = 1.0 - 0.328 * std::log(431.0 * omh2) * fb + 0.38 * std::log(22.3 * omh2) * fb * fb;
  const double ks = 0.43 * k * h * s;
  const double gam = om * h * (al + (1.0 - al) / (1.0 + ks * ks * ks * ks));
  const double q = k * th * th / gam;
  const double l0 = std::log(2.0 * 2.718281828459045235360287 + 1.8 * q);
  const double c0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return l0 / (l0 + c0 * q * q);
}

double tophat(double x) {
  if (x < 1e-4) return 1.0 - x * x / 10.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

}  // namespace

extern "C" {

double pm_cosmo_hubble_e(const pm_cosmology* c, double a) { return hubble(c, a); }

double pm_cosmo_omega_m_a(const pm_cosmology* c, double a) {
  const double e = hubble(c, a);
  return c->omega_m / (a * a * a) / (e * e);
}

double pm_cosmo_growth(const pm_cosmology* c, double a) {
  return 2.5 * c->omega_m * hubble(c, a) * growth_integral(c, a);
}

double pm_cosmo_growth_rate(const pm_cosmology* c, double a) {
  const double e = hubble(c, a);
  return -1.5 * pm_cosmo_omega_m_a(c, a) + 1.0 / (a * a * e * e * e * growth_integral(c, a));
}

// K = int da/(a^2 E) and Dr = int da/(a^3 E), with a = u^2 to keep the integrands smooth.
double pm_cosmo_kick(const pm_cosmology* c, double a0, double a1) {
  auto f = [c](double u) {
    const double x = u * u;
    return 2.0 / (u * u * u * hubble(c, x));
  };
  return integrate(f, std::sqrt(a0), std::sqrt(a1), 16);
}

double pm_cosmo_drift(const pm_cosmology* c, double a0, double a1) {
  auto f = [c](double u) {
    const double x = u * u;
    return 2.0 / (u * u * u * u * u * hubble(c, x));
  };
  return integrate(f, std::sqrt(a0), std::sqrt(a1), 16);
}

void pm_kdk_factors(const pm_cosmology* c, double a0, double a1, double out[3]) {
  const double ah = std::sqrt(a0 * a1);
  out[0] = pm_cosmo_kick(c, a0, ah);
  out[1] = pm_cosmo_drift(c, a0, a1);
  out[2] = pm_cosmo_kick(c, ah, a1);
}

int pm_log_steps(double a_start, double a_end, int n_steps, double* a) {
  if (!a || n_steps < 1 || !(a_start > 0.0) || !(a_end > 0.0))
    return pm::set_error(PM_ERR_ARG, "pm_log_steps: need a, n_steps >= 1 and positive a_start, a_end");
  const double la = std::log(a_start), lb = std::log(a_end);
  for (int j = 0; j <= n_steps; ++j) a[j] = std::exp(la + (lb - la) * j / n_steps);
  return PM_OK;
}

int pm_leapfrog_factors(const pm_cosmology* c, const double* a, int n_steps, double* kick, double* drift) {
  if (!c || !a || !kick || !drift || n_steps < 1)
    return pm::set_error(PM_ERR_ARG, "pm_leapfrog_factors: null argument or n_steps < 1");
  for (int j = 0; j <= n_steps; ++j)
    if (!(a[j] > 0.0) || (j > 0 && !(a[j] > a[j - 1])))
      return pm::set_error(PM_ERR_ARG, "pm_leapfrog_factors: a must be positive and increasing");
  double k2_prev = 0.0;  // second half kick of the previous step
  for (int j = 0; j < n_steps; ++j) {
    double f[3];
    pm_kdk_factors(c, a[j], a[j + 1], f);
    kick[j] = k2_prev + f[0];
    drift[j] = f[1];
    k2_prev = f[2];
  }
  kick[n_steps] = k2_prev;
  drift[n_steps] = 0.0;
  return PM_OK;
}

void pm_gauge_params(const pm_cosmology* c, double box_mpch, int n_mesh, double a, double a_prev,
                     pm_solve_params* out) {
  const double dx = box_mpch / n_mesh;
  const double cg = kC_over_H0 / dx;
  out->kind = PM_POISSON_GAUGE;
  out->grad = PM_GRAD_SPECTRAL;
  out->omega_m = c->omega_m;
  out->a = a;
  out->om_a = pm_cosmo_omega_m_a(c, a);
  out->calh = a * hubble(c, a) / cg;
  out->c_g = cg;
  out->inv_dtau = a_prev > 0.0 ? 1.0 / (cg * pm_cosmo_kick(c, a_prev, a)) : 0.0;
}

double pm_power_eh98_amplitude(const pm_cosmology* c, double n_s, double sigma8) {
  const double r = 8.0;
  auto f = [c, n_s, r](double lnk) {
    const double k = std::exp(lnk);
    const double t = eh98_t(c, k);
    const double w = tophat(k * r);
    return std::pow(k, 3.0 + n_s) * t * t * w * w / (2.0 * pm::kPi * pm::kPi);
  };
  const double s2 = integrate(f, std::log(1e-6), std::log(1e3), 4000);
  return sigma8 * sigma8 / s2;
}

double pm_power_law_amplitude(int n, double box, double rms, double index) {
  const double dx = box / n;
  const double s = 2.0 * pm::kPi / n;
  double sum = 0.0;
  const int h = n / 2;
  for (int a = -h + 1; a < h; ++a)
    for (int b = -h + 1; b < h; ++b)
      for (int d = -h + 1; d < h; ++d) {
        if (a == 0 && b == 0 && d == 0) continue;
        const double kg2 = s * s * (double)(a * a + b * b + d * d);
        sum += std::pow(kg2, (index - 2.0) / 2.0);
      }
  sum *= std::pow(dx, -index);
  return rms * rms * dx * dx * dx * (double)n * n * n / sum;
}

// ----------------------------------------------------- initial conditions ----

static pm::IcSymbol ic_symbol_of(const pm_plan* p, const pm_ic_params* ic, int kpow, double coef) {
  using namespace pm;
  IcSymbol sy;
  sy.pk_kind = ic->pk_kind;
  sy.amp = ic->amp;
  sy.index = ic->index;
  sy.om = ic->cosmo.omega_m;
  sy.ob = ic->cosmo.omega_b;
  sy.h = ic->cosmo.h;
  sy.tcmb = ic->cosmo.t_cmb;
  sy.kf = 2.0 * kPi / p->box;
  const double dx = p->box / p->n;
  sy.inv_dx3 = 1.0 / (dx * dx * dx);
  sy.growth = pm_cosmo_growth(&ic->cosmo, ic->a_init) / pm_cosmo_growth(&ic->cosmo, ic->a_norm);
  sy.coef = coef / ((double)p->n * p->n * p->n);
  sy.kpow = kpow;
  sy.mode = 0;
  return sy;
}

static int ic_common(pm_plan* p, const void* noise, const pm_ic_params* ic, void* disp, int kpow, double coef,
                     hipStream_t s) {
  using namespace pm;
  int rc = fft3_r2c(p, noise, cbuf(p, 0), s);
  if (rc) return rc;
  rc = launch_ic_symbol(p, ic_symbol_of(p, ic, kpow, coef), false, s);
  if (rc) return rc;
  return fft3_c2r(p, 3 * p->nb, cbuf(p, 0), cstride(p), disp, s);
}

static int check_ic(pm_plan* p, const void* noise, const pm_ic_params* ic, const void* disp, const char* who) {
  using namespace pm;
  if (!p) return set_error(PM_ERR_ARG, "%s: null plan", who);
  if (!noise || !ic || !disp) return set_error(PM_ERR_ARG, "%s: null pointer", who);
  if (ic->pk_kind != PM_PK_POWERLAW && ic->pk_kind != PM_PK_EH98) return set_error(PM_ERR_ARG, "%s: bad pk_kind", who);
  if (!(ic->a_init > 0.0) || !(ic->a_norm > 0.0)) return set_error(PM_ERR_ARG, "%s: bad scale factors", who);
  return PM_OK;
}

int pm_ic_zeldovich(pm_plan* p, const void* noise, const pm_ic_params* ic, void* disp, void* pos, void* mom,
                    void* stream) {
  using namespace pm;
  int rc = check_ic(p, noise, ic, disp, "pm_ic_zeldovich");
  if (rc) return rc;
  p->dens_valid = false;
  if (!pos || !mom) return set_error(PM_ERR_ARG, "pm_ic_zeldovich: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = ic_common(p, noise, ic, disp, 1, 1.0, s);
  if (rc) return rc;
  const double a = ic->a_init;
  const double fac = a * a * pm_cosmo_hubble_e(&ic->cosmo, a) * pm_cosmo_growth_rate(&ic->cosmo, a);
  return launch_ic_lattice(p, disp, pos, mom, fac, s);
}

int pm_ic_2lpt(pm_plan* p, const void* noise, const pm_ic_params* ic, void* disp, void* pos, void* mom,
               void* stream) {
  using namespace pm;
  int rc = check_ic(p, noise, ic, disp, "pm_ic_2lpt");
  if (rc) return rc;
  p->dens_valid = false;
  if (!pos || !mom) return set_error(PM_ERR_ARG, "pm_ic_2lpt: null pointer");
  if (p->nb != 1) return set_error(PM_ERR_ARG, "pm_ic_2lpt: needs a single-box plan");
  if (noise == disp || noise == pos || noise == mom || disp == pos || disp == mom || pos == mom)
    return set_error(PM_ERR_ARG, "pm_ic_2lpt: noise, disp, pos and mom must be distinct buffers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t cs = cstride(p);
  IcSymbol sy = ic_symbol_of(p, ic, 1, 1.0);
  // S = sum_{i<j} (chi_ii chi_jj - chi_ij^2) on the lattice, into disp[0]; the three
  // Hessian components of each half pass through mom
  for (int pass = 0; pass < 2; ++pass) {
    rc = fft3_r2c(p, noise, cbuf(p, 0), s);
    if (rc) return rc;
    sy.mode = 1 + pass;
    rc = launch_ic_symbol(p, sy, false, s);
    if (rc) return rc;
    rc = fft3_c2r(p, 3, cbuf(p, 0), cs, mom, s);
    if (rc) return rc;
    rc = launch_lpt2_source(p, mom, disp, pass, s);
    if (rc) return rc;
  }
  // Psi2 = c2 IDFT(i k DFT(S) / k^2) into mom
  const pm_cosmology* c = &ic->cosmo;
  const double a = ic->a_init;
  const double om = pm_cosmo_omega_m_a(c, a);
  const double c2 = (3.0 / 7.0) * std::pow(om, -1.0 / 143.0);
  rc = fft3_r2c(p, disp, cbuf(p, 0), s);
  if (rc) return rc;
  IcSymbol s3 = sy;
  s3.mode = 3;
  s3.coef = c2 / ((double)p->n * p->n * p->n);
  rc = launch_ic_symbol(p, s3, false, s);
  if (rc) return rc;
  rc = fft3_c2r(p, 3, cbuf(p, 0), cs, mom, s);
  if (rc) return rc;
  // Psi1 into disp
  rc = ic_common(p, noise, ic, disp, 1, 1.0, s);
  if (rc) return rc;
  const double ae = a * a * pm_cosmo_hubble_e(c, a);
  const double f1 = pm_cosmo_growth_rate(c, a);
  const double f2 = 2.0 * f1 + (3.0 / 143.0) * (1.0 - om);
  return launch_ic_lattice2(p, disp, mom, pos, mom, ae * f1, ae * f2, s);
}

int pm_noise_fix(pm_plan* p, const void* noise, int pair_mode, void* noise_out, void* stream) {
  using namespace pm;
  if (!p) return set_error(PM_ERR_ARG, "pm_noise_fix: null plan");
  if (!noise || !noise_out) return set_error(PM_ERR_ARG, "pm_noise_fix: null pointer");
  if (pair_mode < 0 || pair_mode > 2) return set_error(PM_ERR_ARG, "pm_noise_fix: bad pair_mode %d", pair_mode);
  if (pair_mode == 2 && p->nb % 2 != 0)
    return set_error(PM_ERR_ARG, "pm_noise_fix: pair_mode 2 needs an even number of boxes (%d)", p->nb);
  p->dens_valid = false;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = fft3_r2c(p, noise, cbuf(p, 0), s);
  if (rc) return rc;
  const double n = (double)p->n;
  const int mask = pair_mode == 0 ? 0 : (pair_mode == 1 ? 3 : 2);
  rc = launch_fix_spectrum(p, std::pow(n, 1.5) / (n * n * n), mask, s);
  if (rc) return rc;
  return fft3_c2r(p, p->nb, cbuf(p, 0), cstride(p), noise_out, s);
}

int pm_ic_zeldovich_adjoint(pm_plan* p, const pm_ic_params* ic, const void* lam_pos, const void* lam_mom,
                            void* disp_scratch, void* lam_noise, void* stream) {
  using namespace pm;
  if (!p) return set_error(PM_ERR_ARG, "pm_ic_zeldovich_adjoint: null plan");
  if (p->nb != 1) return set_error(PM_ERR_ARG, "pm_ic_zeldovich_adjoint: needs a single-box plan");
  p->dens_valid = false;
  if (!ic || !lam_pos || !lam_mom || !disp_scratch || !lam_noise)
    return set_error(PM_ERR_ARG, "pm_ic_zeldovich_adjoint: null pointer");
  if (ic->pk_kind != PM_PK_POWERLAW && ic->pk_kind != PM_PK_EH98)
    return set_error(PM_ERR_ARG, "pm_ic_zeldovich_adjoint: bad pk_kind");
  if (!(ic->a_init > 0.0) || !(ic->a_norm > 0.0))
    return set_error(PM_ERR_ARG, "pm_ic_zeldovich_adjoint: bad scale factors");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double a = ic->a_init;
  const double fac = a * a * pm_cosmo_hubble_e(&ic->cosmo, a) * pm_cosmo_growth_rate(&ic->cosmo, a);
  int rc = launch_ic_lattice_adj(p, lam_pos, lam_mom, disp_scratch, fac, s);
  if (rc) return rc;
  rc = fft3_r2c_n(p, 3, disp_scratch, cbuf(p, 0), s);  // the three components in one set of launches
  if (rc) return rc;
  rc = launch_ic_symbol(p, ic_symbol_of(p, ic, 1, 1.0), true, s);
  if (rc) return rc;
  return fft3_c2r(p, 1, cbuf(p, 0), 0, lam_noise, s);
}

int pm_ic_2lpt_adjoint(pm_plan* p, const void* noise, const pm_ic_params* ic, const void* lam_pos,
                       const void* lam_mom, void* scratch, void* lam_noise, void* stream) {
  using namespace pm;
  int rc = check_ic(p, noise, ic, scratch, "pm_ic_2lpt_adjoint");
  if (rc) return rc;
  p->dens_valid = false;
  if (p->nb != 1) return set_error(PM_ERR_ARG, "pm_ic_2lpt_adjoint: needs a single-box plan");
  if (!lam_pos || !lam_mom || !lam_noise) return set_error(PM_ERR_ARG, "pm_ic_2lpt_adjoint: null pointer");
  if (lam_noise == noise || lam_noise == scratch)
    return set_error(PM_ERR_ARG, "pm_ic_2lpt_adjoint: lam_noise must not alias noise or scratch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  const int64_t cs = cstride(p);
  char* h = static_cast<char*>(scratch);               // [6][N^3]: the Hessian of chi, then its cotangents
  char* t = h + 6 * n3 * (int64_t)p->esize;            // [3][N^3]
  char* t1 = t + n3 * (int64_t)p->esize;
  const pm_cosmology* c = &ic->cosmo;
  const double a = ic->a_init;
  const double ae = a * a * pm_cosmo_hubble_e(c, a);
  const double om = pm_cosmo_omega_m_a(c, a);
  const double f1 = pm_cosmo_growth_rate(c, a);
  const double f2 = 2.0 * f1 + (3.0 / 143.0) * (1.0 - om);
  const double c2 = (3.0 / 7.0) * std::pow(om, -1.0 / 143.0);
  IcSymbol sy = ic_symbol_of(p, ic, 1, 1.0);
  // first order: the Zel'dovich map's transpose applied to lam_pos + ae f1 lam_mom
  rc = launch_ic_lattice_adj(p, lam_pos, lam_mom, t, ae * f1, s);
  if (rc) return rc;
  rc = fft3_r2c_n(p, 3, t, cbuf(p, 0), s);
  if (rc) return rc;
  rc = launch_ic_symbol(p, sy, true, s);
  if (rc) return rc;
  rc = fft3_c2r(p, 1, cbuf(p, 0), 0, lam_noise, s);
  if (rc) return rc;
  // the six Hessian components of chi (as the forward pass computes them)
  for (int pass = 0; pass < 2; ++pass) {
    rc = fft3_r2c(p, noise, cbuf(p, 0), s);
    if (rc) return rc;
    sy.mode = 1 + pass;
    rc = launch_ic_symbol(p, sy, false, s);
    if (rc) return rc;
    rc = fft3_c2r(p, 3, cbuf(p, 0), cs, h + pass * 3 * n3 * (int64_t)p->esize, s);
    if (rc) return rc;
  }
  // cotangent of S: the transpose of Psi2 = c2 IDFT(i k DFT(S) / k^2) applied to
  // lam_pos + ae f2 lam_mom
  rc = launch_ic_lattice_adj(p, lam_pos, lam_mom, t, ae * f2, s);
  if (rc) return rc;
  rc = fft3_r2c_n(p, 3, t, cbuf(p, 0), s);
  if (rc) return rc;
  IcSymbol s3 = sy;
  s3.mode = 3;
  s3.coef = c2 / ((double)n3);
  rc = launch_ic_symbol(p, s3, true, s);
  if (rc) return rc;
  rc = fft3_c2r(p, 1, cbuf(p, 0), 0, t, s);
  if (rc) return rc;
  // cotangents of the Hessian components, then the transposes of their symbols
  rc = launch_lpt2_source_adj(p, h, t, s);
  if (rc) return rc;
  for (int pass = 0; pass < 2; ++pass) {
    rc = fft3_r2c_n(p, 3, h + pass * 3 * n3 * (int64_t)p->esize, cbuf(p, 0), s);
    if (rc) return rc;
    sy.mode = 1 + pass;
    rc = launch_ic_symbol(p, sy, true, s);
    if (rc) return rc;
    rc = fft3_c2r(p, 1, cbuf(p, 0), 0, t1, s);
    if (rc) return rc;
    rc = launch_accumulate(p, lam_noise, t1, n3, s);
    if (rc) return rc;
  }
  return PM_OK;
}

int pm_noise_truncate(pm_plan* fine, const void* noise_fine, pm_plan* coarse, void* noise_coarse, void* stream) {
  using namespace pm;
  if (!fine || !coarse) return set_error(PM_ERR_ARG, "pm_noise_truncate: null plan");
  if (!noise_fine || !noise_coarse) return set_error(PM_ERR_ARG, "pm_noise_truncate: null pointer");
  if (fine->nb != 1 || coarse->nb != 1) return set_error(PM_ERR_ARG, "pm_noise_truncate: needs single-box plans");
  if (fine->dtype != coarse->dtype) return set_error(PM_ERR_ARG, "pm_noise_truncate: plans differ in dtype");
  if (coarse->n > fine->n || fine->n % coarse->n != 0)
    return set_error(PM_ERR_ARG, "pm_noise_truncate: coarse N (%d) must divide fine N (%d)", coarse->n, fine->n);
  fine->dens_valid = coarse->dens_valid = false;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = fft3_r2c(fine, noise_fine, cbuf(fine, 0), s);
  if (rc) return rc;
  rc = launch_truncate_spectrum(fine, coarse, s);
  if (rc) return rc;
  return fft3_c2r(coarse, 1, cbuf(coarse, 0), 0, noise_coarse, s);
}

// Coefficient g(a) of the linear Poisson-gauge displacement xi_lin(a) = g(a) IDFT(i k
// delta_L_hat / k^4) (delta_L at a_init) and its derivative g'(a) = dg/dlna:
// g = (3f + (9/2) Omega_m(a)) calh(a)^2 D(a)/D(a_init), calh in inverse cells.
static void gr_shift_coefficients(const pm_cosmology* c, double a, double a_init, double dx, double* g, double* gp) {
  const double cg = kC_over_H0 / dx;
  const double e = pm_cosmo_hubble_e(c, a);
  const double h2 = (a * e / cg) * (a * e / cg);
  const double om = pm_cosmo_omega_m_a(c, a);
  const double f = pm_cosmo_growth_rate(c, a);
  const double dratio = pm_cosmo_growth(c, a) / pm_cosmo_growth(c, a_init);
  // df/dlna from the growth equation; dOm/dlna = -3 Om (1 - Om); dcalH^2/dlna = calH^2 (2 - 3 Om); dD/dlna = f D
  const double fp = 1.5 * om - f * f - (2.0 - 1.5 * om) * f;
  const double sfac = 3.0 * f + 4.5 * om;
  *g = sfac * h2 * dratio;
  *gp = h2 * dratio * (3.0 * fp - 13.5 * om * (1.0 - om) + sfac * (2.0 - 3.0 * om + f));
}

int pm_ic_gauge(pm_plan* p, const void* noise, const pm_ic_params* ic, void* disp, const void* pos_n,
                const void* mom_n, void* pos_gr, void* mom_gr, void* stream) {
  using namespace pm;
  int rc = check_ic(p, noise, ic, disp, "pm_ic_gauge");
  if (rc) return rc;
  p->dens_valid = false;
  if (p->nb != 1) return set_error(PM_ERR_ARG, "pm_ic_gauge: needs a single-box plan");
  if (!pos_n || !mom_n || !pos_gr || !mom_gr) return set_error(PM_ERR_ARG, "pm_ic_gauge: null pointer");
  const pm_cosmology* c = &ic->cosmo;
  const double a = ic->a_init;
  double g, gp;
  gr_shift_coefficients(c, a, a, p->box / p->n, &g, &gp);
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = ic_common(p, noise, ic, disp, 2, g, s);
  if (rc) return rc;
  const double fac = a * a * pm_cosmo_hubble_e(c, a) * (gp / g);
  return launch_ic_gauge_lattice(p, disp, pos_n, mom_n, pos_gr, mom_gr, fac, s);
}

int pm_xi_linear(pm_plan* p, const void* noise, const pm_ic_params* ic, double a, void* xi, void* stream) {
  using namespace pm;
  int rc = check_ic(p, noise, ic, xi, "pm_xi_linear");
  if (rc) return rc;
  p->dens_valid = false;
  if (p->nb != 1) return set_error(PM_ERR_ARG, "pm_xi_linear: needs a single-box plan");
  if (!(a > 0.0)) return set_error(PM_ERR_ARG, "pm_xi_linear: bad scale factor");
  double g, gp;
  gr_shift_coefficients(&ic->cosmo, a, ic->a_init, p->box / p->n, &g, &gp);
  return ic_common(p, noise, ic, xi, 2, g, static_cast<hipStream_t>(stream));
}

}  // extern "C"
