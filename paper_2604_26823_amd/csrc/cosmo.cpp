// Host FP64 cosmology of the forward model.
//
// Flat LCDM without radiation, E(a)^2 = Om a^-3 + 1 - Om.  Growth factors
// come from the growth equations in x = ln a,
//   D'' + (2 - 3/2 Om(a)) D' - 3/2 Om(a) D = 0,
//   D2'' + (2 - 3/2 Om(a)) D2' - 3/2 Om(a) D2 = -3/2 Om(a) D1^2,
// Om(a) = Om a^-3 / E^2, integrated with classical fourth-order Runge-Kutta
// from a = 1e-6 on the growing modes D1 = a, D2 = -3/7 a^2, then normalised
// by D1(1) (D2 by its square).  The FastPM factors move the linear growing
// mode exactly: with G = a^3 E dD1/da = a^2 E f1 D1,
//   drift Dr_n = [D1(a_{n+1}) - D1(a_n)] / G(a_{n+1/2}),
//   kicks K1_n = [G(a_{n+1/2}) - G(a_n)] / D1(a_n),
//         K2_n = [G(a_{n+1}) - G(a_{n+1/2})] / D1(a_{n+1}).
// The power spectrum is A k^ns T_BBKS(k)^2 with shape Om h and A fixed by
// sigma8 (top hat of 8 Mpc/h), integrated by composite Gauss-Legendre in ln k.
#include "cosmo.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace ic {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct GrowthState {
  double d1, d1p, d2, d2p;
};

GrowthState rhs(double x, const GrowthState& y, double om) {
  const double a3 = std::exp(-3.0 * x);
  const double e2 = om * a3 + 1.0 - om;
  const double oma = om * a3 / e2;
  const double damp = 2.0 - 1.5 * oma;
  GrowthState d;
  d.d1 = y.d1p;
  d.d1p = -damp * y.d1p + 1.5 * oma * y.d1;
  d.d2 = y.d2p;
  d.d2p = -damp * y.d2p + 1.5 * oma * y.d2 - 1.5 * oma * y.d1 * y.d1;
  return d;
}

GrowthState axpy(const GrowthState& a, double h, const GrowthState& b) {
  return {a.d1 + h * b.d1, a.d1p + h * b.d1p, a.d2 + h * b.d2, a.d2p + h * b.d2p};
}

void rk4_step(double x, double h, GrowthState& y, double om) {
  const GrowthState k1 = rhs(x, y, om);
  const GrowthState k2 = rhs(x + 0.5 * h, axpy(y, 0.5 * h, k1), om);
  const GrowthState k3 = rhs(x + 0.5 * h, axpy(y, 0.5 * h, k2), om);
  const GrowthState k4 = rhs(x + h, axpy(y, h, k3), om);
  y.d1 += h / 6.0 * (k1.d1 + 2 * k2.d1 + 2 * k3.d1 + k4.d1);
  y.d1p += h / 6.0 * (k1.d1p + 2 * k2.d1p + 2 * k3.d1p + k4.d1p);
  y.d2 += h / 6.0 * (k1.d2 + 2 * k2.d2 + 2 * k3.d2 + k4.d2);
  y.d2p += h / 6.0 * (k1.d2p + 2 * k2.d2p + 2 * k3.d2p + k4.d2p);
}

double hubble_E(double a, double om) { return std::sqrt(om / (a * a * a) + 1.0 - om); }

double tophat(double x) {
  if (x < 1e-2) return 1.0 - x * x / 10.0 + x * x * x * x / 280.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

const double kGLx[4] = {0.1834346424956498049, 0.5255324099163289858, 0.7966664774136267396,
                        0.9602898564975362317};
const double kGLw[4] = {0.3626837833783619830, 0.3137066458778872873, 0.2223810344533744706,
                        0.1012285362903762591};

}  // namespace

double bbks_power_unnormalised(const CosmoParams& p, double k) {
  const double q = k / (p.omega_m * p.h);
  const double x = 2.34 * q;
  const double lead = x > 0 ? std::log1p(x) / x : 1.0;
  const double poly = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) +
                      std::pow(6.71 * q, 4);
  const double t = lead * std::pow(poly, -0.25);
  return std::pow(k, p.n_s) * t * t;
}

void growth_at(const CosmoParams& p, const std::vector<double>& a, std::vector<double>& D1,
               std::vector<double>& f1, std::vector<double>& D2, std::vector<double>& f2) {
  const double om = p.omega_m;
  const double a0 = 1e-6;
  std::vector<double> xs;
  for (double v : a) xs.push_back(std::log(v));
  xs.push_back(0.0);
  std::vector<size_t> order(xs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](size_t i, size_t j) { return xs[i] < xs[j]; });
  std::vector<GrowthState> at(xs.size());
  GrowthState y{a0, a0, -3.0 / 7.0 * a0 * a0, -6.0 / 7.0 * a0 * a0};
  double x = std::log(a0);
  const double hmax = 2.5e-4;
  for (size_t oi : order) {
    const double target = xs[oi];
    while (x < target) {
      const double h = std::min(hmax, target - x);
      rk4_step(x, h, y, om);
      x = (target - x <= hmax) ? target : x + h;
    }
    at[oi] = y;
  }
  const double norm = at.back().d1;
  D1.resize(a.size());
  f1.resize(a.size());
  D2.resize(a.size());
  f2.resize(a.size());
  for (size_t i = 0; i < a.size(); ++i) {
    D1[i] = at[i].d1 / norm;
    f1[i] = at[i].d1p / at[i].d1;
    D2[i] = at[i].d2 / (norm * norm);
    f2[i] = at[i].d2p / at[i].d2;
  }
}

Coeffs compute_coeffs(const CosmoParams& p) {
  if (p.n_steps < 1) throw std::invalid_argument("n_steps must be >= 1");
  const int S = p.n_steps;
  Coeffs c;
  for (int n = 0; n <= S; ++n) c.a.push_back(p.a_init + n * (p.a_final - p.a_init) / S);
  for (int n = 0; n < S; ++n) c.a_mid.push_back(0.5 * (c.a[n] + c.a[n + 1]));
  std::vector<double> all = c.a;
  all.insert(all.end(), c.a_mid.begin(), c.a_mid.end());
  std::vector<double> D1, f1, D2, f2;
  growth_at(p, all, D1, f1, D2, f2);
  auto G = [&](size_t i) { return all[i] * all[i] * hubble_E(all[i], p.omega_m) * f1[i] * D1[i]; };
  for (int n = 0; n < S; ++n) {
    const size_t i0 = n, i1 = n + 1, im = S + 1 + n;
    c.Dr.push_back((D1[i1] - D1[i0]) / G(im));
    c.K1.push_back((G(im) - G(i0)) / D1[i0]);
    c.K2.push_back((G(i1) - G(im)) / D1[i1]);
  }
  c.kick.push_back(c.K1[0]);
  for (int n = 1; n < S; ++n) c.kick.push_back(c.K2[n - 1] + c.K1[n]);
  c.kick.push_back(c.K2[S - 1]);
  c.D1_init = D1[0];
  c.f1_init = f1[0];
  c.D2_init = D2[0];
  c.f2_init = f2[0];
  c.E_init = hubble_E(p.a_init, p.omega_m);
  c.rsd_factor = 1.0 / (p.a_final * p.a_final * hubble_E(p.a_final, p.omega_m));

  // sigma8 normalisation: (1/2 pi^2) int k^3 P W(8k)^2 dlnk over [1e-5, 1e3].
  const double lo = std::log(1e-5), hi = std::log(1e3);
  const int panels = 8192;
  const double w = (hi - lo) / panels;
  double acc = 0;
  for (int i = 0; i < panels; ++i) {
    const double mid = lo + (i + 0.5) * w;
    double part = 0;
    for (int g = 0; g < 4; ++g) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double lk = mid + sgn * kGLx[g] * 0.5 * w;
        const double k = std::exp(lk);
        const double win = tophat(8.0 * k);
        part += kGLw[g] * k * k * k * bbks_power_unnormalised(p, k) * win * win;
      }
    }
    acc += part * 0.5 * w;
  }
  const double sig2 = acc / (2.0 * kPi * kPi);
  c.pk_amplitude = p.sigma8 * p.sigma8 / sig2;
  return c;
}

std::vector<double> whitening_table(const CosmoParams& p, double amplitude, double box,
                                    int n_side) {
  const int h = n_side / 2;
  const int n2max = 3 * h * h;
  const double kf = 2.0 * kPi / box;
  const double dq3 = std::pow(box / n_side, 3);
  std::vector<double> w(n2max + 1, 0.0);
  for (int n2 = 1; n2 <= n2max; ++n2) {
    const double k = kf * std::sqrt(static_cast<double>(n2));
    w[n2] = std::sqrt(amplitude * bbks_power_unnormalised(p, k) / dq3);
  }
  return w;
}

double comoving_distance(double omega_m, double a) {
  constexpr double kCH0 = 2997.92458;
  constexpr int kN = 4096;
  if (a >= 1.0) return 0.0;
  const double h = (1.0 - a) / kN;
  auto f = [&](double x) { return 1.0 / (x * x * hubble_E(x, omega_m)); };
  double s = f(a) + f(1.0);
  for (int i = 1; i < kN; ++i) s += (i % 2 ? 4.0 : 2.0) * f(a + i * h);
  return kCH0 * s * h / 3.0;
}

LightconeTable lightcone_table(double omega_m, double a_lo, double a_hi, int n) {
  constexpr double kCH0 = 2997.92458;
  constexpr int kSub = 64;
  LightconeTable t;
  t.chi_min = comoving_distance(omega_m, a_hi);
  t.chi_max = comoving_distance(omega_m, a_lo);
  t.h = (t.chi_max - t.chi_min) / (n - 1);
  auto rate = [&](double a) { return -a * a * hubble_E(a, omega_m) / kCH0; };
  t.a.resize(n);
  t.slope.resize(n);
  double a = a_hi;
  const double dc = t.h / kSub;
  for (int k = 0; k < n; ++k) {
    t.a[k] = a;
    t.slope[k] = rate(a);
    if (k + 1 == n) break;
    for (int i = 0; i < kSub; ++i) {
      const double k1 = rate(a), k2 = rate(a + 0.5 * dc * k1), k3 = rate(a + 0.5 * dc * k2),
                   k4 = rate(a + dc * k3);
      a += dc * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
    }
  }
  return t;
}

}  // namespace ic
