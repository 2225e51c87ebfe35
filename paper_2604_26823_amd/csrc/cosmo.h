// Host FP64 cosmology: growth factors, FastPM step factors and the
// whitening multiplier table (paper section 2.2.1 items 1-2).
#pragma once

#include <vector>

namespace ic {

struct Coeffs {
  std::vector<double> a;      // a_n, n = 0..S
  std::vector<double> a_mid;  // (a_n + a_{n+1}) / 2
  std::vector<double> Dr;     // drift factors, n = 0..S-1
  std::vector<double> K1, K2; // first / second half-kick factors
  std::vector<double> kick;   // merged kicks c_0..c_S applied before drift n (c_S last)
  double D1_init = 0, f1_init = 0, D2_init = 0, f2_init = 0, E_init = 0;
  double rsd_factor = 0;      // 1 / (a_final^2 E(a_final))
  double pk_amplitude = 0;    // A of P(k) = A k^ns T(k)^2
};

struct CosmoParams {
  double omega_m, h, n_s, sigma8, a_init, a_final;
  int n_steps;
};

// Solves the growth equations and the sigma8 normalisation.
Coeffs compute_coeffs(const CosmoParams& p);

// w(n2) = sqrt(P(k) / dq^3), k = (2 pi / box) sqrt(n2), for n2 = 0..n2_max;
// w(0) = 0.
std::vector<double> whitening_table(const CosmoParams& p, double amplitude, double box,
                                    int n_side);

// Linear growth D1(a) / f1(a) and second-order D2 / f2 (exposed for tests).
void growth_at(const CosmoParams& p, const std::vector<double>& a, std::vector<double>& D1,
               std::vector<double>& f1, std::vector<double>& D2, std::vector<double>& f2);

double bbks_power_unnormalised(const CosmoParams& p, double k);

// Comoving distance chi(a) = (c/H0) int_a^1 da' / (a'^2 E(a')) in Mpc/h
// (c/H0 = 2997.92458 Mpc/h), composite Simpson over 4096 intervals.
double comoving_distance(double omega_m, double a);

// Inverse comoving distance for the lightcone (section 2.2.1 item 3,
// appendix A): a(chi) on n nodes chi_k = chi_min + k h spanning
// [chi(a_hi), chi(a_lo)], with slopes da/dchi = -a^2 E(a) / (c/H0), for
// cubic Hermite interpolation.  The values come from the ODE
// da/dchi = -a^2 E / (c/H0) integrated by classical Runge-Kutta (64 substeps
// per node interval) from a(chi_min) = a_hi.
struct LightconeTable {
  double chi_min = 0, chi_max = 0, h = 0;
  std::vector<double> a, slope;
};
LightconeTable lightcone_table(double omega_m, double a_lo, double a_hi, int n);

}  // namespace ic
