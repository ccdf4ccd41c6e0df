// Gas density of the local fuel/N2 mixture (Section 2.5, eq. 24) and its
// inversion from the vapour content, on the device, in FP64.
//
// rho_G(T, omega) = p M / (Z R T) with the vapour mole fraction y of the mass
// fraction omega, M = y M_v + (1 - y) M_G, and Z = 1 (ideal model) or the
// largest root of the Peng-Robinson cubic of the mixture (the mixing rules of
// the equilibrium: a = sum y_i y_j sqrt(a_i a_j)(1 - k_ij), b = sum y_i b_i).
// The inversion finds omega with rho_G(T, omega) omega = q (vapour mass per
// unit gas volume): the ideal model's closed form, refined for Peng-Robinson
// by Newton's method on F(omega) = rho_G omega - q inside the bracket
// [q/rho_G(T, 1), q/rho_G(T, 0)], dF by dual numbers.
#pragma once
#include "ds_thermo.h"

namespace dsv {

template <class S>
__device__ inline S gas_mole_fraction(const DevParams& P, S om) {
  S a = om / P.M_v;
  return a / (a + (1.0 - om) / P.M_G);
}

template <class S>
__device__ inline S gas_rho(const DevParams& P, double T, S om) {
  S y = gas_mole_fraction(P, om);
  S M = y * P.M_v + (1.0 - y) * P.M_G;
  const double RT = R_GAS * T;
  if (P.eq_model == 0) return M * (P.p / RT);
  double a1, a2, b1, b2;
  pr_ab<double>(T, P.Tc, P.Pc, P.om, a1, b1);
  pr_ab<double>(T, P.Tc_G, P.Pc_G, P.om_G, a2, b2);
  const double a12 = sqrt(a1 * a2) * (1.0 - P.kij);
  S y2 = 1.0 - y;
  S a = y * y * a1 + 2.0 * y * y2 * a12 + y2 * y2 * a2;
  S b = y * b1 + y2 * b2;
  S A = a * (P.p / (RT * RT));
  S B = b * (P.p / RT);
  S Z = pr_root(A, B);
  return (M * (P.p / RT)) / Z;
}

// (omega, rho_G) of the gas at temperature T holding q kg of vapour per m^3
// of gas; q <= 0 (round-off undershoot) gives omega = q/rho_G(T, 0).
__device__ inline void gas_invert(const DevParams& P, double T, double q, double& om, double& rho) {
  const double r0 = gas_rho<double>(P, T, 0.0);
  if (!(q > 0.0)) {
    om = q / r0;
    rho = r0;
    return;
  }
  const double a = q * R_GAS * T / P.p;
  double w = (a / P.M_G) / (1.0 - a / P.M_v + a / P.M_G);   // ideal gas: exact
  if (P.eq_model != 0) {
    double lo = q / gas_rho<double>(P, T, 1.0), hi = fmin(q / r0, 1.0);
    w = fmin(fmax(w, lo), hi);
    for (int it = 0; it < 60; ++it) {
      const dual r = gas_rho<dual>(P, T, mkd(w, 1.0));
      const double F = r.v * w - q, dF = r.d * w + r.v;
      if (F > 0.0) hi = w;
      else lo = w;
      double wn = w - F / dF;
      if (!(wn >= lo && wn <= hi)) wn = 0.5 * (lo + hi);
      const double step = fabs(wn - w);
      w = wn;
      if (step <= 1e-15 * w) break;
    }
  }
  om = w;
  rho = gas_rho<double>(P, T, w);
}

}  // namespace dsv
