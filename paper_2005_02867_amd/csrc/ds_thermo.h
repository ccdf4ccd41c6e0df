// Interface phase equilibrium on the device (Section 2.5, eqs. 22-25),
// always in FP64.
//
// Ideal model: Clausius-Clapeyron vapour pressure about (T_ref, p_ref),
// y = p0/p.  Peng-Robinson model: eq. 22 with x = 1 solved for y by Newton's
// method on g(y) = ln y + ln phi_hat(T, p, y) - ln[p0 phi(T, p0) Poy / p],
// the derivative of ln phi_hat taken by forward-mode dual numbers through
// the mixing rules and the cubic's largest root (implicit-function rule).
#pragma once
#include "ds_device.h"

namespace dsv {

struct dual {
  double v, d;
};
__device__ __forceinline__ dual mkd(double v, double d = 0.0) { return dual{v, d}; }
__device__ __forceinline__ dual operator+(dual a, dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dual operator-(dual a, dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dual operator*(dual a, dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ dual operator/(dual a, dual b) {
  double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ dual operator-(dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ dual operator+(dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ dual operator+(double a, dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ dual operator-(dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ dual operator-(double a, dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ dual operator*(dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ dual operator*(double a, dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ dual operator/(dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ dual operator/(double a, dual b) {
  double q = a / b.v;
  return {q, -q * b.d / b.v};
}
__device__ __forceinline__ dual dlog(dual a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ dual dexp(dual a) {
  double e = exp(a.v);
  return {e, e * a.d};
}
__device__ __forceinline__ dual dsqrt(dual a) {
  double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}
__device__ __forceinline__ double dlog(double a) { return log(a); }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(dual a) { return a.v; }
template <class S>
__device__ inline S cst(double v);
template <>
__device__ inline double cst<double>(double v) { return v; }
template <>
__device__ inline dual cst<dual>(double v) { return dual{v, 0.0}; }

// Largest real root of Z^3 - (1-B) Z^2 + (A - 3B^2 - 2B) Z - (AB - B^2 - B^3):
// Newton from the Cauchy bound (monotone on the convex branch right of the
// largest root), derivative by the implicit-function rule.
__device__ inline double pr_root_value(double A, double B) {
  const double c2 = -(1.0 - B), c1 = A - 3.0 * B * B - 2.0 * B, c0 = -(A * B - B * B - B * B * B);
  double z = 1.0 + fmax(fabs(c2), fmax(fabs(c1), fabs(c0)));
  for (int it = 0; it < 200; ++it) {
    const double f = ((z + c2) * z + c1) * z + c0;
    const double fp = (3.0 * z + 2.0 * c2) * z + c1;
    const double dz = f / fp;
    z -= dz;
    // converged to within two units in the last place (a tighter test is
    // never met once the iterate oscillates by one ulp)
    if (fabs(dz) <= 4.5e-16 * fabs(z)) break;
  }
  return z;
}
__device__ inline double pr_root(double A, double B) { return pr_root_value(A, B); }
__device__ inline dual pr_root(dual A, dual B) {
  const double a = A.v, b = B.v;
  const double z = pr_root_value(a, b);
  const double c2 = -(1.0 - b), c1 = a - 3.0 * b * b - 2.0 * b;
  const double FZ = (3.0 * z + 2.0 * c2) * z + c1;
  const double FA = z - b;
  const double FB = z * z + (-6.0 * b - 2.0) * z + (-a + 2.0 * b + 3.0 * b * b);
  return {z, -(FA * A.d + FB * B.d) / FZ};
}

template <class S>
__device__ inline void pr_ab(S T, double Tc, double Pc, double om, S& a, double& b) {
  const double kap = 0.37464 + 1.54226 * om - 0.26992 * om * om;
  S s = 1.0 + kap * (1.0 - dsqrt(T / Tc));
  a = (0.45724 * R_GAS * R_GAS * Tc * Tc / Pc) * (s * s);
  b = 0.07780 * R_GAS * Tc / Pc;
}

// ln of the fuel fugacity coefficient in a fuel(y)/gas(1-y) mixture at (T, p).
template <class S>
__device__ inline S pr_lnphi_fuel(const DevParams& P, S T, S p, S y) {
  S a1, a2;
  double b1, b2;
  pr_ab(T, P.Tc, P.Pc, P.om, a1, b1);
  pr_ab(T, P.Tc_G, P.Pc_G, P.om_G, a2, b2);
  S a12 = dsqrt(a1 * a2) * (1.0 - P.kij);
  S y2 = 1.0 - y;
  S a = y * y * a1 + 2.0 * y * y2 * a12 + y2 * y2 * a2;
  S b = y * b1 + y2 * b2;
  S RT = R_GAS * T;
  S A = a * p / (RT * RT);
  S B = b * p / RT;
  S Z = pr_root(A, B);
  S sum_ya = y * a1 + y2 * a12;
  const double s2 = 1.4142135623730951;
  S lnq = dlog((Z + (1.0 + s2) * B) / (Z + (1.0 - s2) * B));
  return (b1 / b) * (Z - 1.0) - dlog(Z - B) - A / (2.0 * s2 * B) * (2.0 * sum_ya / a - b1 / b) * lnq;
}

template <class S>
__device__ inline S vapour_pressure(const DevParams& P, S T, S dh) {
  return P.p_ref * dexp(-(dh * P.M_v / R_GAS) * (1.0 / T - 1.0 / P.T_ref));
}

// Right-hand side of eq. 23 in logs: ln[p0 phi(T, p0) Poy / p] (x = 1).
template <class S>
__device__ inline S pr_lnrhs(const DevParams& P, S T, S dh) {
  S p0 = vapour_pressure(P, T, dh);
  S lnphi_pure = pr_lnphi_fuel<S>(P, T, p0, cst<S>(1.0));
  const double vL = P.M_v / P.rho_L;
  return dlog(p0) + lnphi_pure + vL * (P.p - p0) / (R_GAS * T) - log(P.p);
}

// Interface vapour mole fraction y(T).
__device__ inline double equilibrium_y(const DevParams& P, double T) {
  const double p0 = vapour_pressure(P, T, P.dh);
  double y = fmin(p0 / P.p, 1.0 - 1e-12);
  if (P.eq_model == 0) return y;
  const double L = pr_lnrhs<double>(P, T, P.dh);
  // Stop when the step is below 1e-15 y, or below 1e-14 y and no longer
  // shrinking: at the rounding floor of g some temperatures (about 1 in 500)
  // alternate between two iterates 1.2e-15 apart, and without the second
  // test they ran to the iteration cap, holding their whole wave for ten
  // times the usual six iterations.
  double prev = INFINITY;
  for (int it = 0; it < 60; ++it) {
    dual yd = mkd(y, 1.0);
    dual g = dlog(yd) + pr_lnphi_fuel<dual>(P, mkd(T), mkd(P.p), yd) - L;
    double ynew = y - g.v / g.d;
    if (!(ynew > 0.0)) ynew = 0.5 * y;
    ynew = fmin(ynew, 1.0 - 1e-12);
    const double step = fabs(ynew - y);
    const bool done = step <= 1e-15 * ynew || (step <= 1e-14 * ynew && step >= prev);
    prev = step;
    y = ynew;
    if (done) break;
  }
  return y;
}

// y(T) with its derivatives in T and dh_ev: closed form for the ideal model,
// the implicit-function rule on g(y, T, dh) = 0 for Peng-Robinson
// (dy = -g_T dT/g_y - g_dh ddh/g_y, partials by dual numbers).  A value held
// at the cap 1 - 1e-12 has zero derivatives.
__device__ inline double equilibrium_y_grad(const DevParams& P, double T, double& dT, double& ddh) {
  const double cap = 1.0 - 1e-12;
  const double y = equilibrium_y(P, T);
  dT = 0.0;
  ddh = 0.0;
  if (P.eq_model == 0) {
    const double yr = vapour_pressure(P, T, P.dh) / P.p;
    if (yr <= cap) {
      dT = yr * (P.dh * P.M_v / R_GAS) / (T * T);
      ddh = -yr * (P.M_v / R_GAS) * (1.0 / T - 1.0 / P.T_ref);
    }
    return y;
  }
  if (y >= cap) return y;
  const dual gy = dlog(mkd(y, 1.0)) + pr_lnphi_fuel<dual>(P, mkd(T), mkd(P.p), mkd(y, 1.0));
  const dual gT = pr_lnphi_fuel<dual>(P, mkd(T, 1.0), mkd(P.p), mkd(y)) - pr_lnrhs<dual>(P, mkd(T, 1.0), mkd(P.dh));
  const dual gH = -pr_lnrhs<dual>(P, mkd(T), mkd(P.dh, 1.0));
  dT = -gT.d / gy.d;
  ddh = -gH.d / gy.d;
  return y;
}

__device__ __forceinline__ double mass_fraction(const DevParams& P, double y) {
  return y * P.M_v / (y * P.M_v + (1.0 - y) * P.M_G);
}

}  // namespace dsv
