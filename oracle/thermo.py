"""Phase equilibrium and gas density (paper Section 2.5, eqs. 22-25).

Test infrastructure: the CPU oracle only.

* Ideal limit: vapour pressure from Clausius-Clapeyron about the normal
  boiling point (T_ref, p_ref) with the latent heat of the configuration;
  fugacity coefficients 1 and no Poynting factor, so eq. 23 reads y = p0/p.
* Non-ideal: Peng-Robinson (1976) cubic equation of state for the
  compressibility factor Z and the gas-phase fugacity coefficients of the
  pure fuel (phi at p0) and of the fuel in the fuel/N2 mixture (phi_hat at
  p), Poynting factor with v_L = M_v/rho_L (eq. 25); eq. 23 is iterated as
  written (y on the left, phi_hat(y) on the right) to convergence, with a
  pure liquid (x = 1).
* Gas density, eq. 24: rho_G = p M_G / (Z R T) for the ambient nitrogen
  (Z = 1 in the ideal model, PR Z of pure N2 otherwise).
"""
from __future__ import annotations

import math

import numpy as np
import torch

R_GAS = 8.314462618
SQRT2 = math.sqrt(2.0)


# ---------------------------------------------------------------- ideal
def vapour_pressure(T, prm):
    """Clausius-Clapeyron p0(T) = p_ref exp[-(dh_ev M_v / R)(1/T - 1/T_ref)]."""
    dh_molar = prm["dh_ev"] * prm["M_v"]
    if isinstance(T, torch.Tensor):
        return prm["p_ref"] * torch.exp(-(dh_molar / R_GAS) * (1.0 / T - 1.0 / prm["T_ref"]))
    return prm["p_ref"] * np.exp(-(dh_molar / R_GAS) * (1.0 / np.asarray(T) - 1.0 / prm["T_ref"]))


def mass_fraction(y, prm):
    """Vapour mole fraction -> mass fraction in the binary fuel/N2 gas."""
    return y * prm["M_v"] / (y * prm["M_v"] + (1.0 - y) * prm["M_G"])


# ---------------------------------------------------------------- Peng-Robinson
def pr_pure_ab(T, Tc, Pc, acentric):
    """PR attraction a(T) and co-volume b of one component."""
    kappa = 0.37464 + 1.54226 * acentric - 0.26992 * acentric ** 2
    alpha_T = (1.0 + kappa * (1.0 - np.sqrt(np.asarray(T, dtype=np.float64) / Tc))) ** 2
    a = 0.45724 * R_GAS ** 2 * Tc ** 2 / Pc * alpha_T
    b = 0.07780 * R_GAS * Tc / Pc
    return a, b


def pr_largest_root(A, B):
    """Largest real root Z of Z^3 - (1-B)Z^2 + (A-3B^2-2B)Z - (AB-B^2-B^3) = 0,
    found as companion-matrix eigenvalues (numpy), one cubic per entry."""
    A = np.atleast_1d(np.asarray(A, dtype=np.float64))
    B = np.atleast_1d(np.asarray(B, dtype=np.float64))
    c2 = -(1.0 - B)
    c1 = A - 3.0 * B ** 2 - 2.0 * B
    c0 = -(A * B - B ** 2 - B ** 3)
    n = A.shape[0]
    comp = np.zeros((n, 3, 3))
    comp[:, 0, :] = np.stack([-c2, -c1, -c0], axis=1)
    comp[:, 1, 0] = 1.0
    comp[:, 2, 1] = 1.0
    ev = np.linalg.eigvals(comp)
    real = np.abs(ev.imag) <= 1e-10 * np.maximum(1.0, np.abs(ev.real))
    zr = np.where(real, ev.real, -np.inf)
    return zr.max(axis=1)


def pr_components(T, prm):
    """(a1, b1) fuel and (a2, b2) nitrogen at temperature T."""
    a1, b1 = pr_pure_ab(T, prm["Tc"], prm["Pc"], prm["acentric"])
    a2, b2 = pr_pure_ab(T, prm["Tc_G"], prm["Pc_G"], prm["acentric_G"])
    return a1, b1, a2, b2


def pr_ln_phi_fuel(T, p, y, prm):
    """ln of the fuel fugacity coefficient in a fuel(y)/N2(1-y) gas at (T, p),
    and the mixture Z.  y = 1 gives the pure-fuel coefficient."""
    T = np.asarray(T, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64) * np.ones_like(T)
    a1, b1, a2, b2 = pr_components(T, prm)
    a12 = np.sqrt(a1 * a2) * (1.0 - prm["kij"])
    y2 = 1.0 - y
    a = y * y * a1 + 2.0 * y * y2 * a12 + y2 * y2 * a2
    b = y * b1 + y2 * b2
    RT = R_GAS * T
    A = a * p / RT ** 2
    B = b * p / RT
    Z = pr_largest_root(A.ravel(), B.ravel()).reshape(A.shape)
    sum_ya = y * a1 + y2 * a12            # sum_j y_j a_1j
    lnphi = (b1 / b) * (Z - 1.0) - np.log(Z - B) - A / (2.0 * SQRT2 * B) * (
        2.0 * sum_ya / a - b1 / b) * np.log((Z + (1.0 + SQRT2) * B) / (Z + (1.0 - SQRT2) * B))
    return lnphi, Z


def pr_Z_pure_gas(T, p, prm):
    """PR compressibility of pure nitrogen (the ambient gas)."""
    a2, b2 = pr_pure_ab(T, prm["Tc_G"], prm["Pc_G"], prm["acentric_G"])
    RT = R_GAS * np.asarray(T, dtype=np.float64)
    return pr_largest_root(a2 * p / RT ** 2, b2 * p / RT)[0] if np.ndim(T) == 0 else \
        pr_largest_root(a2 * p / RT ** 2, b2 * p / RT)


def equilibrium_y(T, prm, max_iter=200):
    """Interface vapour mole fraction y(T) from eq. 23 with x = 1.

    Ideal model: y = p0(T)/p.  PR model: y_{k+1} = p0 phi(T,p0) Poy / (p
    phi_hat(T,p,y_k)), starting from the ideal value, until the change is
    below 1e-15 (relative).  The result is capped at 1 - 1e-12.
    """
    T = np.asarray(T, dtype=np.float64)
    p = prm["p"]
    p0 = vapour_pressure(T, prm)
    y = np.minimum(p0 / p, 1.0 - 1e-12)
    if prm["eq_model"] == 0:
        return y
    ln_phi_pure, _ = pr_ln_phi_fuel(T, p0, np.ones_like(T), prm)
    vL = prm["M_v"] / prm["rho_L"]
    ln_poy = vL * (p - p0) / (R_GAS * T)
    ln_rhs = np.log(p0) + ln_phi_pure + ln_poy - math.log(p)
    for _ in range(max_iter):
        ln_phihat, _ = pr_ln_phi_fuel(T, p, y, prm)
        y_new = np.minimum(np.exp(ln_rhs - ln_phihat), 1.0 - 1e-12)
        done = np.all(np.abs(y_new - y) <= 1e-15 * np.abs(y_new))
        y = y_new
        if done:
            break
    return y


def equilibrium_residual(T, y, prm):
    """ln of (left side / right side) of eq. 22 with x = 1 (PR model)."""
    T = np.asarray(T, dtype=np.float64)
    p = prm["p"]
    p0 = vapour_pressure(T, prm)
    ln_phi_pure, _ = pr_ln_phi_fuel(T, p0, np.ones_like(T), prm)
    ln_phihat, _ = pr_ln_phi_fuel(T, p, y, prm)
    vL = prm["M_v"] / prm["rho_L"]
    return (np.log(p0) + ln_phi_pure + vL * (p - p0) / (R_GAS * T)) - (math.log(p) + np.log(y) + ln_phihat)


def _richardson(f, x, step):
    """df/dx by central differences at steps `step` and `step`/2, combined
    by Richardson extrapolation (error O(step^4))."""
    d1 = (f(x + step) - f(x - step)) / (2.0 * step)
    d2 = (f(x + 0.5 * step) - f(x - 0.5 * step)) / step
    return (4.0 * d2 - d1) / 3.0


def _prm_float(prm):
    q = dict(prm)
    q["dh_ev"] = float(q["dh_ev"])
    return q


class _PRSaturation(torch.autograd.Function):
    """omega_sat(T) of the Peng-Robinson model as a differentiable function
    of T (per cell) and dh_ev.  The value is the converged fixed point of
    eq. 23; its derivatives are taken by Richardson-extrapolated central
    differences of that converged root (steps 0.05 K and 1e-4 dh_ev)."""

    @staticmethod
    def forward(ctx, T, dh, prm):
        q = _prm_float(prm)
        q["dh_ev"] = float(dh)
        Tn = T.detach().cpu().numpy()
        ctx.save_for_backward(T, dh)
        ctx.q = q
        return torch.as_tensor(mass_fraction(equilibrium_y(Tn, q), q), dtype=torch.float64)

    @staticmethod
    def backward(ctx, gbar):
        T, dh = ctx.saved_tensors
        q = ctx.q
        Tn = T.detach().cpu().numpy()

        def w_of_T(t):
            return mass_fraction(equilibrium_y(t, q), q)

        def w_of_dh(d):
            qq = dict(q)
            qq["dh_ev"] = d
            return mass_fraction(equilibrium_y(Tn, qq), qq)

        dT = torch.as_tensor(_richardson(w_of_T, Tn, 0.05), dtype=torch.float64)
        ddh = torch.as_tensor(_richardson(w_of_dh, q["dh_ev"], 1e-4 * q["dh_ev"]), dtype=torch.float64)
        return gbar * dT, (gbar * ddh).sum().reshape(dh.shape), None


class _PRGasZ(torch.autograd.Function):
    """Peng-Robinson Z of the ambient gas as a differentiable function of
    T_amb (Richardson-extrapolated central differences, step 0.05 K)."""

    @staticmethod
    def forward(ctx, T, prm):
        ctx.save_for_backward(T)
        ctx.prm = prm
        return torch.as_tensor(float(pr_Z_pure_gas(float(T), prm["p"], prm)), dtype=torch.float64)

    @staticmethod
    def backward(ctx, gbar):
        (T,) = ctx.saved_tensors
        prm = ctx.prm
        dZ = _richardson(lambda t: float(pr_Z_pure_gas(t, prm["p"], prm)), float(T), 0.05)
        return gbar * dZ, None


def saturation_omega(T, prm):
    """Interface vapour mass fraction omega_sat(T_int) (torch in, torch out).

    The ideal model stays in torch (differentiable in T and dh_ev).  The PR
    model is evaluated in numpy; when T requires a gradient or dh_ev is a
    tensor, its derivative comes from _PRSaturation."""
    if prm["eq_model"] == 0:
        y = torch.clamp(vapour_pressure(T, prm) / prm["p"], max=1.0 - 1e-12)
        return mass_fraction(y, prm)
    dh = prm["dh_ev"]
    if T.requires_grad or isinstance(dh, torch.Tensor):
        dh_t = dh if isinstance(dh, torch.Tensor) else torch.tensor(float(dh), dtype=torch.float64)
        return _PRSaturation.apply(T, dh_t, _prm_float(prm))
    y = equilibrium_y(T.detach().cpu().numpy(), prm)
    return torch.as_tensor(mass_fraction(y, prm), dtype=torch.float64)


def gas_density(prm, T_amb=None):
    """Eq. 24 for the ambient nitrogen at (T_amb, p)."""
    T = prm["T_amb"] if T_amb is None else T_amb
    if prm["eq_model"] == 0:
        Z = 1.0
    elif isinstance(T, torch.Tensor) and T.requires_grad:
        Z = _PRGasZ.apply(T, _prm_float(prm))
    else:
        Tf = float(T.detach()) if isinstance(T, torch.Tensor) else float(T)
        Z = float(pr_Z_pure_gas(Tf, prm["p"], prm))
    return prm["p"] * prm["M_G"] / (Z * R_GAS * T)
