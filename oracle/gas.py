"""Variable-density gas (Section 2.2, eq. 7; Section 2.5, eq. 24).

Test infrastructure: the CPU oracle only.

With gas_density = 1 the gas density is a field instead of the ambient
constant:
* eq. 24 for the local fuel/N2 mixture, rho_G = p M / (Z R T), with the
  vapour mole fraction y from its mass fraction omega and M = y M_v +
  (1 - y) M_G; Z = 1 in the ideal model, else the largest root of the
  Peng-Robinson cubic of the mixture (the mixing rules and k_ij of the
  equilibrium, thermo.pr_ln_phi_fuel).
* State reading: the vapour content c (mass per cell volume) and T are the
  primary variables; omega and rho_G follow from them through the vapour
  mass per unit gas volume q = c/theta: omega solves rho_G(T, omega) omega
  = q.  rho_G omega grows with omega (heavier molecules, and a smaller Z as
  the fuel share rises), so the root is unique; it lies between
  q/rho_G(T, 1) and q/rho_G(T, 0) and is found here by bisection.  q <= 0
  (round-off undershoot) maps to omega = q/rho_G(T, 0), rho_G = rho_G(T, 0).
* Compressibility, the (1 - alpha)/rho_G D rho_G/Dt term of eq. 7: the step
  splits advection from diffusion and sources, so the material change of a
  gas parcel's density over the step is its change from the advected state
  (T', omega') to the end of the step (T^{n+1}, omega^{n+1}):
      (1/rho_G) D rho_G/Dt = ln(rho_G^{n+1}/rho_G')/dt,
  evaluated as log1p((rho_G^{n+1} - rho_G')/rho_G')/dt.
* The liquid density is constant, so the alpha source's D rho_L/Dt term
  (eqs. 2 and 4) stays zero.
"""
from __future__ import annotations

import numpy as np
import torch

from . import thermo

R_GAS = thermo.R_GAS


def mole_fraction(omega, prm):
    """Vapour mass fraction -> mole fraction in the fuel/N2 gas."""
    a = omega / prm["M_v"]
    return a / (a + (1.0 - omega) / prm["M_G"])


def compressibility(T, y, prm):
    """Z of the gas at (T, p) and vapour mole fraction y (numpy arrays)."""
    T = np.asarray(T, dtype=np.float64)
    if prm["eq_model"] == 0:
        return np.ones_like(T)
    _, Z = thermo.pr_ln_phi_fuel(T, prm["p"], np.asarray(y, dtype=np.float64), prm)
    return Z


def density_np(T, omega, prm):
    """eq. 24 for the local mixture (numpy in, numpy out)."""
    T = np.asarray(T, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64) * np.ones_like(T)
    y = mole_fraction(omega, prm)
    M = y * prm["M_v"] + (1.0 - y) * prm["M_G"]
    Z = compressibility(T, y, prm)
    return prm["p"] * M / (Z * R_GAS * T)


def density(T, omega, prm):
    """eq. 24 per cell (torch in, torch out)."""
    r = density_np(T.detach().cpu().numpy(), omega.detach().cpu().numpy(), prm)
    return torch.as_tensor(r, dtype=torch.float64)


def invert_np(T, q, prm, iters=200):
    """(omega, rho_G) with rho_G(T, omega) omega = q, by bisection."""
    T = np.asarray(T, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64) * np.ones_like(T)
    r0 = density_np(T, 0.0, prm)
    pos = q > 0.0
    lo = np.where(pos, q / density_np(T, 1.0, prm), 0.0)
    hi = np.where(pos, np.minimum(q / r0, 1.0), 0.0)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.all((mid == lo) | (mid == hi) | ~pos):   # no double left between the ends
            break
        f = density_np(T, mid, prm) * mid - q
        up = f > 0.0
        hi = np.where(pos & up, mid, hi)
        lo = np.where(pos & ~up, mid, lo)
    om = np.where(pos, 0.5 * (lo + hi), q / r0)
    rho = np.where(pos, density_np(T, om, prm), r0)
    return om, rho


def invert(T, q, prm):
    """(omega, rho_G) per cell from T and q (torch in, torch out)."""
    om, rho = invert_np(T.detach().cpu().numpy(), q.detach().cpu().numpy(), prm)
    return torch.as_tensor(om, dtype=torch.float64), torch.as_tensor(rho, dtype=torch.float64)


def compressibility_source(ab, rho_new, rho_adv, dt):
    """(1 - alpha) (1/rho_G) D rho_G/Dt per cell over the step."""
    return (1.0 - ab) * torch.log1p((rho_new - rho_adv) / rho_adv) / dt
