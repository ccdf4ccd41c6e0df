"""Liquid-fraction source and flux-limited advection (paper Section 2.1).

Test infrastructure: the CPU oracle only.

The paper splits eq. 2 into the evaporation source (eq. 4) and pure
advection (eq. 3), with a geometric (isoAdvector) or a flux-limited (MULES)
advection scheme.  The reading taken here:
* source first: alpha1 = alpha - dt mdot / rho_L (D rho_L/Dt = 0 for a
  constant liquid density);
* then one explicit, unsplit, conservative advection step with face values
  from a TVD van Leer limiter, donor cell by the sign of the face velocity:
      r = (phi_C - phi_U)/(phi_D - phi_C),  psi = (r + |r|)/(1 + |r|),
      phi_f = phi_C + psi (phi_D - phi_C)/2   (phi_f = phi_C if phi_D = phi_C);
  where the far-upwind cell U lies outside the box, U := C (first order);
  at boundary faces the face value is the donor cell value on outflow and the
  ambient value on inflow (alpha 0, omega 0, T_amb);
* the same face interpolation serves alpha, the vapour mass fraction omega
  and T.  The vapour partial density c = rho_G theta omega moves with the gas
  volume flux (1 - alpha_f) u_f; T is advected in non-conservative form.
No clipping of alpha is applied (the update stays exactly conservative).
"""
from __future__ import annotations

import torch


def limited_face_values(phi, uf, ambient):
    """Face values along axis 0 for cell field phi (n, ...) and face
    velocities uf (n+1, ...)."""
    n = phi.shape[0]
    out = torch.zeros_like(uf)
    # interior faces f = 1..n-1 between L = f-1 and R = f
    L = phi[:-1]
    R = phi[1:]
    Lm = torch.cat([phi[:1], phi[:-2]], dim=0)      # cell f-2 (or L itself at f = 1)
    Rp = torch.cat([phi[2:], phi[-1:]], dim=0)      # cell f+1 (or R itself at f = n-1)
    ui = uf[1:-1]
    pos = ui > 0
    C = torch.where(pos, L, R)
    D = torch.where(pos, R, L)
    U = torch.where(pos, Lm, Rp)
    denom = D - C
    same = denom == 0
    r = (C - U) / torch.where(same, torch.ones_like(denom), denom)
    psi = (r + r.abs()) / (1.0 + r.abs())
    face = torch.where(same, C, C + 0.5 * psi * denom)
    out[1:-1] = torch.where(ui == 0, torch.zeros_like(face), face)
    # boundary faces: inflow carries the ambient value, outflow the donor value
    amb = torch.full_like(uf[0], ambient)
    out[0] = torch.where(uf[0] > 0, amb, phi[0])
    out[n] = torch.where(uf[n] < 0, amb, phi[n - 1])
    return out


def _along(axis, t):
    return torch.movedim(t, axis, 0)


def _back(axis, t):
    return torch.movedim(t, 0, axis)


def advect(alpha1, omega, T, c, u, v, w, prm, rho_G, T_amb=None, advect_T=True, U_liq=None):
    """One advection step.  Returns alpha', c', T' and the boundary outflow
    tallies (kg of liquid, kg of vapour leaving the box during dt).
    U_liq (optional): face velocities that move the liquid marker; the
    vapour and temperature move with (u, v, w)."""
    dt, h = prm["dt"], prm["h"]
    Ta = prm["T_amb"] if T_amb is None else T_amb
    dalpha = torch.zeros_like(alpha1)
    dc = torch.zeros_like(alpha1)
    dT = torch.zeros_like(alpha1)
    B_L = torch.zeros((), dtype=torch.float64)
    B_v = torch.zeros((), dtype=torch.float64)
    for axis, uf in enumerate((u, v, w)):
        a_ = _along(axis, alpha1)
        o_ = _along(axis, omega)
        T_ = _along(axis, T)
        uf_ = _along(axis, uf)
        af = limited_face_values(a_, uf_, 0.0)
        of = limited_face_values(o_, uf_, 0.0)
        if U_liq is None:
            F = uf_ * af                              # liquid volume flux / area
        else:
            ul_ = _along(axis, U_liq[axis])
            F = ul_ * limited_face_values(a_, ul_, 0.0)
        G = rho_G * of * (1.0 - af) * uf_             # vapour mass flux / area
        dalpha += _back(axis, F[1:] - F[:-1])
        dc += _back(axis, G[1:] - G[:-1])
        if advect_T:
            if isinstance(Ta, torch.Tensor):
                Tf = limited_face_values(T_, uf_, 0.0)
                # inflow boundary faces carry T_amb (kept differentiable)
                Tf = Tf.clone()
                Tf[0] = torch.where(uf_[0] > 0, Ta * torch.ones_like(Tf[0]), Tf[0])
                Tf[-1] = torch.where(uf_[-1] < 0, Ta * torch.ones_like(Tf[-1]), Tf[-1])
            else:
                Tf = limited_face_values(T_, uf_, Ta)
            dT += _back(axis, uf_[1:] * (Tf[1:] - T_) - uf_[:-1] * (Tf[:-1] - T_))
        area_dt = h * h * dt
        B_L = B_L + prm["rho_L"] * area_dt * (F[-1].sum() - F[0].sum())
        B_v = B_v + area_dt * (G[-1].sum() - G[0].sum())
    alpha_new = alpha1 - (dt / h) * dalpha
    c_new = c - (dt / h) * dc
    T_new = T - (dt / h) * dT if advect_T else T
    return alpha_new, c_new, T_new, B_L, B_v
