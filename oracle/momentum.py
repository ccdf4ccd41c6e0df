"""Momentum predictor and pressure projection (paper Sections 2.2 and 2.6).

Test infrastructure: the CPU oracle only.

Eq. 30 divided by rho, with mu = 0 (the configurations give no viscosity),
one predictor and one projection per step (the reading of PIMPLE here):
    u* = u^n - dt (u . grad) u + dt [ -(g . r_f) (rho_R - rho_L)/h (1/rho)_f
                                      + alpha_f (xi_R - xi_L)/h ]
    u^{n+1} = u* - dt (1/rho)_f (p_R - p_L)/h
on the staggered faces; r is measured from the droplet centre x0 (the
origin of p_rgh = p - rho g.r), xi = xi0 (D_f/2)/max(r, r_fib) is the
potential of eq. 29 (regularised at the fiber radius) and alpha_f the face
mean of alpha.  The advection term is first-order upwind with 4-point
averages of the transverse velocities and zero-gradient ghosts.  Faces on
walls and on a forced inlet keep their prescribed normal velocity; open
boundary faces keep u^n in the predictor and are corrected by the
projection with p_rgh = 0 half a cell outside.
"""
from __future__ import annotations

import torch

from .operators import box_faces, OPEN, FARFIELD, INLET, WALL


def potential(prm):
    """xi at cell centres (eq. 29)."""
    nx, ny, nz, h = prm["nx"], prm["ny"], prm["nz"], prm["h"]
    x0 = prm["x0"]
    x = (torch.arange(nx, dtype=torch.float64) + 0.5) * h - x0[0]
    y = (torch.arange(ny, dtype=torch.float64) + 0.5) * h - x0[1]
    z = (torch.arange(nz, dtype=torch.float64) + 0.5) * h - x0[2]
    r = torch.sqrt(x[:, None, None] ** 2 + y[None, :, None] ** 2 + z[None, None, :] ** 2)
    return prm["xi0"] * (0.5 * prm["Df"]) / torch.clamp(r, min=prm["r_fib"])


def _face_coords(prm, axis):
    """Coordinates (relative to x0) of the centres of the faces normal to axis."""
    n = [prm["nx"], prm["ny"], prm["nz"]]
    h = prm["h"]
    coords = []
    for b in range(3):
        if b == axis:
            c = torch.arange(n[b] + 1, dtype=torch.float64) * h
        else:
            c = (torch.arange(n[b], dtype=torch.float64) + 0.5) * h
        coords.append(c - prm["x0"][b])
    return coords


def _perm(a, b):
    c = 3 - a - b
    return (a, b, c)


def _inv(perm):
    inv = [0, 0, 0]
    for i, p in enumerate(perm):
        inv[p] = i
    return tuple(inv)


def advection_term(U, a, h):
    """(u . grad) u_a on the faces normal to axis a (zero on boundary faces),
    in the natural (x, y, z) layout of the face array."""
    Fa = U[a]
    F0 = torch.movedim(Fa, a, 0)
    uc = F0[1:-1]
    back = (F0[1:-1] - F0[:-2]) / h
    fwd = (F0[2:] - F0[1:-1]) / h
    t0 = torch.zeros_like(F0)
    t0[1:-1] = uc * torch.where(uc > 0, back, fwd)
    term = torch.movedim(t0, 0, a)
    for b in range(3):
        if b == a:
            continue
        perm = _perm(a, b)
        F = Fa.permute(perm)                    # (na+1, nb, nc)
        V = U[b].permute(perm)                  # (na, nb+1, nc)
        vbar = 0.25 * (V[:-1, :-1] + V[:-1, 1:] + V[1:, :-1] + V[1:, 1:])   # (na-1, nb, nc)
        Fi = F[1:-1]
        lo = torch.cat([Fi[:, :1], Fi[:, :-1]], dim=1)
        hi = torch.cat([Fi[:, 1:], Fi[:, -1:]], dim=1)
        d = torch.where(vbar > 0, (Fi - lo) / h, (hi - Fi) / h)
        tb = torch.zeros_like(F)
        tb[1:-1] = vbar * d
        term = term + tb.permute(_inv(perm))
    return term


def predictor(U, alpha_bar, rho, prm, xi=None):
    """u* on all faces (list of three face arrays)."""
    dt, h = prm["dt"], prm["h"]
    if xi is None:
        xi = potential(prm)
    g = prm["g"]
    beta = 1.0 / rho
    kinds = box_faces(prm)
    out = []
    for a in range(3):
        Fa = torch.movedim(U[a], a, 0)
        adv = torch.movedim(advection_term(U, a, h), a, 0)
        r_ = torch.movedim(rho, a, 0)
        b_ = torch.movedim(beta, a, 0)
        al = torch.movedim(alpha_bar, a, 0)
        xi_ = torch.movedim(xi, a, 0)
        coords = _face_coords(prm, a)
        gr = (g[0] * coords[0][:, None, None] + g[1] * coords[1][None, :, None]
              + g[2] * coords[2][None, None, :])
        gr = torch.movedim(gr.expand(U[a].shape), a, 0)
        bf = 0.5 * (b_[:-1] + b_[1:])
        force = (-gr[1:-1] * (r_[1:] - r_[:-1]) / h * bf
                 + 0.5 * (al[:-1] + al[1:]) * (xi_[1:] - xi_[:-1]) / h)
        new = Fa.clone()
        new[1:-1] = Fa[1:-1] - dt * adv[1:-1] + dt * force
        for side in range(2):
            kind = kinds[(a, side)]
            idx = 0 if side == 0 else -1
            if kind == WALL:
                new[idx] = 0.0
            elif kind == INLET:
                new[idx] = prm["w_in"]
            else:
                new[idx] = Fa[idx]
        out.append(torch.movedim(new, 0, a))
    return out


def project(Ustar, p, rho, prm):
    """u^{n+1} = u* - dt (1/rho)_f grad_h p on all faces."""
    dt, h = prm["dt"], prm["h"]
    beta = 1.0 / rho
    kinds = box_faces(prm)
    out = []
    for a in range(3):
        F = torch.movedim(Ustar[a], a, 0).clone()
        p_ = torch.movedim(p, a, 0)
        b_ = torch.movedim(beta, a, 0)
        F[1:-1] = F[1:-1] - dt * 0.5 * (b_[:-1] + b_[1:]) * (p_[1:] - p_[:-1]) / h
        if kinds[(a, 0)] in (OPEN, FARFIELD):
            F[0] = F[0] - 2.0 * dt * b_[0] * p_[0] / h
        if kinds[(a, 1)] in (OPEN, FARFIELD):
            F[-1] = F[-1] + 2.0 * dt * b_[-1] * p_[-1] / h
        out.append(torch.movedim(F, 0, a))
    return out


def solenoidal_part(U, prm, tol=None, maxit=None, solver=None):
    """Discretely divergence-free part of the face velocity field:
    U_s = U - G phi with D G phi = D U (G: face gradient, D: divergence, the
    same boundary kinds as the pressure: phi = 0 half a cell outside open
    faces, no flux through walls and inlets).  Used to move the liquid
    marker: the Stefan expansion (volume created in the gas) carries no
    liquid.  Returns (U_s, phi, iterations)."""
    from . import operators
    dt, h = prm["dt"], prm["h"]
    shape = (prm["nx"], prm["ny"], prm["nz"])
    ones = torch.full(shape, 1.0 / dt, dtype=torch.float64)     # (dt/h^2) * (1/dt) = 1/h^2 per face
    op = operators.pressure_operator(ones, prm)
    b = -operators.divergence(*U, h)
    solve = operators.pcg if solver is None else solver
    phi, it, res, ok = solve(op, b, torch.zeros(shape, dtype=torch.float64),
                             prm["tol"] if tol is None else tol,
                             prm["maxit"] if maxit is None else maxit)
    Us = project(U, phi, torch.full(shape, dt, dtype=torch.float64), prm)   # dt/rho = 1
    return Us, phi, it
