"""Implicit viscous momentum (Section 2.2, eq. 5; Section 2.6, eq. 30).

Test infrastructure: the CPU oracle only.

The viscous stress divergence div mu (grad v + grad v^T) of the momentum
equation, with mu mixed by eq. 31 (mu = alpha mu_L + (1 - alpha) mu_G on
alpha' clamped to [0, 1]), is added to the predictor on the staggered faces.
Reading (split of the term): the part div(mu grad u_a) of component a is
implicit and its transpose part sum_b d_b(mu d_a u_b) explicit from u^n, so
each component solves the symmetric positive definite system

    (rho_f/dt) u_a** - div(mu grad u_a**) = (rho_f/dt) u_a* + sum_b d_b(mu d_a u_b^n)

on its interior faces, with u* the inviscid predictor of momentum.py and
rho_f = 1/(1/rho)_f, the face density whose inverse the predictor's forces
and the projection use.  Discretisation on the MAC grid:
* along a, the flux between faces i and i+1 sits in cell i with mu of that
  cell; across b != a, the flux sits on the edge between two faces, with mu
  the mean of the four cells around the edge (of the two inside the box on a
  boundary edge);
* the box faces normal to a keep the predictor's values (walls 0, the forced
  inlet w_in, open faces u^n) and enter as known neighbours;
* tangential conditions: no slip on walls and on the forced inlet (a ghost
  -u_a half a cell outside), zero gradient on open and far-field faces;
* the transpose part uses d_a u_b on those edges and cells from the u^n
  face values, boundary faces included.
"""
from __future__ import annotations

import torch

from .operators import Operator, box_faces, WALL, INLET


def viscosity(alpha_bar, prm):
    """eq. 31 for mu on alpha clamped to [0, 1]."""
    return alpha_bar * prm["mu_L"] + (1.0 - alpha_bar) * prm["mu_G"]


def _mv(t, a):
    return torch.movedim(t, a, 0)


def _face_mean_a(q, a):
    """Mean of the two cells on either side of each interior face normal to a
    (n_a - 1 planes along a)."""
    t = _mv(q, a)
    return torch.movedim(0.5 * (t[:-1] + t[1:]), 0, a)


def _edge_mu(mu, a, b):
    """mu on the edges between neighbouring interior a-faces across b: shape
    n_a - 1 along a, n_b + 1 along b (boundary edges: mean of the two cells
    inside the box; interior edges: of the four cells around the edge)."""
    ma = _face_mean_a(mu, a)                  # interior a-faces, cells along b
    t = _mv(ma, b)
    inner = 0.5 * (t[:-1] + t[1:])
    e = torch.cat([t[:1], inner, t[-1:]], dim=0)
    return torch.movedim(e, 0, b)


def _interior_faces(F, a):
    t = _mv(F, a)
    return torch.movedim(t[1:-1], 0, a)


def face_system(a, mu, rho, prm):
    """Operator of the viscous system of component a on its interior faces and
    the coefficients of the two known box faces along a (for the right-hand
    side): (Operator, K_lo, K_hi)."""
    dt, h = prm["dt"], prm["h"]
    ih2 = 1.0 / (h * h)
    kinds = box_faces(prm)
    beta_f = _face_mean_a(1.0 / rho, a)
    m = 1.0 / (dt * beta_f)
    K = [None, None, None]
    # along a: cells between faces, mu of the cell; n_a entries (the first and
    # last couple the end unknowns with the known box faces)
    K[a] = mu * ih2
    for b in range(3):
        if b == a:
            continue
        Kb = _edge_mu(mu, a, b) * ih2
        t = _mv(Kb, b).clone()
        for side, idx in ((0, 0), (1, -1)):
            if kinds[(b, side)] in (WALL, INLET):
                t[idx] = 2.0 * t[idx]          # no slip: ghost -u half a cell outside
            else:
                t[idx] = 0.0                   # zero gradient
        K[b] = torch.movedim(t, 0, b)
    op = Operator(m, K)
    t = _mv(K[a], a)
    return op, t[0], t[-1]


def transpose_term(a, U, mu, prm):
    """sum_b d_b(mu d_a u_b) on the interior faces of component a, from the
    face velocities U (boundary faces included)."""
    h = prm["h"]
    Fa = _mv(U[a], a)
    cell_stress = _mv(mu, a) * (Fa[1:] - Fa[:-1]) / h          # mu d_a u_a in the cells
    out = (cell_stress[1:] - cell_stress[:-1]) / h              # interior faces
    out = torch.movedim(out, 0, a)
    for b in range(3):
        if b == a:
            continue
        Ub = _mv(U[b], a)                                       # along a: cells
        dau = (Ub[1:] - Ub[:-1]) / h                            # interior a-faces, b-faces
        dau = torch.movedim(dau, 0, a)
        st = _edge_mu(mu, a, b) * dau                           # on the edges
        t = _mv(st, b)
        out = out + torch.movedim((t[1:] - t[:-1]) / h, 0, b)
    return out


def implicit_viscosity(Us, U, alpha_bar, rho, prm, tol, solver):
    """u** on all faces from the inviscid predictor Us (list of 3 face arrays)
    and the start-of-step U.  Returns (new face arrays, iterations per
    component, converged)."""
    dt = prm["dt"]
    mu = viscosity(alpha_bar, prm)
    out, its, ok_all = [], [], True
    for a in range(3):
        op, K_lo, K_hi = face_system(a, mu, rho, prm)
        Fs = _mv(Us[a], a)                       # box faces normal to a: known values
        x0 = _interior_faces(Us[a], a)
        rhs = op.m * x0 + transpose_term(a, U, mu, prm)
        r = _mv(rhs, a).clone()
        r[0] = r[0] + K_lo * Fs[0]
        r[-1] = r[-1] + K_hi * Fs[-1]
        rhs = torch.movedim(r, 0, a)
        x, it, res, ok = solver(op, rhs, x0, tol, prm["maxit"])
        new = Fs.clone()
        new[1:-1] = _mv(x, a)
        out.append(torch.movedim(new, 0, a))
        its.append(it)
        ok_all = ok_all and ok
    return out, its, ok_all
