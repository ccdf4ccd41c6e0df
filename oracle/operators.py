"""Implicit diffusion and pressure systems, and their Jacobi PCG solve.

Test infrastructure: the CPU oracle only.

Every system of the step has the finite-volume form (cell c, faces f)
    m_c x_c + sum_f K_f (x_c - x_nb(f)) = b_c,
with x_nb = 0 across a Dirichlet boundary face (its boundary value goes to
b) and K_f = 0 across a zero-gradient boundary face.  The operator is
symmetric, and positive definite whenever some K_b > 0 or m > 0.  It is
stored here as face-coefficient arrays (one per axis, n+1 faces along the
axis) and a cell array m, and applied by differences of shifted arrays.

Systems (implicit Euler, Section 3.1; face values are arithmetic means of
the cell values -- the reading for the unstated face interpolation):
* energy, eq. 8:  m = rho cp / dt, K_f = k_f/h^2, Dirichlet K_b = 2 k_G/h^2,
  b = m T' - mdot dh_ev + K_b T_amb.  (beta Dp/Dt = 0 at constant p; the
  sum of j_d,i cp,i grad T vanishes with one gas cp since sum j_d,i = 0.)
* species, eq. 9 in the conservative form for c = rho_G theta omega:
  m = rho_G theta/dt, K_f = rho_G D theta_f/h^2, Dirichlet K_b = 2 rho_G D/h^2
  (omega_b = 0), b = c'/dt + mdot.
* pressure, eq. 7 with the projection of eq. 30:
  K_f = (dt/h^2) (1/rho)_f with (1/rho)_f the mean of the two cells' 1/rho,
  p_rgh = 0 faces K_b = 2 dt/(rho_c h^2), m = 0,
  b = mdot (1/rho_G - 1/rho_L) - (1/h) sum_f sigma_f u*_f.
"""
from __future__ import annotations

import torch

WALL, INLET, OPEN, FARFIELD = 0, 1, 2, 3


def box_faces(prm):
    """Boundary kind of the six box faces, {(axis, side): kind}; side 0 = low.

    Mapping of the paper's cylinder boundaries onto a box: z- is the inlet,
    z+ the outlet, the four lateral faces the outer wall (boundary-condition
    table); 'farfield' makes every face open with ambient Dirichlet values.
    """
    mode = prm["bc_mode"]
    kinds = {}
    for axis in range(3):
        for side in range(2):
            if mode == 2:
                kinds[(axis, side)] = FARFIELD
            elif axis < 2:
                kinds[(axis, side)] = WALL
            elif side == 1:
                kinds[(axis, side)] = OPEN
            else:
                kinds[(axis, side)] = INLET if mode == 1 else OPEN
    return kinds


def scalar_dirichlet(kind, uface, side):
    """Boolean mask over a boundary face plane: does the scalar (T, omega)
    take its ambient value there?  Open faces are 'inletOutlet': fixed value
    where the face velocity points into the box, zero gradient otherwise."""
    if kind == WALL:
        return torch.zeros_like(uface, dtype=torch.bool)
    if kind in (INLET, FARFIELD):
        return torch.ones_like(uface, dtype=torch.bool)
    return uface > 0 if side == 0 else uface < 0


def _mv(axis, t):
    return torch.movedim(t, axis, 0)


def face_mean(q, axis):
    """Arithmetic mean of q over the interior faces along axis (n-1 planes)."""
    a = _mv(axis, q)
    return torch.movedim(0.5 * (a[:-1] + a[1:]), 0, axis)


class Operator:
    def __init__(self, m, K):
        self.m = m            # (nx,ny,nz) or None
        self.K = K            # [Kx (nx+1,ny,nz), Ky, Kz]

    def apply(self, x):
        y = torch.zeros_like(x) if self.m is None else self.m * x
        for axis in range(3):
            Ka = _mv(axis, self.K[axis])
            xa = _mv(axis, x)
            zero = torch.zeros_like(xa[:1])
            x_lo = torch.cat([zero, xa[:-1]], dim=0)
            x_hi = torch.cat([xa[1:], zero], dim=0)
            y = y + torch.movedim(Ka[:-1] * (xa - x_lo) + Ka[1:] * (xa - x_hi), 0, axis)
        return y

    def diagonal(self):
        d = torch.zeros_like(self.K[0][:-1]) if self.m is None else self.m.clone()
        for axis in range(3):
            Ka = _mv(axis, self.K[axis])
            d = d + torch.movedim(Ka[:-1] + Ka[1:], 0, axis)
        return d


def pcg(op, b, x0, tol, maxit):
    """Jacobi-preconditioned conjugate gradients.  Stops when the updated
    residual satisfies ||r||_2 <= tol ||b||_2.  Returns (x, iters, rel_res,
    converged)."""
    bnorm = torch.linalg.vector_norm(b)
    if float(bnorm) == 0.0:
        return torch.zeros_like(b), 0, 0.0, True
    x = x0.clone()
    r = b - op.apply(x)
    res = float(torch.linalg.vector_norm(r) / bnorm)
    if res <= tol:
        return x, 0, res, True
    dinv = 1.0 / op.diagonal()
    z = dinv * r
    p = z.clone()
    rz = torch.dot(r.ravel(), z.ravel())
    for it in range(1, maxit + 1):
        q = op.apply(p)
        a = rz / torch.dot(p.ravel(), q.ravel())
        x = x + a * p
        r = r - a * q
        res = float(torch.linalg.vector_norm(r) / bnorm)
        if res <= tol:
            return x, it, res, True
        z = dinv * r
        rz_new = torch.dot(r.ravel(), z.ravel())
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, res, False


def _boundary_planes(K, axis, side):
    a = _mv(axis, K)
    return a[0] if side == 0 else a[-1]


def _set_plane(K, axis, side, val):
    a = _mv(axis, K).clone()
    if side == 0:
        a[0] = val
    else:
        a[-1] = val
    return torch.movedim(a, 0, axis)


def _interior(K, axis, val):
    a = _mv(axis, K).clone()
    a[1:-1] = _mv(axis, val)
    return torch.movedim(a, 0, axis)


def _face_shape(shape, axis):
    s = list(shape)
    s[axis] += 1
    return s


def _cell_plane(q, axis, side):
    a = _mv(axis, q)
    return a[0] if side == 0 else a[-1]


def scalar_system(m, q_cell, scale, Kb, ambient, uvw, prm):
    """Face coefficients for a diffusion system with interior K_f = scale *
    mean(q) and ambient Dirichlet faces K_b (inletOutlet on open faces).
    Returns (Operator, boundary rhs contribution)."""
    shape = m.shape
    kinds = box_faces(prm)
    K = []
    rhs_b = torch.zeros(shape, dtype=torch.float64)
    for axis in range(3):
        Ka = torch.zeros(_face_shape(shape, axis), dtype=torch.float64)
        Ka = _interior(Ka, axis, scale * face_mean(q_cell, axis))
        for side in range(2):
            uface = _boundary_planes(uvw[axis], axis, side)
            mask = scalar_dirichlet(kinds[(axis, side)], uface, side)
            val = torch.where(mask, Kb * torch.ones_like(uface), torch.zeros_like(uface))
            Ka = _set_plane(Ka, axis, side, val)
            contrib = torch.zeros(shape, dtype=torch.float64)
            contrib = _set_plane_cells(contrib, axis, side, val * ambient)
            rhs_b = rhs_b + contrib
        K.append(Ka)
    return Operator(m, K), rhs_b


def _set_plane_cells(c, axis, side, val):
    a = _mv(axis, c).clone()
    if side == 0:
        a[0] = a[0] + val
    else:
        a[-1] = a[-1] + val
    return torch.movedim(a, 0, axis)


def pressure_operator(beta, prm):
    """Pressure operator from the cell field beta = 1/rho."""
    dt, h = prm["dt"], prm["h"]
    s = dt / (h * h)
    kinds = box_faces(prm)
    K = []
    for axis in range(3):
        Ka = torch.zeros(_face_shape(beta.shape, axis), dtype=torch.float64)
        Ka = _interior(Ka, axis, s * face_mean(beta, axis))
        for side in range(2):
            if kinds[(axis, side)] in (OPEN, FARFIELD):
                Ka = _set_plane(Ka, axis, side, 2.0 * s * _cell_plane(beta, axis, side))
        K.append(Ka)
    return Operator(None, K)


def divergence(u, v, w, h):
    """(1/h) sum_f sigma_f u_f per cell."""
    return ((u[1:] - u[:-1]) + (v[:, 1:] - v[:, :-1]) + (w[:, :, 1:] - w[:, :, :-1])) / h
