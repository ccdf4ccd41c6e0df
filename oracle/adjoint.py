"""Derivative of the droplet volume after a run of steps (differentiation
form of the method): dV_N/d(D_v, dh_ev, T_amb) and dV_N/d(initial fields).

Test infrastructure: the CPU oracle only.

Definition.  V_N = h^3 sum(alpha^N) after N steps of step.step from the
initial fields (vapour c^0 = rho_G theta omega^0 as in step.to_state).  The
derivative is the exact derivative of the discrete step with its integer
decisions held at their forward values: interface classes and adj, donor,
upwind and limiter branches, inletOutlet switches and the clamps of the
mixing rule.  At a kink of a written expression the rule of that expression
with d|r|/dr = 0 at r = 0 applies (the van Leer limiter then has slope 1 at
r = 0).  T_amb enters through the gas density (eq. 24), the ambient boundary
temperature and the inflow face temperature; its effect through the initial
temperature field is the caller's (the gradient with respect to T^0 is
returned).

Computed by reverse-mode automatic differentiation (torch autograd) through
the oracle's own step, with two links of the chain written out:
* every linear solve x = A^-1 b is differentiated implicitly.  With A
  symmetric, the backward solves A lam = xbar and returns bbar = lam and, for
  the operator's coefficients, -lam^T (dA) x: mbar = -lam x for the mass
  term and Kbar_f = -(lam_lo - lam_hi)(x_lo - x_hi) for a face coefficient
  (zero values outside the box, so a boundary face gives -lam_c x_c);
* Peng-Robinson quantities that the oracle computes in numpy (the interface
  mole fraction and the ambient-gas Z) carry derivatives by extrapolated
  central differences (thermo._PRSaturation, thermo._PRGasZ).
"""
from __future__ import annotations

import torch

from . import operators, step as S, thermo


def _face_pairs(lam, x, axis):
    """(lam_lo - lam_hi)(x_lo - x_hi) on every face along axis, zero values
    outside the box."""
    pad = [0, 0, 0, 0, 0, 0]
    pad[2 * (2 - axis)] = 1
    pad[2 * (2 - axis) + 1] = 1
    lp = torch.nn.functional.pad(lam[None, None], pad)[0, 0]
    xp = torch.nn.functional.pad(x[None, None], pad)[0, 0]
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[axis] = slice(0, -1)
    hi[axis] = slice(1, None)
    return (lp[tuple(lo)] - lp[tuple(hi)]) * (xp[tuple(lo)] - xp[tuple(hi)])


class _LinearSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, Kx, Ky, Kz, b, x0, tol, maxit):
        op = operators.Operator(m, [Kx, Ky, Kz])
        x, it, res, ok = operators.pcg(op, b, x0, tol, maxit)
        if not ok:
            raise RuntimeError(f"linear solve did not converge ({it} iterations, residual {res:.3e})")
        ctx.save_for_backward(m if m is not None else torch.empty(0), Kx, Ky, Kz, x)
        ctx.has_m = m is not None
        ctx.tol, ctx.maxit = tol, maxit
        return x

    @staticmethod
    def backward(ctx, xbar):
        m, Kx, Ky, Kz, x = ctx.saved_tensors
        op = operators.Operator(m if ctx.has_m else None, [Kx, Ky, Kz])
        lam, it, res, ok = operators.pcg(op, xbar.contiguous(), torch.zeros_like(x), ctx.tol, ctx.maxit)
        if not ok:
            raise RuntimeError(f"adjoint solve did not converge ({it} iterations, residual {res:.3e})")
        mbar = -lam * x if ctx.has_m else None
        Kbar = [-_face_pairs(lam, x, a) for a in range(3)]
        return mbar, Kbar[0], Kbar[1], Kbar[2], lam, None, None, None


def solve(op, b, x0, tol, maxit):
    """Drop-in for operators.pcg with the implicit derivative."""
    x = _LinearSolve.apply(op.m, op.K[0], op.K[1], op.K[2], b, x0.detach(), tol, maxit)
    return x, 0, 0.0, True


def volume_and_gradients(fields, prm, steps, D_v=None, dh_ev=None, T_amb=None, dJ_dV=1.0):
    """Run `steps` oracle steps from `fields` and differentiate V_N.

    Returns dict(volume, dD_v, ddh_ev, dT_amb, grads) with grads the
    derivatives with respect to the initial alpha, T, omega, u, v, w
    (torch float64, the fields' shapes).  D_v, dh_ev, T_amb default to the
    parameter values.
    """
    D = torch.tensor(float(prm["D_v"] if D_v is None else D_v), dtype=torch.float64, requires_grad=True)
    dh = torch.tensor(float(prm["dh_ev"] if dh_ev is None else dh_ev), dtype=torch.float64, requires_grad=True)
    Ta = torch.tensor(float(prm["T_amb"] if T_amb is None else T_amb), dtype=torch.float64, requires_grad=True)
    leaves = {}
    for k in ("alpha", "T", "omega", "u", "v", "w"):
        leaves[k] = torch.as_tensor(fields[k], dtype=torch.float64).clone().requires_grad_(True)
    f = dict(leaves)
    f["p"] = torch.as_tensor(fields["p"], dtype=torch.float64).clone()
    q = dict(prm, D_v=D.item(), dh_ev=dh.item(), T_amb=Ta.item())
    rho_G = thermo.gas_density(q, Ta)
    st = S.to_state(f, q, rho_G=rho_G)
    for _ in range(steps):
        st, _d = S.step(st, q, T_amb=Ta, D_v=D, dh_ev=dh, rho_G=rho_G, solver=solve)
    V = prm["h"] ** 3 * st["alpha"].sum()
    inputs = [D, dh, Ta] + [leaves[k] for k in ("alpha", "T", "omega", "u", "v", "w")]
    g = torch.autograd.grad(V * dJ_dV, inputs, allow_unused=True)
    g = [torch.zeros_like(x) if gi is None else gi for gi, x in zip(g, inputs)]
    return dict(volume=float(V), dD_v=float(g[0]), ddh_ev=float(g[1]), dT_amb=float(g[2]),
                grads={k: g[3 + i].detach() for i, k in enumerate(("alpha", "T", "omega", "u", "v", "w"))})


def volume_after(fields, prm, steps, tol=None):
    """V_N of the plain oracle run (for finite-difference checks)."""
    st = S.to_state(fields, prm)
    for _ in range(steps):
        st, _d = S.step(st, prm, tol=tol)
    return S.droplet_volume(st, prm)
