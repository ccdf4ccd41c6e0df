"""Pins of the oracle's momentum advection (oracle/momentum.py: first-order
upwind (u . grad) u on the staggered faces, Section 2.6 eq. 30 with mu = 0).

First-order upwind differences are exact on linear data, so on fields linear
in one coordinate the term has a closed form:
* along the face axis: u_x = U0 + a x on the x faces gives u_x a on every
  interior face, for flow in +x and in -x (a wrong upwind side, sign, index
  or 1/h fails it);
* along the face axis on quadratic data, u_x = U0 + c x^2: the upwind
  difference is c (2x - h) for flow in +x and c (2x + h) in -x, so this case
  fixes which side the difference takes (the linear case cannot);
* across it: u_x = b y with a uniform transverse v = V0 gives V0 b on the
  interior rows and 0 on the row at the box face the flow comes from (its
  zero-gradient ghost), for V0 of either sign; the 4-point average of v is
  V0 exactly, so a dropped or misplaced average shows as a wrong factor;
* the predictor with no gravity and no potential force moves the interior
  faces by exactly -dt times the term and leaves the faces normal to the
  other axes at rest.
"""

import pytest
import torch

import workloads as W
from oracle import momentum as M

def _prm(n=(7, 6, 5)):
    prm, _ = W.config("C1", bc_mode=W.BC_FARFIELD, g=(0.0, 0.0, 0.0), xi0=0.0)
    return W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], x0=None))

def _zeros(n):
    return [torch.zeros(n[0] + 1, n[1], n[2], dtype=torch.float64),
            torch.zeros(n[0], n[1] + 1, n[2], dtype=torch.float64),
            torch.zeros(n[0], n[1], n[2] + 1, dtype=torch.float64)]

@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("U0", [2.5, -2.5])
def test_along_axis_linear_profile(axis, U0):
    prm = _prm()
    n = (prm["nx"], prm["ny"], prm["nz"])
    h = prm["h"]
    a = 0.7 / (n[axis] * h)          # |a x| < |U0|: one flow direction everywhere
    U = _zeros(n)
    xf = torch.arange(n[axis] + 1, dtype=torch.float64) * h
    shape = [1, 1, 1]
    shape[axis] = n[axis] + 1
    U[axis] = (U0 + a * xf).reshape(shape).expand(U[axis].shape).clone()
    term = M.advection_term(U, axis, h)
    want = (U0 + a * xf) * a
    got = torch.movedim(term, axis, 0)
    inner = got[1:-1]
    ref = want[1:-1].reshape(-1, 1, 1).expand(inner.shape)
    assert torch.max(torch.abs(inner - ref)) <= 1e-13 * abs(U0 * a)
    assert torch.all(got[0] == 0) and torch.all(got[-1] == 0)   # box faces: no term
    # the other face arrays are at rest and stay so
    for b in range(3):
        if b != axis:
            assert torch.all(M.advection_term(U, b, h) == 0)

@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("U0", [4.0, -4.0])
def test_along_axis_quadratic_profile_takes_the_upwind_side(axis, U0):
    prm = _prm()
    n = (prm["nx"], prm["ny"], prm["nz"])
    h = prm["h"]
    L = n[axis] * h
    c = 1.0 / (L * L)                # |c x^2| <= 1 < |U0|: one flow direction everywhere
    U = _zeros(n)
    xf = torch.arange(n[axis] + 1, dtype=torch.float64) * h
    shape = [1, 1, 1]
    shape[axis] = n[axis] + 1
    U[axis] = (U0 + c * xf * xf).reshape(shape).expand(U[axis].shape).clone()
    got = torch.movedim(M.advection_term(U, axis, h), axis, 0)[1:-1]
    x = xf[1:-1]
    slope = c * (2.0 * x - h) if U0 > 0 else c * (2.0 * x + h)
    ref = ((U0 + c * x * x) * slope).reshape(-1, 1, 1).expand(got.shape)
    assert torch.max(torch.abs(got - ref)) <= 1e-12 * abs(U0) * c * L


@pytest.mark.parametrize("axis,across", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
@pytest.mark.parametrize("V0", [1.5, -1.5])
def test_transverse_linear_profile(axis, across, V0):
    prm = _prm()
    n = (prm["nx"], prm["ny"], prm["nz"])
    h = prm["h"]
    b = 3.0 / (n[across] * h)
    U = _zeros(n)
    yc = (torch.arange(n[across], dtype=torch.float64) + 0.5) * h   # the faces normal to axis sit at cell centres along `across`
    shape = [1, 1, 1]
    shape[across] = n[across]
    U[axis] = (b * yc).reshape(shape).expand(U[axis].shape).clone()
    U[across] = torch.full(U[across].shape, V0, dtype=torch.float64)
    t = torch.movedim(M.advection_term(U, axis, h), axis, 0)
    term = torch.movedim(t, across + 1 if across < axis else across, 1)
    inner = term[1:-1]                       # interior faces along axis; dim 1 runs along `across`
    want = torch.full(inner.shape, V0 * b, dtype=torch.float64)
    ghost_row = 0 if V0 > 0 else -1          # the row whose upwind neighbour is the ghost
    want[:, ghost_row] = 0.0
    assert torch.max(torch.abs(inner - want)) <= 1e-13 * abs(V0 * b)
    assert torch.all(term[0] == 0) and torch.all(term[-1] == 0)

def test_predictor_moves_faces_by_the_term():
    prm = _prm()
    n = (prm["nx"], prm["ny"], prm["nz"])
    h, dt = prm["h"], prm["dt"]
    U = _zeros(n)
    a = 0.5 / (n[0] * h)
    xf = torch.arange(n[0] + 1, dtype=torch.float64) * h
    U[0] = (1.0 + a * xf).reshape(-1, 1, 1).expand(U[0].shape).clone()
    rho = torch.full(n, 3.0, dtype=torch.float64)
    alpha = torch.zeros(n, dtype=torch.float64)
    Us = M.predictor(U, alpha, rho, prm)
    inner = Us[0][1:-1] - U[0][1:-1]
    ref = (-dt * (1.0 + a * xf[1:-1]) * a).reshape(-1, 1, 1).expand(inner.shape)
    assert torch.max(torch.abs(inner - ref)) <= 1e-12 * dt * a
    # far-field box faces keep u^n in the predictor (the projection corrects them)
    assert torch.equal(Us[0][0], U[0][0]) and torch.equal(Us[0][-1], U[0][-1])
    assert torch.all(Us[1] == 0) and torch.all(Us[2] == 0)
