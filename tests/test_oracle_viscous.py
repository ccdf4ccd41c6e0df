"""Pins of the oracle's implicit viscous momentum (eq. 5 / eq. 30, viscous
stress div mu (grad v + grad v^T); mu mixed by eq. 31).

* The implicit part is exact on discrete eigenmodes: with uniform mu and
  rho, a face field that is a product of sines across no-slip walls and
  cosines across open faces, held by its known box faces at the decayed
  amplitude, is returned as amplitude / (1 + dt (mu/rho) lambda) with lambda
  the sum of (4/h^2) sin^2(k pi/(2N)) over the transverse axes -- a wrong
  wall factor, a missed transverse direction or a wrong face density moves
  the amplitude.
* The transpose part obeys sum_b d_b(d_a u_b) = d_a(div u) on the MAC grid,
  so with uniform mu it equals mu d_a(D U) for any U (and vanishes for a
  discretely divergence-free U) -- a shifted index or a wrong edge fails it.
* Every component's system is symmetric positive definite (dense 4x5x6 with
  a random mu field), and PCG reaches numpy.linalg.solve.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O
from oracle import viscous as V

MODES = (W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD)


def _prm(mode, n=(6, 7, 8), **kw):
    prm, _ = W.config("C1", bc_mode=mode, **kw)
    return W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], x0=None, mu_L=4e-4, mu_G=3.5e-5))


def _div(U, h):
    u, v, w = U
    return ((u[1:] - u[:-1]) + (v[:, 1:] - v[:, :-1]) + (w[:, :, 1:] - w[:, :, :-1])) / h


def _dense(op, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for j in range(n):
        e = torch.zeros(n, dtype=torch.float64)
        e[j] = 1.0
        A[:, j] = op.apply(e.reshape(shape)).ravel().numpy()
    return A


def _mode_1d(N, lo_wall, hi_wall, k):
    """Eigenvector (cell-centred samples) and eigenvalue (unit h) of the 1-D
    second difference with no slip (ghost -x half a cell outside) or zero
    gradient at each end: sines, cosines, or quarter-wave sines."""
    n = np.arange(N) + 0.5
    if lo_wall and hi_wall:
        return np.sin(np.pi * k * n / N), 4.0 * np.sin(np.pi * k / (2 * N)) ** 2
    if not lo_wall and not hi_wall:
        return np.cos(np.pi * k * n / N), 4.0 * np.sin(np.pi * k / (2 * N)) ** 2
    assert lo_wall and not hi_wall
    return np.sin(np.pi * (k + 0.5) * n / N), 4.0 * np.sin(np.pi * (k + 0.5) / (2 * N)) ** 2


@pytest.mark.parametrize("mode", MODES)
def test_implicit_part_exact_on_eigenmodes(mode):
    prm = _prm(mode)
    n = (prm["nx"], prm["ny"], prm["nz"])
    h, dt = prm["h"], prm["dt"]
    kinds = O.box_faces(prm)
    mu0, rho0 = 3.0e-3, 5.0                        # uniform; dt mu/(rho h^2) ~ 0.4
    prm = dict(prm, mu_L=mu0, mu_G=mu0)
    alpha = torch.full(n, 0.25, dtype=torch.float64)
    rho = torch.full(n, rho0, dtype=torch.float64)
    for a in range(3):
        # uniform along a (its box faces are known values), eigenmodes across b != a
        shape = list(n)
        shape[a] += 1
        field = np.ones(shape)
        lam = 0.0
        for b in range(3):
            if b == a:
                continue
            lo = kinds[(b, 0)] in (O.WALL, O.INLET)
            hi = kinds[(b, 1)] in (O.WALL, O.INLET)
            vec, l = _mode_1d(n[b], lo, hi, 2)
            sh = [1, 1, 1]
            sh[b] = n[b]
            field = field * vec.reshape(sh)
            lam += l / h ** 2
        c = 1.0 / (1.0 + dt * mu0 / rho0 * lam)
        Us = [torch.zeros(n[0] + 1, n[1], n[2], dtype=torch.float64),
              torch.zeros(n[0], n[1] + 1, n[2], dtype=torch.float64),
              torch.zeros(n[0], n[1], n[2] + 1, dtype=torch.float64)]
        F = torch.tensor(field)
        t = torch.movedim(F, a, 0).clone()
        t[0] = c * t[0]                                # known box faces at the decayed amplitude
        t[-1] = c * t[-1]
        Us[a] = torch.movedim(t, 0, a)
        U0 = [torch.zeros_like(x) for x in Us]         # no transpose part
        out, its, ok = V.implicit_viscosity(Us, U0, alpha, rho, prm, 1e-14, O.pcg)
        assert ok and its[a] > 0
        got = torch.movedim(out[a], a, 0)[1:-1]
        want = c * torch.movedim(F, a, 0)[1:-1]
        err = float((got - want).abs().max() / want.abs().max())
        print(mode, a, c, err)
        assert err < 1e-12, (a, err)


@pytest.mark.parametrize("mode", MODES)
def test_transpose_part_is_gradient_of_divergence(mode):
    prm = _prm(mode)
    n = (prm["nx"], prm["ny"], prm["nz"])
    h = prm["h"]
    f = W.random_fields(prm, seed=9)
    U = [torch.tensor(f[k]) for k in ("u", "v", "w")]
    mu0 = 2.5e-4
    mu = torch.full(n, mu0, dtype=torch.float64)
    D = _div(U, h)
    for a in range(3):
        T = V.transpose_term(a, U, mu, prm)
        Da = torch.movedim(D, a, 0)
        want = torch.movedim(mu0 * (Da[1:] - Da[:-1]) / h, 0, a)
        err = float((T - want).abs().max() / want.abs().max())
        assert err < 1e-12, (a, err)


def test_transpose_part_vanishes_for_divergence_free_field():
    prm = _prm(W.BC_NATURAL)
    n = (prm["nx"], prm["ny"], prm["nz"])
    rng = np.random.default_rng(2)
    psi = rng.integers(-8, 9, (n[0] + 1, n[1] + 1, n[2])).astype(np.float64)
    psi[0], psi[-1], psi[:, 0], psi[:, -1] = 0.0, 0.0, 0.0, 0.0
    s = 2.0 ** -10
    U = [torch.tensor(s * (psi[:, 1:] - psi[:, :-1])), torch.tensor(-s * (psi[1:] - psi[:-1])),
         torch.full((n[0], n[1], n[2] + 1), 0.125, dtype=torch.float64)]
    assert float(_div(U, prm["h"]).abs().max()) == 0.0
    mu = torch.full(n, 1e-3, dtype=torch.float64)
    for a in range(3):
        assert float(V.transpose_term(a, U, mu, prm).abs().max()) < 1e-18


@pytest.mark.parametrize("mode", MODES)
def test_systems_spd_and_dense_solve(mode):
    prm = _prm(mode, n=(4, 5, 6))
    n = (4, 5, 6)
    rng = np.random.default_rng(5)
    alpha = torch.tensor(rng.uniform(0, 1, n))
    rho = alpha * prm["rho_L"] + (1 - alpha) * 0.5
    mu = V.viscosity(alpha, prm)
    for a in range(3):
        op, _, _ = V.face_system(a, mu, rho, prm)
        shape = tuple(op.m.shape)
        A = _dense(op, shape)
        assert np.max(np.abs(A - A.T)) <= 1e-14 * np.max(np.abs(A))
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
        b = rng.standard_normal(int(np.prod(shape)))
        x_ref = np.linalg.solve(A, b)
        x, it, res, ok = O.pcg(op, torch.tensor(b).reshape(shape), torch.zeros(shape, dtype=torch.float64),
                               1e-14, 500)
        assert ok
        assert np.linalg.norm(x.ravel().numpy() - x_ref) / np.linalg.norm(x_ref) < 1e-12


@pytest.mark.parametrize("mode", MODES)
def test_viscous_step_conserves_fuel_and_projects(mode):
    """The whole step with viscosity on a random droplet state with flow (15^3):
    the fuel balance closes to 1e-10 per step and div u = mdot (1/rho_G -
    1/rho_L) after the projection, as without viscosity; the viscous solve
    ran in every component; and the flow differs from the inviscid step's."""
    from oracle import step as S
    prm, _ = W.config("C1", bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0, viscous=1,
                      tol=1e-13, tol_phi=1e-13)
    prm = W.finalize(dict(prm, nx=15, ny=15, nz=15, x0=None))
    f = W.random_fields(prm, seed=17)
    st = S.to_state(f, prm)
    st0 = S.to_state(f, prm)
    new, d = S.step(st, prm)
    inv, _ = S.step(st0, dict(prm, viscous=0))
    rel = abs(d["fuel_mass"] - d["fuel_mass_before"] + d["B_L"] + d["B_v"]) / d["fuel_mass_before"]
    assert rel <= 1e-10 and d["converged"]
    assert min(d["iters"]["visc"]) > 0
    rec = {}
    S.step(S.to_state(f, prm), prm, record=rec)
    div = _div([new["u"], new["v"], new["w"]], prm["h"])
    src = rec["mdot"] * (1.0 / rec["rho_G"] - 1.0 / prm["rho_L"])
    scale = max(float(src.abs().max()), float(div.abs().max()))
    assert float((div - src).abs().max()) <= 1e-9 * scale
    dv = float((new["u"] - inv["u"]).abs().max()) / float(inv["u"].abs().max())
    assert dv > 1e-6
