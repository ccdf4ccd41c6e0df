"""Pins of the oracle's implicit operators and PCG (implicit Euler of
eqs. 7-9): manufactured solutions at second order, brute-force dense
solves, symmetry/definiteness, exact decay of discrete Fourier modes."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O
from oracle import step as S
from oracle import thermo as th


def _grid(n, mode=W.BC_NATURAL, L=4e-3, **kw):
    prm, _ = W.config("C1", bc_mode=mode, **kw)
    prm = W.finalize(dict(prm, nx=n, ny=n, nz=n, h=L / n, x0=None))
    return prm


def _centres(prm):
    h = prm["h"]
    ax = [(torch.arange(prm[k], dtype=torch.float64) + 0.5) * h for k in ("nx", "ny", "nz")]
    return torch.meshgrid(*ax, indexing="ij")


def _dense(op, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for j in range(n):
        e = torch.zeros(n, dtype=torch.float64)
        e[j] = 1.0
        A[:, j] = op.apply(e.reshape(shape)).ravel().numpy()
    return A


def _systems(prm, seed=0):
    """The three operators of a step on a random droplet state at 8^3."""
    f = W.random_fields(prm, seed)
    st = S.to_state(f, prm)
    rho_G = th.gas_density(prm)
    ab, rho, cp, k, theta = S.properties(st["alpha"], prm, rho_G)
    U = [st["u"], st["v"], st["w"]]
    h, dt = prm["h"], prm["dt"]
    opT, rbT = O.scalar_system(rho * cp / dt, k, 1 / h ** 2, 2 * prm["k_G"] / h ** 2, prm["T_amb"], U, prm)
    opS, _ = O.scalar_system(rho_G * theta / dt, theta, rho_G * prm["D_v"] / h ** 2,
                             2 * rho_G * prm["D_v"] / h ** 2, 0.0, U, prm)
    opP = O.pressure_operator(1.0 / rho, prm)
    return dict(T=opT, omega=opS, p=opP)


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_dense_solve_8cubed(mode):
    """PCG agrees with numpy.linalg.solve on the assembled 8^3 matrices."""
    prm = _grid(8, mode)
    rng = np.random.default_rng(3)
    for name, op in _systems(prm).items():
        shape = (8, 8, 8)
        A = _dense(op, shape)
        b = rng.standard_normal(512)
        x_ref = np.linalg.solve(A, b)
        x, it, res, ok = O.pcg(op, torch.tensor(b).reshape(shape), torch.zeros(shape, dtype=torch.float64),
                               1e-14, 5000)
        assert ok, name
        err = np.linalg.norm(x.ravel().numpy() - x_ref) / np.linalg.norm(x_ref)
        assert err < 1e-12, (name, err)
        # symmetric positive definite
        assert np.max(np.abs(A - A.T)) <= 1e-14 * np.max(np.abs(A)), name
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0, name
        # matrix diagonal equals the operator's diagonal() used by Jacobi
        assert np.allclose(np.diag(A), op.diagonal().ravel().numpy(), rtol=1e-15, atol=0)


def test_pressure_manufactured_solution_second_order():
    """Natural boundaries: p_rgh = 0 on z faces, zero flux on x/y walls.
    p = cos(pi x/L) cos(pi y/L) sin(pi z/L) with a smooth 1/rho field; A p_h
    = -dt div(beta grad p) at cell centres; error falls ~4x per halving."""
    errs = []
    for n in (16, 32, 64):
        prm = _grid(n)
        L = n * prm["h"]
        X, Y, Z = _centres(prm)
        k = math.pi / L
        beta = 1.0 + 0.5 * torch.sin(k * X) * torch.sin(k * Y) * torch.cos(k * Z) ** 2 + 0.3 * torch.cos(k * Z)
        # analytic beta gradient
        bx = 0.5 * k * torch.cos(k * X) * torch.sin(k * Y) * torch.cos(k * Z) ** 2
        by = 0.5 * k * torch.sin(k * X) * torch.cos(k * Y) * torch.cos(k * Z) ** 2
        bz = -0.5 * k * torch.sin(k * X) * torch.sin(k * Y) * torch.sin(2 * k * Z) - 0.3 * k * torch.sin(k * Z)
        p = torch.cos(k * X) * torch.cos(k * Y) * torch.sin(k * Z)
        px = -k * torch.sin(k * X) * torch.cos(k * Y) * torch.sin(k * Z)
        py = -k * torch.cos(k * X) * torch.sin(k * Y) * torch.sin(k * Z)
        pz = k * torch.cos(k * X) * torch.cos(k * Y) * torch.cos(k * Z)
        lap = -3 * k * k * p
        f = -prm["dt"] * (beta * lap + bx * px + by * py + bz * pz)
        op = O.pressure_operator(beta, prm)
        x, it, res, ok = O.pcg(op, f, torch.zeros_like(f), 1e-13, 20000)
        assert ok
        errs.append(float((x - p).abs().max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8, errs


def test_species_operator_fourier_mode_decay_exact():
    """Farfield, alpha = 0: m = rho_G/dt, K = rho_G D/h^2, Dirichlet faces 2K.
    prod_a sin(k_a pi (i+1/2)/N) is an exact eigenvector: one implicit step
    scales it by 1/(1 + dt D sum_a (4/h^2) sin^2(k_a pi/(2N)))."""
    n = 12
    prm = _grid(n, W.BC_FARFIELD)
    h, dt, D = prm["h"], prm["dt"], prm["D_v"]
    rho_G = th.gas_density(prm)
    theta = torch.ones(n, n, n, dtype=torch.float64)
    U = [torch.zeros(n + 1, n, n), torch.zeros(n, n + 1, n), torch.zeros(n, n, n + 1)]
    U = [u.double() for u in U]
    op, rb = O.scalar_system(rho_G * theta / dt, theta, rho_G * D / h ** 2, 2 * rho_G * D / h ** 2, 0.0, U, prm)
    assert float(rb.abs().max()) == 0.0
    i = torch.arange(n, dtype=torch.float64) + 0.5
    for kk in [(1, 1, 1), (2, 3, 1), (5, 1, 4)]:
        mode = (torch.sin(kk[0] * math.pi * i / n)[:, None, None] * torch.sin(kk[1] * math.pi * i / n)[None, :, None]
                * torch.sin(kk[2] * math.pi * i / n)[None, None, :])
        c_prime = rho_G * mode
        om, it, res, ok = O.pcg(op, c_prime / dt, mode, 1e-15, 1000)
        factor = 1.0 / (1.0 + dt * D * sum(4.0 / h ** 2 * math.sin(k_ * math.pi / (2 * n)) ** 2 for k_ in kk))
        assert float((om - factor * mode).abs().max()) < 1e-13


def test_energy_wall_cosine_mode_decay_exact():
    """Zero-gradient walls (natural mode, x and y): cos(k pi (i+1/2)/N) along x
    with uniform z-profile and u = 0 (open z faces then zero-gradient for T):
    exact factor 1/(1 + dt (k/(rho cp)) (4/h^2) sin^2(k pi/(2N)))."""
    n = 10
    prm = _grid(n, W.BC_NATURAL)
    h, dt = prm["h"], prm["dt"]
    alpha = torch.zeros(n, n, n, dtype=torch.float64)
    rho_G = th.gas_density(prm)
    ab, rho, cp, k, theta = S.properties(alpha, prm, rho_G)
    U = [torch.zeros(n + 1, n, n, dtype=torch.float64), torch.zeros(n, n + 1, n, dtype=torch.float64),
         torch.zeros(n, n, n + 1, dtype=torch.float64)]
    m = rho * cp / dt
    op, rb = O.scalar_system(m, k, 1 / h ** 2, 2 * prm["k_G"] / h ** 2, prm["T_amb"], U, prm)
    i = torch.arange(n, dtype=torch.float64) + 0.5
    for kx in (1, 3):
        mode = torch.cos(kx * math.pi * i / n)[:, None, None].expand(n, n, n).clone()
        T, it, res, ok = O.pcg(op, m * mode + rb, mode, 1e-15, 1000)
        lam = prm["k_G"] * 4.0 / h ** 2 * math.sin(kx * math.pi / (2 * n)) ** 2
        factor = 1.0 / (1.0 + dt * lam / (rho_G * prm["cp_G"]))
        assert float((T - factor * mode).abs().max()) < 1e-13


def test_energy_sink_without_conduction_is_exact():
    """k = 0, u = 0: Delta T = -dt mdot dh_ev/(rho cp) exactly (eq. 8)."""
    n = 6
    prm = _grid(n, W.BC_NATURAL, k_L=0.0, k_G=0.0)
    rng = np.random.default_rng(1)
    alpha = torch.tensor(rng.uniform(0, 1, (n, n, n)))
    Tp = torch.tensor(rng.uniform(300, 700, (n, n, n)))
    mdot = torch.tensor(rng.uniform(-50, 50, (n, n, n)))
    rho_G = th.gas_density(prm)
    ab, rho, cp, k, theta = S.properties(alpha, prm, rho_G)
    U = [torch.zeros(n + 1, n, n, dtype=torch.float64), torch.zeros(n, n + 1, n, dtype=torch.float64),
         torch.zeros(n, n, n + 1, dtype=torch.float64)]
    m = rho * cp / prm["dt"]
    op, rb = O.scalar_system(m, k, 1 / prm["h"] ** 2, 0.0, prm["T_amb"], U, prm)
    T, it, res, ok = O.pcg(op, m * Tp - mdot * prm["dh_ev"] + rb, Tp, 1e-15, 100)
    expect = Tp - prm["dt"] * mdot * prm["dh_ev"] / (rho * cp)
    assert float(((T - expect) / expect).abs().max()) < 1e-14


def test_pcg_zero_rhs_and_warm_start():
    prm = _grid(8)
    op = _systems(prm)["p"]
    z = torch.zeros(8, 8, 8, dtype=torch.float64)
    x, it, res, ok = O.pcg(op, z, torch.ones_like(z), 1e-10, 100)
    assert it == 0 and float(x.abs().max()) == 0.0
    b = torch.ones_like(z)
    x, it, res, ok = O.pcg(op, b, z, 1e-12, 1000)
    x2, it2, res2, ok2 = O.pcg(op, b, x, 1e-10, 1000)
    assert it2 == 0
