"""Pins of the oracle's flux-limited advection (Section 2.1, eq. 3)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import vof as V
from oracle import thermo as th


def _prm(n=(12, 10, 8), **kw):
    prm, _ = W.config("C1", **kw)
    return W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], x0=None))


def _divfree_dyadic(shape, seed):
    """Face velocities from an integer stream function (x-y plane) scaled by
    2^-12: every difference and sum is exact, so the discrete divergence is
    exactly zero and boundary normal velocities vanish."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    psi = rng.integers(-8, 9, (nx + 1, ny + 1, nz)).astype(np.float64)
    psi[0, :, :] = 0.0
    psi[-1, :, :] = 0.0
    psi[:, 0, :] = 0.0
    psi[:, -1, :] = 0.0
    s = 2.0 ** -12
    u = s * (psi[:, 1:, :] - psi[:, :-1, :])          # (nx+1, ny, nz)
    v = -s * (psi[1:, :, :] - psi[:-1, :, :])         # (nx, ny+1, nz)
    w = np.zeros((nx, ny, nz + 1))
    return [torch.tensor(a) for a in (u, v, w)]


def test_uniform_field_unchanged_exactly():
    prm = _prm()
    shape = (prm["nx"], prm["ny"], prm["nz"])
    u, v, w = _divfree_dyadic(shape, 1)
    div = (u[1:] - u[:-1]) + (v[:, 1:] - v[:, :-1]) + (w[:, :, 1:] - w[:, :, :-1])
    assert float(div.abs().max()) == 0.0
    a = torch.full(shape, 0.375, dtype=torch.float64)
    om = torch.full(shape, 0.25, dtype=torch.float64)
    T = torch.full(shape, 500.0, dtype=torch.float64)
    c = torch.full(shape, 0.125, dtype=torch.float64)
    rho_G = th.gas_density(prm)
    a2, c2, T2, BL, Bv = V.advect(a, om, T, c, u, v, w, prm, rho_G)
    assert torch.equal(a2, a) and torch.equal(T2, T)
    assert float(BL) == 0.0 and float(Bv) == 0.0


def test_sum_conserved_without_boundary_flux():
    prm = _prm()
    shape = (prm["nx"], prm["ny"], prm["nz"])
    u, v, w = _divfree_dyadic(shape, 2)
    rng = np.random.default_rng(0)
    a = torch.tensor(rng.uniform(0, 1, shape))
    om = torch.tensor(rng.uniform(0, 0.3, shape))
    c = torch.tensor(rng.uniform(0, 0.1, shape))
    rho_G = th.gas_density(prm)
    a2, c2, T2, BL, Bv = V.advect(a, om, a.clone(), c, u, v, w, prm, rho_G)
    assert float(a2.sum()) == pytest.approx(float(a.sum()), rel=1e-14)
    assert float(c2.sum()) == pytest.approx(float(c.sum()), rel=1e-14)
    assert not torch.equal(a2, a)


def test_limiter_reduces_to_central_on_linear_profile():
    """van Leer psi(1) = 1: on a linear profile away from the boundary the
    face value is the midpoint, so alpha' = alpha - dt U dalpha/dx exactly
    (to rounding) in the cells whose faces all see r = 1."""
    prm = _prm(n=(16, 3, 3))
    nx, ny, nz = 16, 3, 3
    h, dt = prm["h"], prm["dt"]
    x = torch.arange(nx, dtype=torch.float64)
    a = (0.2 + 0.03 * x)[:, None, None].expand(nx, ny, nz).contiguous()
    U = 0.05
    u = torch.full((nx + 1, ny, nz), U, dtype=torch.float64)
    v = torch.zeros(nx, ny + 1, nz, dtype=torch.float64)
    w = torch.zeros(nx, ny, nz + 1, dtype=torch.float64)
    rho_G = th.gas_density(prm)
    a2, *_ = V.advect(a, torch.zeros_like(a), a.clone(), torch.zeros_like(a), u, v, w, prm, rho_G)
    expect = a - dt * U * 0.03 / h
    np.testing.assert_allclose(a2[3:-2].numpy(), expect[3:-2].numpy(), rtol=1e-13)


@pytest.mark.parametrize("cfl", [0.1, 0.3, 0.5])
def test_one_dimensional_tvd_bounds(cfl):
    """1D transport at CFL <= 0.5 creates no new extrema (van Leer, psi <= 2)."""
    nx = 64
    prm = _prm(n=(nx, 1, 1))
    h, dt = prm["h"], prm["dt"]
    U = cfl * h / dt
    x = (torch.arange(nx, dtype=torch.float64) + 0.5)
    a = 0.5 * (1 - torch.tanh((x - 20) / 1.5)) * 0.5 * (1 + torch.tanh((x - 8) / 1.5))
    a = a[:, None, None].contiguous()
    u = torch.full((nx + 1, 1, 1), U, dtype=torch.float64)
    v = torch.zeros(nx, 2, 1, dtype=torch.float64)
    w = torch.zeros(nx, 1, 2, dtype=torch.float64)
    rho_G = th.gas_density(prm)
    lo, hi = float(a.min()), float(a.max())
    for _ in range(60):
        a, *_ = V.advect(a, torch.zeros_like(a), a.clone(), torch.zeros_like(a), u, v, w, prm, rho_G)
        assert float(a.max()) <= hi + 1e-15 and float(a.min()) >= lo - 1e-15


def test_boundary_tally_closes_liquid_budget():
    """Outflow through open faces: h^3 rho_L (sum alpha - sum alpha') = B_L."""
    prm = _prm(n=(8, 8, 10))
    shape = (8, 8, 10)
    rng = np.random.default_rng(4)
    a = torch.tensor(rng.uniform(0, 1, shape))
    u = torch.zeros(9, 8, 10, dtype=torch.float64)
    v = torch.zeros(8, 9, 10, dtype=torch.float64)
    w = torch.tensor(rng.uniform(-0.5, 0.5, (8, 8, 11)))
    rho_G = th.gas_density(prm)
    a2, c2, T2, BL, Bv = V.advect(a, torch.zeros_like(a), a.clone(), torch.zeros_like(a), u, v, w, prm, rho_G)
    h = prm["h"]
    assert float(BL) == pytest.approx(prm["rho_L"] * h ** 3 * float(a.sum() - a2.sum()), rel=1e-10)
    # inflow faces carry alpha = 0: only outflow removes liquid
    out = (w[:, :, -1].clamp(min=0) * a[:, :, -1]).sum() + ((-w[:, :, 0]).clamp(min=0) * a[:, :, 0]).sum()
    assert float(BL) == pytest.approx(prm["rho_L"] * h * h * prm["dt"] * float(out), rel=1e-12)
