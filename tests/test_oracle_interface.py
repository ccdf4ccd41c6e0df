"""Pins of the oracle's interface geometry and evaporation source
(Section 2.4, eqs. 15-21)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import interface as I
from oracle import thermo as th


def _planar(nx=24, ny=3, nz=3, width=1.5, x_int=None, flip=False, **kw):
    prm, _ = W.config("C1", **kw)
    h = prm["h"]
    prm = W.finalize(dict(prm, nx=nx, ny=ny, nz=nz, x0=None))
    x = (np.arange(nx) + 0.5) * h
    xi = (0.5 * nx * h if x_int is None else x_int)
    a1 = 0.5 * (1.0 - np.tanh((x - xi) / (width * h)))     # liquid at low x
    if flip:
        a1 = a1[::-1].copy()
    alpha = np.broadcast_to(a1[:, None, None], (nx, ny, nz)).copy()
    return prm, torch.tensor(alpha)


@pytest.mark.parametrize("flip,eps_gas", [(False, 0.5), (True, 0.5), (False, 1e-3), (True, 0.1)])
def test_planar_interface_by_hand(flip, eps_gas):
    """Liquid slab: normals are exactly -+x, adj is the first gas cell
    (alpha <= eps_gas) along the normal, and
    mdot_raw = rho_G D (w_sat(T_int) - w_adj)/d * |dalpha/dx|."""
    prm, alpha = _planar(flip=flip, eps_gas=eps_gas)
    nx, ny, nz, h = prm["nx"], prm["ny"], prm["nz"], prm["h"]
    rng = np.random.default_rng(0)
    T = torch.tensor(rng.uniform(290, 340, (nx, ny, nz)))
    omega = torch.tensor(rng.uniform(0, 0.05, (nx, ny, nz)))
    u = torch.zeros(nx + 1, ny, nz, dtype=torch.float64)
    v = torch.zeros(nx, ny + 1, nz, dtype=torch.float64)
    w = torch.zeros(nx, ny, nz + 1, dtype=torch.float64)
    rho_G = th.gas_density(prm)
    geo = I.geometry(alpha, prm)
    mraw = I.raw_evaporation(alpha, T, omega, u, v, w, geo, prm, rho_G)
    eps = prm["eps_int"]
    eps_gas = prm["eps_gas"]
    a = alpha[:, 0, 0].numpy()
    expect = np.zeros((nx, ny, nz))
    for i in range(nx):
        if not (eps < a[i] < 1 - eps):
            continue
        lo = a[i - 1] if i > 0 else 0.0
        hi = a[i + 1] if i < nx - 1 else 0.0
        step = 1 if hi < lo else -1            # towards the gas
        j = i + step
        while 0 <= j < nx and a[j] > eps_gas:
            j += step
        assert 0 <= j < nx and abs(j - i) <= prm["s_max"]
        d = abs(j - i) * h
        grad = abs(hi - lo) / (2 * h)
        for jj in range(ny):
            for kk in range(nz):
                ws = float(th.mass_fraction(th.equilibrium_y(float(T[i, jj, kk]), prm), prm))
                expect[i, jj, kk] = rho_G * prm["D_v"] * (ws - float(omega[j, jj, kk])) / d * grad
    # the zero ghost of alpha outside the box bends the slab at the lateral
    # walls; the middle column (j = k = 1) is exactly planar
    np.testing.assert_allclose(mraw.numpy()[:, 1, 1], expect[:, 1, 1], rtol=1e-13, atol=1e-300)
    mid = (geo["icells"][:, 1] == 1) & (geo["icells"][:, 2] == 1)
    n = geo["normal"][mid]
    assert torch.all(n[:, 1] == 0) and torch.all(n[:, 2] == 0) and torch.all(n[:, 0].abs() == 1)


def test_convective_part_of_flux_uses_adj_velocity():
    """Uniform x-velocity U through the slab: j.n gains rho_G omega_adj U n_x."""
    prm, alpha = _planar()
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    T = torch.full((nx, ny, nz), 300.0, dtype=torch.float64)
    omega = torch.full((nx, ny, nz), 0.02, dtype=torch.float64)
    Uv = 0.01
    u = torch.full((nx + 1, ny, nz), Uv, dtype=torch.float64)
    v = torch.zeros(nx, ny + 1, nz, dtype=torch.float64)
    w = torch.zeros(nx, ny, nz + 1, dtype=torch.float64)
    rho_G = th.gas_density(prm)
    geo = I.geometry(alpha, prm)
    m1 = I.raw_evaporation(alpha, T, omega, u, v, w, geo, prm, rho_G)
    m0 = I.raw_evaporation(alpha, T, omega, 0 * u, v, w, geo, prm, rho_G)
    diff = (m1 - m0)[:, 1:2, 1:2]
    sel = diff != 0
    gm = geo["gradmag"][:, 1:2, 1:2][sel]
    # liquid at low x, gas at high x: n = +x
    np.testing.assert_allclose((diff[sel] / gm).numpy(), rho_G * 0.02 * Uv, rtol=1e-12)


def test_K_tends_to_8_over_pi_for_resolved_profile():
    """With mdot_raw proportional to |grad alpha| on a well-resolved profile,
    K = sum |grad a| / sum f |grad a| -> 1/int_0^1 sqrt(a(1-a)) da = 8/pi."""
    prm, alpha = _planar(nx=400, ny=3, nz=3, width=20.0, eps_int=1e-8)
    alpha = alpha[:, 1:2, 1:2].contiguous()
    geo = I.geometry(alpha.expand(400, 3, 3).contiguous(), prm)
    mraw = (geo["gradmag"] * (geo["cls"] == I.INTERFACE))[:, 1:2, 1:2]
    mdot, K = I.redistribute(mraw, alpha)
    assert float(K) == pytest.approx(8.0 / math.pi, rel=2e-3)
    # eq. 20: the volume integral is preserved
    assert float(mdot.sum()) == pytest.approx(float(mraw.sum()), rel=1e-13)


def test_redistribution_preserves_integral_random():
    rng = np.random.default_rng(5)
    alpha = torch.tensor(rng.uniform(0, 1, (9, 7, 5)))
    mraw = torch.tensor(rng.uniform(0, 3, (9, 7, 5)))
    mdot, K = I.redistribute(mraw, alpha)
    assert float(mdot.sum()) == pytest.approx(float(mraw.sum()), rel=1e-14)
    f = torch.sqrt(alpha * (1 - alpha))
    assert torch.allclose(mdot, K * f * mraw, rtol=1e-15, atol=0)
    z, K0 = I.redistribute(torch.zeros_like(mraw), alpha)
    assert float(K0) == 0.0 and float(z.abs().max()) == 0.0


def test_classes_and_no_adj_when_march_leaves_box():
    """A liquid slab touching the x+ wall side: cells whose normal points out
    of the box get no adj and no source."""
    prm, alpha = _planar(nx=12, x_int=11.5 * 4e-3 / 32, flip=False)
    # liquid at low x reaching almost the high wall: normals point to +x
    geo = I.geometry(alpha, prm)
    a = alpha[:, 0, 0]
    assert torch.all(geo["cls"][a <= prm["eps_int"]] == I.GAS)
    assert torch.all(geo["cls"][a >= 1 - prm["eps_int"]] == I.LIQUID)
    ic = geo["icells"]
    # cells next to the high wall find no gas cell inside the box
    near = ic[:, 0] >= 11
    assert torch.all(~geo["found"][near])
