"""Pins of the oracle's literal species form (Section 2.5, after eq. 23):
the saturation value assigned to the whole liquid, a central grad(omega) at
the adjacent gas cell, and a species equation without an mdot source.

Closed forms: the ideal equilibrium at the reference point, the exact
Fickian flux of a linear profile across a one-cell interface (where the
literal and conservative readings must agree), and the fuel-mass balance of
a form whose vapour gains no mdot.
"""
from __future__ import annotations

import pytest
import torch

import workloads as W
from oracle import interface as I
from oracle import operators as O
from oracle import step as S
from oracle import thermo as th


def _prm(n=12, **kw):
    prm, _ = W.config("C1", **kw)
    return W.finalize(dict(prm, nx=n, ny=n, nz=n, h=1e-4, x0=None))


def test_assignment_is_the_closed_form_equilibrium():
    """Ideal model at T = T_ref and p = 2 p_ref: y = 1/2, so every liquid cell
    holds omega = M_v/(M_v + M_G); gas cells keep their values; c = rho_G theta omega."""
    prm = _prm(eq_model=W.EQ_IDEAL)
    prm["p"] = 2.0 * prm["p_ref"]
    n = prm["nx"]
    g = torch.Generator().manual_seed(3)
    alpha = torch.rand((n, n, n), generator=g, dtype=torch.float64)
    omega = 0.1 * torch.rand((n, n, n), generator=g, dtype=torch.float64)
    T = torch.full((n, n, n), prm["T_ref"], dtype=torch.float64)
    rho_G = th.gas_density(prm)
    theta = torch.clamp(1.0 - alpha, min=prm["theta_min"])
    st = dict(alpha=alpha, omega=omega, T=T, c=rho_G * theta * omega)
    out = S.assign_liquid_saturation(st, prm, rho_G)
    liquid = alpha > 0.5
    ws = prm["M_v"] / (prm["M_v"] + prm["M_G"])
    assert bool(liquid.any()) and bool((~liquid).any())
    assert torch.allclose(out["omega"][liquid], torch.full_like(out["omega"][liquid], ws), rtol=1e-14, atol=0)
    assert torch.equal(out["omega"][~liquid], omega[~liquid])
    assert torch.equal(out["c"][~liquid], st["c"][~liquid])
    assert torch.allclose(out["c"][liquid], rho_G * (1.0 - alpha[liquid]) * ws, rtol=1e-14, atol=0)


def _one_cell_interface(prm, g_om, U):
    """alpha = 1 below layer i0, 0.7 on it, 0 above; omega linear in x above
    i0 with slope g_om (0 in the liquid, so only the assignment can put the
    saturation value there); uniform velocity U along x."""
    n = prm["nx"]
    i0 = 5
    h = prm["h"]
    alpha = torch.zeros((n, n, n), dtype=torch.float64)
    alpha[:i0] = 1.0
    alpha[i0] = 0.7
    ws = prm["M_v"] / (prm["M_v"] + prm["M_G"])
    xi = torch.arange(n, dtype=torch.float64)
    om1 = ws + g_om * (xi - i0) * h
    omega = om1[:, None, None].expand(n, n, n).clone()
    omega[: i0 + 1] = 0.0
    T = torch.full((n, n, n), prm["T_ref"], dtype=torch.float64)
    u = torch.full((n + 1, n, n), U, dtype=torch.float64)
    v = torch.zeros((n, n + 1, n), dtype=torch.float64)
    w = torch.zeros((n, n, n + 1), dtype=torch.float64)
    rho_G = th.gas_density(prm)
    theta = torch.clamp(1.0 - alpha, min=prm["theta_min"])
    st = dict(alpha=alpha, omega=omega, T=T, u=u, v=v, w=w, c=rho_G * theta * omega)
    return st, i0, ws, rho_G


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("U", [0.0, 0.2])
def test_linear_profile_gives_the_exact_fick_flux(form, U):
    """Across a one-cell interface with the normal along +x and adj one cell
    out, both readings give mdot_raw = (-rho_G D g + rho_G omega_adj U)/(2h)
    for omega = omega_sat + g x: the literal form through the assigned
    liquid value and the central difference at adj, the conservative form
    through (omega_sat - omega_adj)/d.  A gradient taken at the interface
    cell, a missing assignment or a lost factor 2 each fail."""
    prm = _prm(eq_model=W.EQ_IDEAL, species_form=form)
    prm["p"] = 2.0 * prm["p_ref"]
    g_om = -50.0
    st, i0, ws, rho_G = _one_cell_interface(prm, g_om, U)
    mdot, mraw, K, geo = S.evaporation_source(st, prm, rho_G)
    h, D = prm["h"], prm["D_v"]
    om_adj = ws + g_om * h
    expect = (-rho_G * D * g_om + rho_G * om_adj * U) / (2.0 * h)
    inner = mraw[i0, 1:-1, 1:-1]
    assert expect > 0
    assert torch.allclose(inner, torch.full_like(inner, expect), rtol=1e-12, atol=0)
    off = torch.ones_like(mraw, dtype=torch.bool)
    off[i0] = False
    assert float(mraw[off].abs().max()) == 0.0


def test_literal_form_differs_from_conservative_on_a_curved_profile():
    """On a droplet the two readings give different rates (the literal form is
    an alternative, not a rewrite): both positive, and not equal."""
    prm, _ = W.config("C1")
    prm = W.finalize(dict(prm, nx=20, ny=20, nz=20, h=4e-3 / 20, x0=None))
    f = W.initial_fields(prm, D0=1.2e-3, seed=0, T_noise=0.01)
    rates = []
    for form in (0, 1):
        p2 = dict(prm, species_form=form)
        st = S.to_state(f, p2)
        _, d = S.step(st, p2)
        rates.append(d["mdot_total"])
    assert rates[0] > 0 and rates[1] > 0
    assert abs(rates[0] - rates[1]) > 1e-3 * rates[0]


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FARFIELD])
def test_literal_form_fuel_balance_has_no_vapour_source(mode):
    """With no mdot in the species equation the fuel mass, measured from the
    assigned start state, falls by dt h^3 sum(mdot) (the evaporated liquid)
    plus what leaves the box; the new omega solves the source-free species
    system (eq. 9) to the solver tolerance."""
    prm, _ = W.config("C1", bc_mode=mode)
    prm = W.finalize(dict(prm, nx=16, ny=16, nz=16, h=4e-3 / 16, x0=None, species_form=1))
    f = W.initial_fields(prm, D0=1.2e-3, seed=1, T_noise=0.01)
    st = S.to_state(f, prm)
    rho_G = th.gas_density(prm)
    for _ in range(2):
        sa = S.assign_liquid_saturation(st, prm, rho_G)
        vol = prm["h"] ** 3
        M0 = vol * float((prm["rho_L"] * sa["alpha"] + sa["c"]).sum())
        rec = {}
        st, d = S.step(st, prm, record=rec)
        assert d["converged"] and d["mdot_total"] > 0
        expect = M0 - prm["dt"] * d["mdot_total"] - d["B_L"] - d["B_v"]
        assert abs(d["fuel_mass"] - expect) <= 1e-10 * M0
        # omega^{n+1} solves (rho_G theta/dt) w - div(rho_G D theta grad w) = c'/dt
        U = [sa["u"], sa["v"], sa["w"]]
        h, dt = prm["h"], prm["dt"]
        mS = rho_G * rec["theta"] / dt
        opS, _ = O.scalar_system(mS, rec["theta"], rho_G * prm["D_v"] / (h * h),
                                 2.0 * rho_G * prm["D_v"] / (h * h), 0.0, U, prm)
        b = rec["c_p"] / dt
        r = b - opS.apply(st["omega"])
        assert float(r.norm() / b.norm()) <= 1e-9
