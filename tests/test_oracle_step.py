"""Pins of the oracle's whole step: conservation, divergence, hydrostatics,
the static droplet held by the centripetal force, free fall, symmetry."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

import workloads as W
from oracle import operators as O
from oracle import step as S
from oracle import thermo as th


def _cfg(name="C1", n=None, L=None, **kw):
    prm, run = W.config(name, **kw)
    if n is not None:
        L = L if L is not None else prm["h"] * prm["nx"]
        prm = W.finalize(dict(prm, nx=n, ny=n, nz=n, h=L / n, x0=None))
    return prm, run


def _face_div(st, h):
    return O.divergence(st["u"], st["v"], st["w"], h)


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_fuel_mass_conserved_per_step(mode):
    """|M^{n+1} - M^n + B_L + B_v| / M^n <= 1e-10 with M = h^3 sum(rho_L alpha + c)."""
    prm, run = _cfg("C1", n=20, bc_mode=mode, w_in=0.3 if mode == W.BC_FORCED else 0.0)
    f = W.initial_fields(prm, D0=1e-3, seed=0, T_noise=0.01)
    st = S.to_state(f, prm)
    for _ in range(4):
        st, d = S.step(st, prm)
        rel = abs(d["fuel_mass"] - d["fuel_mass_before"] + d["B_L"] + d["B_v"]) / d["fuel_mass_before"]
        assert rel <= 1e-10, rel
        assert d["converged"]
        assert d["mdot_total"] > 0


def test_liquid_budget_exact():
    """Delta V = -dt h^3 sum(mdot)/rho_L - B_L/rho_L (eqs. 3-4)."""
    prm, run = _cfg("C1", n=20, bc_mode=W.BC_FORCED, w_in=0.5)
    f = W.initial_fields(prm, D0=1.2e-3, seed=0, T_noise=0.01)
    st = S.to_state(f, prm)
    for _ in range(3):
        V0 = S.droplet_volume(st, prm)
        st, d = S.step(st, prm)
        dV = d["volume"] - V0
        expect = -prm["dt"] * d["mdot_total"] / prm["rho_L"] - d["B_L"] / prm["rho_L"]
        assert dV == pytest.approx(expect, rel=1e-9, abs=1e-12 * V0)


def test_projection_divergence_matches_stefan_source():
    """div_h u^{n+1} = mdot (1/rho_G - 1/rho_L) to the solve tolerance, and the
    net outflow through the box equals h^3 sum S (divergence theorem)."""
    prm, run = _cfg("C1", n=16, tol=1e-13, tol_phi=1e-13)
    f = W.initial_fields(prm, D0=1e-3, seed=0, T_noise=0.01)
    st = S.to_state(f, prm)
    rec = {}
    new, d = S.step(st, prm, record=rec)
    h = prm["h"]
    Ssrc = rec["mdot"] * (1 / rec["rho_G"] - 1 / prm["rho_L"])
    div = _face_div(new, h)
    scale = float(Ssrc.abs().max())
    assert float((div - Ssrc).abs().max()) <= 1e-8 * scale
    outflow = h * h * float(new["w"][:, :, -1].sum() - new["w"][:, :, 0].sum()
                            + new["u"][-1].sum() - new["u"][0].sum() + new["v"][:, -1].sum() - new["v"][:, 0].sum())
    assert outflow == pytest.approx(h ** 3 * float(Ssrc.sum()), rel=1e-8)


def test_no_evaporation_gives_divergence_free_velocity():
    prm, run = _cfg("C1", n=16, tol=1e-13, evaporation=0)
    f = W.initial_fields(prm, D0=1e-3, seed=0, T_noise=0.01)
    st = S.to_state(f, prm)
    for _ in range(2):
        st, d = S.step(st, prm)
    umax = max(float(st[k].abs().max()) for k in "uvw")
    assert umax > 0
    assert float(_face_div(st, prm["h"]).abs().max()) <= 1e-9 * umax / prm["h"]


def test_static_gas_column_stays_at_rest_exactly():
    """alpha = 0 with gravity: the p_rgh form has no force on a uniform
    density, so u and p_rgh stay exactly zero (eqs. 6-7)."""
    prm, run = _cfg("C1", n=12)
    f = W.initial_fields(prm, D0=1e-3)
    f["alpha"][:] = 0.0
    f["T"][:] = prm["T_amb"]
    st = S.to_state(f, prm)
    for _ in range(2):
        st, d = S.step(st, prm)
    for k in ("u", "v", "w", "p"):
        assert float(st[k].abs().max()) == 0.0, k


def test_free_fall_acceleration():
    """xi0 = 0: one step from rest accelerates the droplet core by
    g (rho_L - rho_G)/(rho_L + rho_G/2) dt (weight, buoyancy and added mass
    of a sphere); the error falls with the grid spacing."""
    errs = []
    for n in (16, 32):
        prm, run = _cfg("C1", n=n, evaporation=0, solve_energy=0, xi0=0.0, tol=1e-13, tol_phi=1e-13)
        f = W.initial_fields(prm, D0=1e-3)
        st = S.to_state(f, prm)
        new, d = S.step(st, prm)
        rho_G = th.gas_density(prm)
        expect = prm["g"][2] * prm["dt"] * (prm["rho_L"] - rho_G) / (prm["rho_L"] + 0.5 * rho_G)
        wc = float(new["w"][n // 2, n // 2, n // 2])           # face at the droplet centre
        errs.append(abs(wc / expect - 1.0))
    assert errs[0] < 0.05 and errs[1] < 0.025 and errs[0] / errs[1] > 1.6, errs


def test_static_droplet_pressure_matches_force_balance():
    """g = 0, no evaporation, xi0 = 1: one projection from rest gives the
    pressure of -grad p + f_m = 0 (Section 5.1),
    p(r) = int_r^inf rho alpha |xi'| ds, with parasitic currents far below
    the force impulse (Section 2.6)."""
    errs = []
    for n in (32, 64):
        prm, run = _cfg("C1", n=n, g=(0.0, 0.0, 0.0), evaporation=0, solve_energy=0, tol=1e-13, tol_phi=1e-13)
        f = W.initial_fields(prm, D0=1e-3)
        st = S.to_state(f, prm)
        new, d = S.step(st, prm)
        h = prm["h"]
        rho_G = th.gas_density(prm)
        R, wdt = 0.5e-3, 1.5 * h

        def integrand(s):
            a = 0.5 * (1 - math.tanh((s - R) / wdt))
            rho = a * prm["rho_L"] + (1 - a) * rho_G
            return rho * a * prm["xi0"] * 0.5 * prm["Df"] / s ** 2 if s > prm["r_fib"] else 0.0

        j = n // 2
        xs = (np.arange(n) + 0.5) * h - prm["x0"][0]
        err = 0.0
        for i in range(n):
            r = math.sqrt(xs[i] ** 2 + 2 * (0.5 * h) ** 2)
            if xs[i] <= 0 or r > 0.45e-3:
                continue
            q = integrate.quad(integrand, r, 4e-3, limit=200)[0]
            err = max(err, abs(float(new["p"][i, j, j]) - q))
        errs.append(err)
        umax = max(float(new[k].abs().max()) for k in "uvw")
        assert umax < 1e-3 * prm["dt"] * prm["xi0"] * 0.5 * prm["Df"] / prm["r_fib"] ** 2
    # second order in h; a few percent of the ~100-300 Pa droplet pressure
    assert errs[0] / errs[1] > 3.0 and errs[1] < 1.0, errs


def test_mirror_symmetry():
    """No noise, g = 0, farfield boundaries: the state stays mirror-symmetric."""
    prm, run = _cfg("C1", n=14, g=(0.0, 0.0, 0.0), bc_mode=W.BC_FARFIELD, tol=1e-13, tol_phi=1e-13)
    f = W.initial_fields(prm, D0=1e-3)
    st = S.to_state(f, prm)
    for _ in range(3):
        st, d = S.step(st, prm)
    for k in ("alpha", "T", "omega", "p"):
        a = st[k]
        scale = float(a.abs().max())
        for ax in range(3):
            assert float((a - torch.flip(a, [ax])).abs().max()) <= 1e-11 * scale, (k, ax)
    u = st["u"]
    assert float((u + torch.flip(u, [0])).abs().max()) <= 1e-11 * float(u.abs().max())
