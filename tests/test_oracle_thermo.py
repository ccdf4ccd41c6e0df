"""Pins of the oracle's phase equilibrium (Section 2.5, eqs. 22-25) against
closed forms and independent routes through the Peng-Robinson equation."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import workloads as W
from oracle import thermo as th

R = 8.314462618


def _prm(**kw):
    prm, _ = W.config("C3", **kw)
    return prm


def test_clausius_clapeyron_reference_point_and_closed_form():
    prm, _ = W.config("C1")
    # p0 equals p_ref at the reference temperature (normal boiling point)
    assert th.vapour_pressure(prm["T_ref"], prm) == pytest.approx(prm["p_ref"], rel=1e-15)
    # closed form ln(p0/p_ref) = -(dh M/R)(1/T - 1/T_ref) at 300 K
    T = 300.0
    expect = prm["p_ref"] * math.exp(-(prm["dh_ev"] * prm["M_v"] / R) * (1 / T - 1 / prm["T_ref"]))
    assert th.vapour_pressure(T, prm) == pytest.approx(expect, rel=1e-14)
    # values quoted for this case: p0(300 K) ~ 8.52 kPa, y ~ 0.0852, omega ~ 0.250 at 1 bar
    assert th.vapour_pressure(T, prm) == pytest.approx(8516.0, abs=1.0)
    y = th.equilibrium_y(T, prm)
    assert y == pytest.approx(0.08516, abs=1e-4)
    assert th.mass_fraction(y, prm) == pytest.approx(0.2498, abs=1e-3)


def test_ideal_gas_density_closed_form():
    prm, _ = W.config("C1")
    assert th.gas_density(prm) == pytest.approx(prm["p"] * prm["M_G"] / (R * prm["T_amb"]), rel=1e-15)


def _Z_from_pressure_explicit(T, p, a, b):
    """Largest-volume root of p = RT/(v-b) - a/(v^2 + 2bv - b^2) (vapour)."""
    f = lambda v: R * T / (v - b) - a / (v * v + 2 * b * v - b * b) - p
    v_hi = 10 * R * T / p + 10 * b
    # bracket just above the largest spinodal/root region: scan down from v_hi
    vs = np.geomspace(b * 1.0001, v_hi, 20000)
    fs = np.array([f(v) for v in vs])
    idx = np.where(np.sign(fs[:-1]) != np.sign(fs[1:]))[0]
    i = idx[-1]
    v = optimize.brentq(f, vs[i], vs[i + 1], xtol=1e-30, rtol=1e-15)
    return p * v / (R * T)


@pytest.mark.parametrize("T,p", [(773.0, 2e6), (773.0, 1e6), (300.0, 1e5), (350.0, 5e5)])
def test_pr_Z_matches_pressure_explicit_form(T, p):
    prm = _prm()
    a2, b2 = th.pr_pure_ab(T, prm["Tc_G"], prm["Pc_G"], prm["acentric_G"])
    Z = th.pr_Z_pure_gas(T, p, prm)
    assert Z == pytest.approx(_Z_from_pressure_explicit(T, p, a2, b2), rel=1e-11)
    # fuel vapour (pure) at a subcritical state below its vapour pressure
    a1, b1 = th.pr_pure_ab(T, prm["Tc"], prm["Pc"], prm["acentric"])
    pv = min(p, 0.5 * th.vapour_pressure(T, prm)) if T < prm["Tc"] else p
    lnphi, Zf = th.pr_ln_phi_fuel(np.array([T]), pv, np.array([1.0]), prm)
    assert Zf[0] == pytest.approx(_Z_from_pressure_explicit(T, pv, a1, b1), rel=1e-10)


def _mixture_ab(T, y, prm):
    a1, b1, a2, b2 = th.pr_components(T, prm)
    a12 = math.sqrt(a1 * a2) * (1 - prm["kij"])
    a = y * y * a1 + 2 * y * (1 - y) * a12 + (1 - y) ** 2 * a2
    b = y * b1 + (1 - y) * b2
    return a, b


def _ln_phi_mix_quadrature(T, p, y, prm):
    """ln phi of the whole mixture = int_0^p (Z - 1)/p' dp' (exact thermodynamics)."""
    a, b = _mixture_ab(T, y, prm)

    def Zm(pp):
        A = a * pp / (R * T) ** 2
        B = b * pp / (R * T)
        return th.pr_largest_root(A, B)[0]

    val, err = integrate.quad(lambda pp: (Zm(pp) - 1.0) / pp, 0.0, p, epsabs=1e-14, epsrel=1e-12, limit=200)
    return val


@pytest.mark.parametrize("T,p", [(773.0, 2e6), (320.0, 2e6), (300.0, 1e6)])
def test_pr_pure_fugacity_matches_quadrature(T, p):
    """ln phi_pure(T, p) = int_0^p (Z-1)/p' dp' for the pure fuel (vapour branch)."""
    prm = _prm()
    pv = p if T > prm["Tc"] else 0.9 * th.vapour_pressure(T, prm)
    lnphi, _ = th.pr_ln_phi_fuel(np.array([T]), pv, np.array([1.0]), prm)
    assert lnphi[0] == pytest.approx(_ln_phi_mix_quadrature(T, pv, 1.0, prm), abs=1e-9)


@pytest.mark.parametrize("T,p,y", [(773.0, 2e6, 0.3), (500.0, 2e6, 0.05), (350.0, 1e6, 0.02)])
def test_pr_mixture_fugacity_is_partial_molar_derivative(T, p, y):
    """ln phi_hat_1 = d(n ln phi_mix)/d n_1 = G + (1-y) dG/dy for a binary,
    G(y) = ln phi_mix by quadrature (independent of the closed form)."""
    prm = _prm()
    G = lambda yy: _ln_phi_mix_quadrature(T, p, yy, prm)
    hstep = 1e-4
    dG = (G(y + hstep) - G(y - hstep)) / (2 * hstep)
    expect = G(y) + (1 - y) * dG
    lnphi, _ = th.pr_ln_phi_fuel(np.array([T]), p, np.array([y]), prm)
    assert lnphi[0] == pytest.approx(expect, abs=2e-7)


def test_pr_limits():
    prm = _prm()
    T = np.array([400.0])
    # p -> 0: ideal gas, phi -> 1
    lnphi, Z = th.pr_ln_phi_fuel(T, 1e-3, np.array([0.4]), prm)
    assert abs(lnphi[0]) < 1e-8 and abs(Z[0] - 1) < 1e-8
    # y -> 1 with any kij: phi_hat = phi_pure
    p1 = dict(prm, kij=0.0)
    a, _ = th.pr_ln_phi_fuel(T, 5e4, np.array([1.0]), prm)
    b, _ = th.pr_ln_phi_fuel(T, 5e4, np.array([1.0]), p1)
    assert a[0] == pytest.approx(b[0], rel=1e-14)


@pytest.mark.parametrize("P", [2e6, 1e6, 1e5])
def test_pr_equilibrium_solves_eq22_and_matches_bracketed_root(P):
    prm = _prm(p=P)
    T = np.array([300.0, 330.0, 360.0])
    y = th.equilibrium_y(T, prm)
    assert np.max(np.abs(th.equilibrium_residual(T, y, prm))) < 1e-13
    for Ti, yi in zip(T, y):
        f = lambda yy: th.equilibrium_residual(np.array([Ti]), np.array([yy]), prm)[0]
        hi = min(0.999, 3.0 * th.vapour_pressure(Ti, prm) / P)   # above the ideal value
        root = optimize.brentq(f, 1e-8, hi, xtol=1e-17, rtol=1e-15)
        assert yi == pytest.approx(root, rel=1e-12)
    # non-ideality raises the high-pressure vapour content above the ideal p0/p
    if P >= 1e6:
        assert np.all(y > th.vapour_pressure(T, prm) / P)


def test_pr_gas_density_uses_nitrogen_Z():
    prm = _prm()
    Z = th.pr_Z_pure_gas(prm["T_amb"], prm["p"], prm)
    assert th.gas_density(prm) == pytest.approx(prm["p"] * prm["M_G"] / (Z * R * prm["T_amb"]), rel=1e-15)
    assert 1.0 < Z < 1.02
