"""Pins of the oracle's variable-density gas (eq. 24 per cell, eq. 7's
compressibility term; oracle/gas.py).

* eq. 24, ideal model: Dalton's law, p = p_vapour + p_N2 with each partial
  pressure from its own partial density (a swapped molar mass or a
  mole/mass mix-up fails it); omega = 0 gives the ambient constant.
* eq. 24, Peng-Robinson: omega = 0 gives the pure-N2 route of thermo; two
  identical components (fuel data set to N2's, k_ij = 0) give a density
  independent of omega (a dropped or doubled cross term of the mixing rule
  fails it); at low pressure the second virial coefficient is quadratic in
  the mole fraction with the van der Waals one-fluid cross coefficient
  B_12 = (b_1 + b_2)/2 - sqrt(a_1 a_2)(1 - k_ij)/RT (Z = 1 + B p/RT + O(p^2)).
* Inversion: rho_G(T, omega) omega = q to round-off, monotone in q, and the
  ideal model's closed form omega = (a/M_G)/(1 - a/M_v + a/M_G), a = qRT/p.
* Compressibility source: for an ideal gas without vapour rho_G is
  proportional to 1/T, so (1 - alpha) ln(rho^{n+1}/rho')/dt equals
  -(1 - alpha) ln(T^{n+1}/T')/dt from the recorded temperatures.
* Whole steps: with T = T_amb and no vapour the variable path reproduces the
  constant one; fuel mass balance to 1e-10 per step; div u = S after the
  projection with the compressibility term in S; a gas box with a cold and a
  hot half develops the circulation of heavier gas sinking, which the
  constant-density gas does not.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import gas, step as S, thermo

R = thermo.R_GAS


def _prm(eq=W.EQ_IDEAL, **kw):
    prm, _ = W.config("C1", eq_model=eq, gas_density=1, **kw)
    return prm


@pytest.mark.parametrize("T", [300.0, 550.0, 873.0])
def test_ideal_density_dalton(T):
    prm = _prm(W.EQ_IDEAL, p=2.0e6)
    om = np.array([0.0, 1e-6, 0.05, 0.3, 0.7, 0.999])
    rho = gas.density_np(np.full(om.shape, T), om, prm)
    p_v = rho * om * R * T / prm["M_v"]
    p_n = rho * (1.0 - om) * R * T / prm["M_G"]
    assert np.max(np.abs(p_v + p_n - prm["p"])) <= 1e-13 * prm["p"]
    assert abs(rho[0] - float(thermo.gas_density(dict(prm, T_amb=T), T))) <= 1e-15 * rho[0]


def test_pr_pure_nitrogen_limit():
    prm = _prm(W.EQ_PR, p=2.0e6)
    T = np.array([300.0, 450.0, 773.0])
    rho = gas.density_np(T, np.zeros(3), prm)
    for t, r in zip(T, rho):
        ref = float(thermo.gas_density(dict(prm, T_amb=float(t)), float(t)))
        assert abs(r - ref) <= 1e-13 * ref


def test_pr_identical_components():
    prm = _prm(W.EQ_PR, p=2.0e6)
    prm = dict(prm, Tc=prm["Tc_G"], Pc=prm["Pc_G"], acentric=prm["acentric_G"], kij=0.0, M_v=prm["M_G"])
    om = np.linspace(0.0, 1.0, 7)
    rho = gas.density_np(np.full(om.shape, 400.0), om, prm)
    assert np.max(np.abs(rho - rho[0])) <= 1e-13 * rho[0]


def test_pr_second_virial_coefficient():
    """Z = 1 + B p/RT + C' p^2 + ...: B from Richardson extrapolation of
    (Z - 1) RT/p at 200 and 400 Pa (the O(p) part, ~1e-5 of B there,
    cancels); a wrong cross term moves B by percents of B_11."""
    T = 600.0
    RT = R * T
    prm = _prm(W.EQ_PR)
    a1, b1, a2, b2 = thermo.pr_components(T, prm)
    B11, B22 = b1 - a1 / RT, b2 - a2 / RT
    B12 = 0.5 * (b1 + b2) - math.sqrt(a1 * a2) * (1.0 - prm["kij"]) / RT
    scale = max(abs(B11), abs(B22))

    def B_at(p, y):
        Z = float(gas.compressibility(np.array([T]), np.array([y]), dict(prm, p=p))[0])
        return (Z - 1.0) * RT / p

    for y in (0.0, 0.2, 0.5, 0.9, 1.0):
        B = 2.0 * B_at(200.0, y) - B_at(400.0, y)
        want = y * y * B11 + 2.0 * y * (1.0 - y) * B12 + (1.0 - y) ** 2 * B22
        assert abs(B - want) <= 1e-8 * scale, (y, B, want)


@pytest.mark.parametrize("eq", [W.EQ_IDEAL, W.EQ_PR])
def test_inversion_round_trip(eq):
    prm = _prm(eq, p=2.0e6)
    rng = np.random.default_rng(3)
    T = rng.uniform(320.0, 873.0, 400)
    om_true = np.concatenate([np.zeros(10), 10.0 ** rng.uniform(-9, -0.3, 390)])
    q = gas.density_np(T, om_true, prm) * om_true
    om, rho = gas.invert_np(T, q, prm)
    assert np.max(np.abs(rho * om - q) / np.maximum(q, 1e-300)) <= 1e-13
    assert np.max(np.abs(om - om_true) / np.maximum(om_true, 1e-300)) <= 1e-12
    assert np.all(om[:10] == 0.0)
    # monotone in q at fixed T
    qs = np.linspace(0.0, 0.5 * q.max(), 50)
    o2, _ = gas.invert_np(np.full(qs.shape, 500.0), qs, prm)
    assert np.all(np.diff(o2) > 0.0)


def test_inversion_ideal_closed_form():
    prm = _prm(W.EQ_IDEAL, p=1.0e6)
    rng = np.random.default_rng(4)
    T = rng.uniform(300.0, 900.0, 200)
    q = rng.uniform(0.0, 3.0, 200)
    om, _ = gas.invert_np(T, q, prm)
    a = q * R * T / prm["p"]
    closed = (a / prm["M_G"]) / (1.0 - a / prm["M_v"] + a / prm["M_G"])
    assert np.max(np.abs(om - closed) / closed) <= 1e-13


def _gas_box(prm, T_field, seed=0):
    """All-gas state (no droplet) with temperature T_field."""
    n = (prm["nx"], prm["ny"], prm["nz"])
    f = dict(alpha=np.zeros(n), T=T_field, omega=np.zeros(n), u=np.zeros((n[0] + 1, n[1], n[2])),
             v=np.zeros((n[0], n[1] + 1, n[2])), w=np.zeros((n[0], n[1], n[2] + 1)), p=np.zeros(n))
    return f


def test_compressibility_source_ideal_closed_form():
    prm = _prm(W.EQ_IDEAL, evaporation=0, tol=1e-13)
    prm = W.finalize(dict(prm, nx=10, ny=9, nz=11, x0=None))
    rng = np.random.default_rng(6)
    T0 = 500.0 + 200.0 * rng.uniform(0, 1, (10, 9, 11))
    f = _gas_box(prm, T0)
    f["w"][:, :, 1:-1] = 0.01 * rng.uniform(-1, 1, f["w"][:, :, 1:-1].shape)
    st = S.to_state(f, prm)
    rec = {}
    new, d = S.step(st, prm, record=rec)
    assert d["converged"]
    want = -torch.log(new["T"] / rec["T_p"]) / prm["dt"]
    got = rec["S_comp"]
    err = float((got - want).abs().max() / want.abs().max())
    assert err <= 1e-10, err
    assert float(want.abs().max()) > 1.0   # a real source, not a vanishing one


@pytest.mark.parametrize("eq", [W.EQ_IDEAL, W.EQ_PR])
def test_reduces_to_constant_gas(eq):
    """T = T_amb everywhere and no vapour: rho_G is the ambient constant in
    every cell, the source vanishes and the step equals the constant path."""
    prm = _prm(eq, evaporation=0, tol=1e-13)
    prm = W.finalize(dict(prm, nx=9, ny=8, nz=10, x0=None))
    f = W.random_fields(prm, seed=5)
    f["T"] = np.full(f["alpha"].shape, prm["T_amb"])
    f["omega"] = np.zeros_like(f["alpha"])
    a, _ = S.step(S.to_state(f, prm), prm)
    b, _ = S.step(S.to_state(f, dict(prm, gas_density=0)), dict(prm, gas_density=0))
    for k in ("alpha", "c", "T", "p", "u", "v", "w"):
        den = max(float(b[k].abs().max()), 1e-300)
        assert float((a[k] - b[k]).abs().max()) <= 1e-12 * den, k


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_variable_gas_conserves_fuel_and_projects(mode):
    prm, _ = W.config("C1", bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0, gas_density=1,
                      eq_model=W.EQ_PR, p=2.0e6, tol=1e-13, tol_phi=1e-13)
    prm = W.finalize(dict(prm, nx=14, ny=15, nz=13, x0=None))
    f = W.random_fields(prm, seed=8)
    st = S.to_state(f, prm)
    for _ in range(2):
        rec = {}
        st_new, d = S.step(st, prm, record=rec)
        rel = abs(d["fuel_mass"] - d["fuel_mass_before"] + d["B_L"] + d["B_v"]) / d["fuel_mass_before"]
        assert rel <= 1e-10 and d["converged"], rel
        u, v, w = st_new["u"], st_new["v"], st_new["w"]
        div = ((u[1:] - u[:-1]) + (v[:, 1:] - v[:, :-1]) + (w[:, :, 1:] - w[:, :, :-1])) / prm["h"]
        scale = float(rec["S"].abs().max())
        assert float((div - rec["S"]).abs().max()) <= 1e-9 * scale
        assert float(rec["S_comp"].abs().max()) > 0.0
        # the state's density matches eq. 24 at its own T and omega
        r = gas.density(st_new["T"], st_new["omega"], prm)
        assert float(((r - st_new["rho_G"]) / r).abs().max()) <= 1e-12
        st = st_new


def test_cold_gas_slumps_under_hot_gas():
    """A gas box, cold (400 K) in x < L/2 and hot (773 K) in x > L/2: a
    horizontal density jump is not hydrostatic, so gravity drives the lock
    exchange -- on the plane between the halves the cold gas flows under
    towards the hot side and the hot gas over towards the cold side.  The
    expansion flow of the conduction between the halves is the same with and
    without gravity, so it is taken out by a run with g = 0.  The
    constant-density gas stays at rest."""
    prm, _ = W.config("C1", gas_density=1, evaporation=0, tol=1e-12, tol_phi=1e-12, dt=2e-5)
    prm = W.finalize(dict(prm, nx=12, ny=4, nz=12, x0=None))
    n = (12, 4, 12)
    T = np.where((np.arange(12) < 6)[:, None, None], 400.0, 773.0) * np.ones(n)

    def run(q):
        st = S.to_state(_gas_box(q, T), q)
        for _ in range(5):
            st, d = S.step(st, q)
            assert d["converged"]
        return st["u"][6]   # the x faces between the halves, (ny, nz)

    du = run(prm) - run(dict(prm, g=(0.0, 0.0, 0.0)))
    lower, upper = float(du[:, :6].mean()), float(du[:, 6:].mean())
    assert lower > 1e-4 and upper < -1e-4, (lower, upper)
    uk = run(dict(prm, gas_density=0))
    assert float(uk.abs().max()) < 1e-12
