"""Pins of the oracle's differentiation form (oracle/adjoint.py):
derivatives of the droplet volume after a few steps against central finite
differences of the oracle's forward run, closed forms for one step from
rest, and exact zeros where a parameter cannot act.

Finite-difference directions are chosen so that no integer decision of the
step changes under the perturbation: parameters are perturbed by small
relative steps, and field directions either scale the field (which leaves
every limiter ratio unchanged) or keep every face velocity's sign."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as A
from oracle import interface as I
from oracle import thermo as th

TOL = dict(tol=1e-13, tol_phi=1e-13)
BAR = 2e-5


def _small(mode, eq=W.EQ_IDEAL):
    prm, _ = W.config("C1", bc_mode=mode, eq_model=eq, p=1e5 if eq == W.EQ_IDEAL else 2e6,
                      w_in=0.3 if mode == W.BC_FORCED else 0.0, **TOL)
    return W.finalize(dict(prm, nx=12, ny=13, nz=14, x0=None))


def _fd_param(f, prm, steps, name, rel):
    e = rel * prm[name]
    vp = A.volume_after(f, dict(prm, **{name: prm[name] + e}), steps)
    vm = A.volume_after(f, dict(prm, **{name: prm[name] - e}), steps)
    return (vp - vm) / (2.0 * e)


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_parameter_gradients_match_central_differences(mode):
    prm = _small(mode)
    f = W.random_fields(prm, seed=3)
    steps = 3
    r = A.volume_and_gradients(f, prm, steps)
    for name, key, rel in (("D_v", "dD_v", 1e-3), ("dh_ev", "ddh_ev", 1e-3), ("T_amb", "dT_amb", 1e-4)):
        fd = _fd_param(f, prm, steps, name, rel)
        assert abs(r[key] - fd) <= BAR * abs(fd), (name, r[key], fd)


def test_parameter_gradients_peng_robinson():
    prm = _small(W.BC_NATURAL, eq=W.EQ_PR)
    f = W.random_fields(prm, seed=3)
    steps = 2
    r = A.volume_and_gradients(f, prm, steps)
    # dh_ev step small enough that no interface cell crosses the y <= 1 - 1e-12 cap
    for name, key, rel in (("D_v", "dD_v", 1e-3), ("dh_ev", "ddh_ev", 1e-5), ("T_amb", "dT_amb", 1e-4)):
        fd = _fd_param(f, prm, steps, name, rel)
        assert abs(r[key] - fd) <= BAR * abs(fd), (name, r[key], fd)


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FARFIELD])
def test_field_gradients_match_directional_differences(mode):
    prm = _small(mode)
    f = W.random_fields(prm, seed=4)
    steps = 3
    r = A.volume_and_gradients(f, prm, steps)
    rng = np.random.default_rng(7)
    for k, sc in (("alpha", 1e-6), ("T", 1e-4), ("omega", 1e-4), ("u", 1e-4), ("v", 1e-4), ("w", 1e-4)):
        if k in ("u", "v", "w"):
            d = f[k] * (1.0 + 0.5 * rng.uniform(-1.0, 1.0, f[k].shape))   # signs kept
        else:
            d = f[k].copy()                                                # scaling
        fp = dict(f)
        fm = dict(f)
        fp[k] = f[k] + sc * d
        fm[k] = f[k] - sc * d
        fd = (A.volume_after(fp, prm, steps) - A.volume_after(fm, prm, steps)) / (2.0 * sc)
        ad = float((r["grads"][k] * torch.as_tensor(d)).sum())
        assert abs(ad - fd) <= BAR * abs(fd), (k, ad, fd)


def test_one_step_from_rest_closed_forms():
    """u = 0, omega = 0: the first step moves no liquid (phi = 0, zero face
    fluxes), so V_1 = V_0 - dt h^3 sum(mdot)/rho_L, and sum(mdot) = sum(mdot_raw)
    for any K (eq. 20).  With omega_adj = 0, mdot_raw = rho_G D omega_sat |grad alpha|/d:
      dV_1/dD_v   = -(dt h^3 rho_G / rho_L) sum omega_sat |grad alpha| / d
      dV_1/ddh_ev = -(dt h^3 rho_G D / rho_L) sum (d omega_sat/d dh_ev) |grad alpha| / d
      dV_1/dT_amb = -(V_1 - V_0)/T_amb      (rho_G = p M_G/(R T_amb))."""
    prm, run = W.config("C1", **TOL)
    prm = W.finalize(dict(prm, nx=16, ny=16, nz=16, h=4e-3 / 16, x0=None))
    f = W.initial_fields(prm, D0=1.0e-3, seed=0, T_noise=0.01)
    r = A.volume_and_gradients(f, prm, 1)
    a = torch.as_tensor(f["alpha"])
    T = torch.as_tensor(f["T"])
    geo = I.geometry(a, prm)
    ic, found = geo["icells"][geo["found"]], geo["found"]
    gm = geo["gradmag"][ic[:, 0], ic[:, 1], ic[:, 2]]
    d = geo["dist"][found]
    Ti = T[ic[:, 0], ic[:, 1], ic[:, 2]]
    ws = th.saturation_omega(Ti, prm)
    rho_G = th.gas_density(prm)
    h, dt, rho_L, D = prm["h"], prm["dt"], prm["rho_L"], prm["D_v"]
    assert math.isclose(r["dD_v"], -(dt * h ** 3 * rho_G / rho_L) * float((ws * gm / d).sum()), rel_tol=1e-10)
    # omega_sat = y M_v/(y M_v + (1-y) M_G), y = p0/p capped at 1 - 1e-12
    Mv, MG = prm["M_v"], prm["M_G"]
    y_raw = th.vapour_pressure(Ti, prm) / prm["p"]
    y = torch.clamp(y_raw, max=1.0 - 1e-12)
    dy = torch.where(y_raw <= 1.0 - 1e-12, y_raw * (-(Mv / th.R_GAS) * (1.0 / Ti - 1.0 / prm["T_ref"])),
                     torch.zeros_like(y))
    dws = Mv * MG / (y * Mv + (1.0 - y) * MG) ** 2 * dy
    expect = -(dt * h ** 3 * rho_G * D / rho_L) * float((dws * gm / d).sum())
    assert math.isclose(r["ddh_ev"], expect, rel_tol=1e-10)
    V0 = h ** 3 * float(a.sum())
    assert math.isclose(r["dT_amb"], -(r["volume"] - V0) / prm["T_amb"], rel_tol=1e-9)
    # the first step's volume change: alpha moves only by the source
    assert r["volume"] < V0


def test_no_evaporation_zero_gradients():
    """Without the evaporation source neither D_v nor dh_ev can reach alpha."""
    prm = dict(_small(W.BC_NATURAL), evaporation=0)
    f = W.random_fields(prm, seed=5)
    r = A.volume_and_gradients(f, prm, 2)
    assert r["dD_v"] == 0.0 and r["ddh_ev"] == 0.0
    assert r["dT_amb"] != 0.0          # the gas density still moves the flow
