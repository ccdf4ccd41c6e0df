"""Geometric interface advection (advection = 1) on the GPU against the CPU
oracle, through the C ABI.

* Whole steps on a ragged grid in the three boundary modes, and with the
  liquid moved by u itself: every field within 1e-9 (2-norm and element by
  element).  The planes (bisection on
  the exact cut volume) and the swept face areas (piecewise Simpson) are
  written independently on the two sides.
* The C1 droplet with its Stefan flow, 5 steps.
* A plane at 45 degrees in a uniform far-field flow: a whole step (no
  evaporation, no gravity, so the flow stays uniform) carries it exactly --
  every interior cell equals the exact volume fraction of the translated
  plane to 1e-12.
* 256^3 (the 20 bar Peng-Robinson workload, precision form): fuel balance
  per step, alpha within 1e-6 of [0, 1].
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import geo, step as S

from test_gpu_parity import _compare, _grid_params, _rel_max

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2005_02867_amd as ds
    return ds


def _run(prm, f, steps, tol=1e-13):
    ds = _lib()
    prm = dict(prm, tol=tol, tol_phi=tol, advection=1)
    print(f"geometric advection: nx={prm['nx']} ny={prm['ny']} nz={prm['nz']} bc={prm['bc_mode']} "
          f"eq={prm['eq_model']} steps={steps}", flush=True)
    g = ds.Grid(prm)
    g.set_fields(f)
    st = S.to_state(f, prm)
    for n in range(steps):
        g.step(1)
        st, d = S.step(st, prm)
        gd = g.diagnostics()
        _compare(g.get_fields(), st, f"step {n}")
        assert gd["fuel_mass"] == pytest.approx(d["fuel_mass"], rel=1e-12)
        assert gd["B_L"] == pytest.approx(d["B_L"], rel=1e-9, abs=1e-30)
        rel = abs(gd["fuel_mass"] - gd["fuel_mass_before"] + gd["B_L"] + gd["B_v"]) / gd["fuel_mass_before"]
        assert rel <= 1e-10, rel


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_geometric_step_parity(mode):
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0)
    f = W.random_fields(prm, seed=13)
    _run(prm, f, steps=3)


def test_geometric_step_parity_liquid_moved_by_u():
    """liquid_transport = 0: the liquid moved by u itself (no potential)."""
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, bc_mode=W.BC_FARFIELD, liquid_transport=0)
    f = W.random_fields(prm, seed=14)
    _run(prm, f, steps=3)


def test_geometric_droplet_c1():
    prm, run = W.config("C1")
    f = W.initial_fields(prm, **run)
    _run(prm, f, steps=5)


def _plane_fractions(n_grid, h, normal, c):
    i, j, k = np.indices(n_grid)
    corner = np.stack([i, j, k], axis=-1) * h
    nrm = np.broadcast_to(normal, n_grid + (3,))
    return geo.cell_volume(c - (corner * nrm).sum(-1), nrm, h) / h ** 3


def test_geometric_plane_carried_exactly():
    ds = _lib()
    n = (18, 24, 6)
    prm, _ = _grid_params(n=n, L=n[0] * 1.25e-4, bc_mode=W.BC_FARFIELD, evaporation=0, solve_energy=0,
                          g=(0.0, 0.0, 0.0), xi0=0.0, advection=1, tol=1e-13, tol_phi=1e-13)
    h, dt = prm["h"], prm["dt"]
    U0 = 0.3 * h / dt
    normal = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    c0 = 16.3 * h / math.sqrt(2.0)
    f = W.initial_fields(prm, D0=0.0)
    f["alpha"] = _plane_fractions(n, h, normal, c0)
    f["u"] = np.full(f["u"].shape, U0)
    f["omega"] = np.zeros(n)
    f["T"] = np.full(n, prm["T_amb"])
    g = ds.Grid(prm)
    g.set_fields(f)
    steps = 4
    g.step(steps)
    a = g.get_fields()["alpha"].cpu().numpy()
    ref = _plane_fractions(n, h, normal, c0 + U0 * steps * dt * normal[0])
    win = (slice(steps + 2, n[0] - 1), slice(steps + 2, n[1] - steps - 2), slice(None))
    err = np.abs(a - ref)[win].max()
    print("plane error", err)
    assert err <= 1e-12


def test_geometric_full_size_conservation():
    ds = _lib()
    prm, run = W.config("C3", advection=1)
    f = W.initial_fields(prm, D0=run["D0"], seed=run["seed"], T_noise=run["T_noise"])
    print("geometric advection at 256^3: 5 steps", flush=True)
    g = ds.Grid(prm)
    g.set_fields(f)
    for n in range(5):
        g.step(1)
        d = g.diagnostics()
        rel = abs(d["fuel_mass"] - d["fuel_mass_before"] + d["B_L"] + d["B_v"]) / d["fuel_mass_before"]
        assert rel <= 1e-10 and d["converged"], (n, rel)
        assert d["alpha_min"] >= -1e-6 and d["alpha_max"] <= 1.0 + 1e-6, (d["alpha_min"], d["alpha_max"])
