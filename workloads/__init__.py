"""Seeded synthetic workloads: parameter sets and initial fields.

This module is shared by the CPU oracle and the GPU library's tests and
benchmark.  It holds values and input construction only -- none of the
method's arithmetic (no fluxes, no equilibrium, no operators).

Parameter sets follow the operating conditions the paper uses for its
droplet cases (1D-model comparison table, natural/forced convection tables:
millimetre n-heptane droplets, 300 K liquid, 773-873 K nitrogen, 1-20 bar).
Property constants the paper takes from property databases are fixed here
once ("constant properties"); see the design notes for the reading.

Grid layout used everywhere: cell (i, j, k) has centre ((i+1/2)h, (j+1/2)h,
(k+1/2)h), flat index (i*ny + j)*nz + k (z fastest).  Face velocities are
staggered (MAC): u has shape (nx+1, ny, nz), v (nx, ny+1, nz), w (nx, ny, nz+1).
"""
from __future__ import annotations

import copy
import math

import numpy as np

R_GAS = 8.314462618  # J/mol/K

EQ_IDEAL, EQ_PR = 0, 1
BC_NATURAL, BC_FORCED, BC_FARFIELD = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1

# Fluid pair: n-heptane (critical data of the high-pressure configurations)
# evaporating into nitrogen.
_BASE = dict(
    nx=32, ny=32, nz=32, h=4e-3 / 32,
    dt=1e-5,
    p=1.0e5, T_amb=773.0, T_liq=300.0,
    rho_L=684.0, cp_L=2240.0, k_L=0.12,
    cp_G=1120.0, k_G=0.055,
    D_v=5e-5, dh_ev=3.2e5,
    M_v=0.100204, M_G=0.0280134,
    g=(0.0, 0.0, -9.81),
    xi0=1.0, Df=5e-5, r_fib=5e-5,
    w_in=0.0,
    x0=None,                      # droplet / fiber centre; default = domain centre
    Tc=540.0, Pc=27.4e5, acentric=0.35, kij=0.1,
    Tc_G=126.2, Pc_G=33.98e5, acentric_G=0.0372,
    T_ref=371.58, p_ref=101325.0,
    eps_int=1e-3, eps_gas=0.5, theta_min=1e-8, s_max=16,
    tol=1e-10, tol_phi=1e-8, maxit=20000,
    eq_model=EQ_IDEAL, bc_mode=BC_NATURAL, precision=PREC_FP64,
    solve_energy=1, evaporation=1,
    pressure_precond=1, liquid_transport=1, species_form=0,
    # viscous momentum (off in the configurations, which give no viscosity):
    # n-heptane near 300 K and nitrogen near 773 K (Sutherland's law)
    viscous=0, mu_L=3.9e-4, mu_G=3.4e-5,
    # 0: rho_G of the ambient gas everywhere; 1: eq. 24 per cell (variable gas)
    gas_density=0,
    # liquid advection: 0 flux-limited (TVD van Leer), 1 geometric (a plane per surface cell)
    advection=0,
)

# name -> (overrides, run description)
_CONFIGS = {
    # plain FP64, 32^3 over a 4 mm cube, 1.0 mm droplet, 1 bar / 773 K
    "C1": (dict(nx=32, ny=32, nz=32, h=4e-3 / 32, dt=1e-5, p=1.0e5, T_amb=773.0,
                eq_model=EQ_IDEAL, bc_mode=BC_NATURAL, tol=1e-10),
           dict(D0=1.0e-3, steps=20, seed=0, T_noise=0.01, R_noise=0.0)),
    # 128^3 over 6 mm, 1.5 mm droplet, forced 0.5 m/s inflow at z-
    "C2": (dict(nx=128, ny=128, nz=128, h=6e-3 / 128, dt=5e-6, p=1.0e5, T_amb=773.0,
                eq_model=EQ_IDEAL, bc_mode=BC_FORCED, w_in=0.5, tol=1e-10),
           dict(D0=1.5e-3, steps=200, seed=None, T_noise=0.0, R_noise=0.0)),
    # 256^3 over 8 mm, 20 bar, Peng-Robinson equilibrium, mixed precision
    "C3": (dict(nx=256, ny=256, nz=256, h=8e-3 / 256, dt=5e-6, p=2.0e6, T_amb=773.0,
                eq_model=EQ_PR, bc_mode=BC_NATURAL, precision=PREC_MIXED, tol=1e-10),
           dict(D0=1.0e-3, steps=200, seed=1, T_noise=0.02, R_noise=0.0)),
    # 96^3 over 5 mm, 1 bar / 873 K, natural convection (differentiation form)
    "C4": (dict(nx=96, ny=96, nz=96, h=5e-3 / 96, dt=1e-5, p=1.0e5, T_amb=873.0,
                eq_model=EQ_IDEAL, bc_mode=BC_NATURAL, tol=1e-10),
           dict(D0=1.0e-3, steps=100, seed=None, T_noise=0.0, R_noise=0.0, ckpt=10)),
    # 384^3 over 10 mm, 10 bar, PR, forced 1.0 m/s, mixed precision
    "C5": (dict(nx=384, ny=384, nz=384, h=1e-2 / 384, dt=4e-6, p=1.0e6, T_amb=773.0,
                eq_model=EQ_PR, bc_mode=BC_FORCED, w_in=1.0, precision=PREC_MIXED,
                tol=1e-10),
           dict(D0=2.0e-3, steps=500, seed=2, T_noise=0.01, R_noise=0.005, ckpt=20)),
}


def config(name: str, **overrides) -> tuple[dict, dict]:
    """Return (params, run) for a named configuration, with overrides applied
    to params (keys of params) or run (keys of run)."""
    base, run = _CONFIGS[name]
    params = copy.deepcopy(_BASE)
    params.update(base)
    run = dict(run)
    for k, v in overrides.items():
        if k in params:
            params[k] = v
        elif k in run:
            run[k] = v
        else:
            raise KeyError(k)
    return finalize(params), run


def finalize(params: dict) -> dict:
    """Fill defaults that depend on the grid (droplet centre)."""
    p = dict(params)
    if p.get("x0") is None:
        p["x0"] = (0.5 * p["nx"] * p["h"], 0.5 * p["ny"] * p["h"], 0.5 * p["nz"] * p["h"])
    p["g"] = tuple(float(x) for x in p["g"])
    p["x0"] = tuple(float(x) for x in p["x0"])
    return p


def scaled(name: str, n: int, **overrides) -> tuple[dict, dict]:
    """A configuration shrunk to an n^3 grid over the same physical box."""
    params, run = config(name, **overrides)
    L = params["h"] * params["nx"]
    params.update(nx=n, ny=n, nz=n, h=L / n)
    params["x0"] = None
    return finalize(params), run


def initial_fields(params: dict, D0: float, seed=None, T_noise=0.0, R_noise=0.0,
                   width_cells=1.5, **_ignored) -> dict:
    """Seeded initial state: tanh-smoothed sphere of diameter D0 at x0.

    alpha = 1/2 [1 - tanh((r - R)/(width_cells h))];
    T = alpha T_liq + (1 - alpha) T_amb, times (1 + T_noise U(-1,1));
    omega = 0, u = v = w = 0 (w = w_in on a forced inlet), p = 0.
    U comes from numpy.random.default_rng(seed).uniform(-1, 1, ncell) in C
    order; a second draw of the same generator perturbs the radius per cell.
    """
    nx, ny, nz, h = params["nx"], params["ny"], params["nz"], params["h"]
    x0 = params["x0"]
    xc = (np.arange(nx) + 0.5) * h - x0[0]
    yc = (np.arange(ny) + 0.5) * h - x0[1]
    zc = (np.arange(nz) + 0.5) * h - x0[2]
    r = np.sqrt(xc[:, None, None] ** 2 + yc[None, :, None] ** 2 + zc[None, None, :] ** 2)
    R = np.full(r.shape, 0.5 * D0)
    U = np.zeros(r.shape)
    if seed is not None:
        rng = np.random.default_rng(seed)
        U = rng.uniform(-1.0, 1.0, nx * ny * nz).reshape(nx, ny, nz)
        if R_noise:
            U2 = rng.uniform(-1.0, 1.0, nx * ny * nz).reshape(nx, ny, nz)
            R = R * (1.0 + R_noise * U2)
    alpha = 0.5 * (1.0 - np.tanh((r - R) / (width_cells * h)))
    T = alpha * params["T_liq"] + (1.0 - alpha) * params["T_amb"]
    if T_noise:
        T = T * (1.0 + T_noise * U)
    omega = np.zeros_like(alpha)
    u = np.zeros((nx + 1, ny, nz))
    v = np.zeros((nx, ny + 1, nz))
    w = np.zeros((nx, ny, nz + 1))
    if params["bc_mode"] == BC_FORCED:
        w[:, :, 0] = params["w_in"]
    p = np.zeros_like(alpha)
    return dict(alpha=alpha, T=T, omega=omega, u=u, v=v, w=w, p=p)


def random_fields(params: dict, seed: int, alpha_band=True) -> dict:
    """Random (but physically shaped) state for kernel-level parity cases:
    a perturbed droplet plus small random velocities, vapour and pressure."""
    rng = np.random.default_rng(seed)
    nx, ny, nz, h = params["nx"], params["ny"], params["nz"], params["h"]
    L = min(nx, ny, nz) * h
    f = initial_fields(params, D0=0.45 * L, seed=seed, T_noise=0.01, R_noise=0.05)
    umax = 0.02
    f["u"] = umax * rng.uniform(-1, 1, f["u"].shape)
    f["v"] = umax * rng.uniform(-1, 1, f["v"].shape)
    f["w"] = umax * rng.uniform(-1, 1, f["w"].shape)
    if params["bc_mode"] != BC_FARFIELD:
        f["u"][0] = 0.0
        f["u"][-1] = 0.0
        f["v"][:, 0] = 0.0
        f["v"][:, -1] = 0.0
    if params["bc_mode"] == BC_FORCED:
        f["w"][:, :, 0] = params["w_in"]
    f["omega"] = 0.3 * rng.uniform(0, 1, f["alpha"].shape) * (1.0 - f["alpha"])
    f["p"] = 10.0 * rng.uniform(-1, 1, f["alpha"].shape)
    return f

