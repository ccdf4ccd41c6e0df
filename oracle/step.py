"""One time step of the method, in the paper's segregated order (Section 3.1).

Test infrastructure: the CPU oracle only.

State (torch.float64, CPU):
  alpha (nx,ny,nz)   liquid volume fraction
  c     (nx,ny,nz)   vapour partial density rho_G theta omega (kg/m^3)
  omega (nx,ny,nz)   vapour mass fraction in the gas
  T     (nx,ny,nz)   temperature
  p     (nx,ny,nz)   p_rgh
  u (nx+1,ny,nz), v (nx,ny+1,nz), w (nx,ny,nz+1)   face velocities

Order (the six steps of Section 3.1):
  1. evaporation flux  (interface.geometry, raw_evaporation, redistribute)
  2. alpha source      alpha1 = alpha - dt mdot/rho_L          (eq. 4)
  3. advection         vof.advect (advection = 1: the liquid by geo.advect)  (eq. 3)
  4. properties        eq. 31 on alpha' clamped to [0, 1]; theta = max(1-alpha', theta_min)
  5. energy, species (operators) and momentum predictor (momentum; with
     viscous = 1 its implicit viscous part, viscous.py)
  6. pressure (eq. 7) and velocity correction
Species conservation reading: vapour lives in the gas fraction only; c is
moved with the gas volume flux, gains mdot, and is updated after the
implicit solve in flux form c = c' + dt mdot - dt sum_f K_f (omega_c - omega_nb),
so the fuel mass h^3 sum(rho_L alpha + c) changes only by what crosses the
boundary.
Literal species form (species_form = 1, Section 2.5): at the start of the
step the liquid cells (alpha > eps_gas) take omega = omega_sat(T) and
c = rho_G theta omega_sat; the flux at adj uses a central grad(omega)
(interface.raw_evaporation); the species equation (eq. 9) has no mdot
source, the vapour entering the gas by diffusion from the saturated liquid.
This form does not conserve the fuel mass: the liquid loses dt mdot per
step and the assignment sets the liquid's vapour content.
Variable-density gas (gas_density = 1, gas.py): the state also holds the
gas density field rho_G (eq. 24 for the local mixture, consistent with
c, T and alpha).  The interface flux and the vapour advection use the
start-of-step rho_G^n (the vapour flux carries the face value of rho_G
omega); after the advection (T', c') give (omega', rho_G'), which serves
the properties (rho), the species system (m = rho_G' theta/dt, K_f =
D (rho_G' theta)_f/h^2; the Dirichlet faces keep the ambient gas's
2 rho_G D/h^2), the predictor and the pressure; the end of the step gives
(omega^{n+1}, rho_G^{n+1}) from (T^{n+1}, c^{n+1}), and the pressure source
gains -(1 - alpha') ln(rho_G^{n+1}/rho_G')/dt (eq. 7).
"""
from __future__ import annotations

import torch

from . import gas, interface, momentum, operators, thermo, viscous, vof
from . import geo as geometric


def variable_gas(prm):
    return prm.get("gas_density", 0) == 1


def to_state(fields, prm, rho_G=None):
    """Build the oracle state from numpy/torch initial fields (omega given;
    with gas_density = 1 rho_G is eq. 24 at each cell's T and omega)."""
    st = {k: torch.as_tensor(v, dtype=torch.float64).clone() for k, v in fields.items()}
    if variable_gas(prm):
        rho_G = gas.density(st["T"], st["omega"], prm)
        st["rho_G"] = rho_G
    elif rho_G is None:
        rho_G = thermo.gas_density(prm)
    theta = torch.clamp(1.0 - torch.clamp(st["alpha"], 0.0, 1.0), min=prm["theta_min"])
    st["c"] = rho_G * theta * st["omega"]
    return st


def assign_liquid_saturation(st, prm, rho_G):
    """The literal species form's start of step: omega_sat(T) in every liquid
    cell, c = rho_G theta omega there (a new state dict; gas cells unchanged)."""
    om = interface.liquid_saturation(st["alpha"], st["T"], st["omega"], prm)
    theta = torch.clamp(1.0 - torch.clamp(st["alpha"], 0.0, 1.0), min=prm["theta_min"])
    liquid = st["alpha"] > prm["eps_gas"]
    c = torch.where(liquid, rho_G * theta * om, st["c"])
    return dict(st, omega=om, c=c)


def properties(alpha, prm, rho_G):
    """eq. 31 on alpha clamped to [0, 1] (rho_G a constant or a field)."""
    ab = torch.clamp(alpha, 0.0, 1.0)
    rho = ab * prm["rho_L"] + (1.0 - ab) * rho_G
    cp = ab * prm["cp_L"] + (1.0 - ab) * prm["cp_G"]
    k = ab * prm["k_L"] + (1.0 - ab) * prm["k_G"]
    theta = torch.clamp(1.0 - ab, min=prm["theta_min"])
    return ab, rho, cp, k, theta


def evaporation_source(st, prm, rho_G, D_v=None):
    """Steps S1-S4: (mdot, mdot_raw, K, geometry)."""
    if not prm["evaporation"]:
        z = torch.zeros_like(st["alpha"])
        return z, z, torch.zeros((), dtype=torch.float64), None
    if prm.get("species_form", 0) == 1:
        st = assign_liquid_saturation(st, prm, rho_G)
    geo = interface.geometry(st["alpha"], prm)
    mraw = interface.raw_evaporation(st["alpha"], st["T"], st["omega"], st["u"], st["v"], st["w"],
                                     geo, prm, rho_G, D_v=D_v)
    mdot, K = interface.redistribute(mraw, st["alpha"])
    return mdot, mraw, K, geo


def step(st, prm, tol=None, T_amb=None, D_v=None, dh_ev=None, rho_G=None, record=None, solver=None):
    """Advance the state by one step.  Returns (new_state, diagnostics).

    T_amb, D_v, dh_ev may be passed as tensors (for differentiation); they
    default to the parameter values.  record, if a dict, receives the
    intermediate fields of the step.  solver(op, b, x0, tol, maxit) ->
    (x, iters, rel_res, converged) replaces operators.pcg for every linear
    solve of the step (the differentiation form passes one with an implicit
    derivative).
    """
    solve = operators.pcg if solver is None else solver
    prm = dict(prm)
    if dh_ev is not None:
        prm["dh_ev"] = dh_ev
    D = prm["D_v"] if D_v is None else D_v
    Ta = prm["T_amb"] if T_amb is None else T_amb
    tol = prm["tol"] if tol is None else tol
    var = variable_gas(prm)
    if var and prm.get("species_form", 0) == 1:
        raise NotImplementedError("the literal species form is defined for a constant gas density")
    rho_amb = thermo.gas_density(prm, Ta) if rho_G is None else rho_G
    rho_G = st["rho_G"] if var else rho_amb
    dt, h = prm["dt"], prm["h"]
    st_in = st
    literal = prm.get("species_form", 0) == 1
    if literal and prm["evaporation"]:
        st = assign_liquid_saturation(st, prm, rho_G)
    U = [st["u"], st["v"], st["w"]]

    # 1. evaporation flux
    mdot, mraw, K, geo = evaporation_source(st, prm, rho_G, D_v=D)
    # 2. liquid source
    alpha1 = st["alpha"] - dt * mdot / prm["rho_L"]
    # 3. advection: the liquid marker moves with the divergence-free part of u^n
    if prm["liquid_transport"]:
        U_liq, phi, it_phi = momentum.solenoidal_part(U, prm, tol=prm["tol_phi"], solver=solve)
    else:
        U_liq, phi, it_phi = None, None, 0
    if var:   # the vapour flux carries the face value of rho_G omega
        alpha_p, c_p, T_p, B_L, B_v = vof.advect(alpha1, rho_G * st["omega"], st["T"], st["c"], *U, prm, 1.0,
                                                 T_amb=Ta, advect_T=bool(prm["solve_energy"]), U_liq=U_liq)
    else:
        alpha_p, c_p, T_p, B_L, B_v = vof.advect(alpha1, st["omega"], st["T"], st["c"], *U, prm, rho_G,
                                                 T_amb=Ta, advect_T=bool(prm["solve_energy"]), U_liq=U_liq)
    if prm.get("advection", 0) == 1:   # geometric liquid advection (geo.py) in place of the flux-limited one
        alpha_p, out_vol, _ = geometric.advect(alpha1, U_liq if U_liq is not None else U, prm)
        B_L = prm["rho_L"] * out_vol
    # 4. properties (variable gas: rho_G' from the advected T' and c')
    if var:
        theta_p = torch.clamp(1.0 - torch.clamp(alpha_p, 0.0, 1.0), min=prm["theta_min"])
        _, rho_G = gas.invert(T_p, c_p / theta_p, prm)
    ab, rho, cp, k, theta = properties(alpha_p, prm, rho_G)
    diag = {}
    # 5a. energy
    if prm["solve_energy"]:
        m = rho * cp / dt
        op, rb = operators.scalar_system(m, k, 1.0 / (h * h), 2.0 * prm["k_G"] / (h * h), Ta, U, prm)
        b = m * T_p - mdot * prm["dh_ev"] + rb
        T_new, itT, resT, okT = solve(op, b, T_p, tol, prm["maxit"])
    else:
        T_new, itT, resT, okT = st["T"], 0, 0.0, True
    # 5b. species
    mS = rho_G * theta / dt
    KbS = 2.0 * rho_amb * D / (h * h)
    if var:
        opS, _ = operators.scalar_system(mS, rho_G * theta, D / (h * h), KbS, 0.0, U, prm)
    else:
        opS, _ = operators.scalar_system(mS, theta, rho_G * D / (h * h), KbS, 0.0, U, prm)
    msrc = torch.zeros_like(mdot) if literal else mdot
    bS = c_p / dt + msrc
    omega_p = c_p / (rho_G * theta)
    om, itS, resS, okS = solve(opS, bS, omega_p, tol, prm["maxit"])
    face_part = opS.apply(om) - mS * om
    c_new = c_p + dt * msrc - dt * face_part
    # vapour diffused out through ambient (Dirichlet) boundary faces
    B_diff = torch.zeros((), dtype=torch.float64)
    for axis in range(3):
        Ka = torch.movedim(opS.K[axis], axis, 0)
        oa = torch.movedim(om, axis, 0)
        B_diff = B_diff + (Ka[0] * oa[0]).sum() + (Ka[-1] * oa[-1]).sum()
    B_v = B_v + dt * h ** 3 * B_diff
    if var:
        omega_new, rho_new = gas.invert(T_new, c_new / theta, prm)
        S_comp = gas.compressibility_source(ab, rho_new, rho_G, dt)
    else:
        omega_new = c_new / (rho_G * theta)
    # 5c. momentum predictor (and its implicit viscous part, eqs. 5 and 30)
    Us = momentum.predictor(U, ab, rho, prm)
    if prm.get("viscous", 0):
        Us, it_visc, ok_visc = viscous.implicit_viscosity(Us, U, ab, rho, prm, tol, solve)
    else:
        it_visc, ok_visc = [0, 0, 0], True
    # 6. pressure and correction
    beta = 1.0 / rho
    opP = operators.pressure_operator(beta, prm)
    S = mdot * (1.0 / rho_G - 1.0 / prm["rho_L"])
    if var:
        S = S - S_comp
    bP = S - operators.divergence(*Us, h)
    p_new, itP, resP, okP = solve(opP, bP, st["p"], tol, prm["maxit"])
    Un = momentum.project(Us, p_new, rho, prm)

    new = dict(alpha=alpha_p, c=c_new, omega=omega_new, T=T_new, p=p_new, u=Un[0], v=Un[1], w=Un[2])
    if var:
        new["rho_G"] = rho_new
    vol = h ** 3
    diag.update(
        K=float(K), mdot_total=float(vol * mdot.sum()), B_L=float(B_L), B_v=float(B_v),
        volume=float(vol * alpha_p.sum()),
        fuel_mass=float(vol * (prm["rho_L"] * alpha_p + c_new).sum()),
        fuel_mass_before=float(vol * (prm["rho_L"] * st_in["alpha"] + st_in["c"]).sum()),
        alpha_min=float(alpha_p.min()), alpha_max=float(alpha_p.max()),
        n_interface=0 if geo is None else int(geo["icells"].shape[0]),
        iters=dict(T=itT, omega=itS, p=itP, visc=it_visc), res=dict(T=resT, omega=resS, p=resP),
        converged=bool(okT and okS and okP and ok_visc),
    )
    if record is not None:
        record.update(mdot=mdot, mraw=mraw, K=K, geo=geo, alpha1=alpha1, alpha_p=alpha_p, c_p=c_p,
                      T_p=T_p, rho=rho, theta=theta, ustar=Us, bP=bP, rho_G=rho_G,
                      B_L_adv=B_L, B_diff=B_diff, S=S)
        if var:
            record.update(S_comp=S_comp, rho_G_new=rho_new)
    return new, diag


def droplet_volume(st, prm):
    return float(prm["h"] ** 3 * st["alpha"].sum())


def run(fields, prm, steps, tol=None, callback=None):
    """Initial fields -> state after `steps` steps (and per-step diagnostics)."""
    st = to_state(fields, prm)
    diags = []
    for n in range(steps):
        st, d = step(st, prm, tol=tol)
        diags.append(d)
        if callback is not None:
            callback(n, st, d)
    return st, diags
