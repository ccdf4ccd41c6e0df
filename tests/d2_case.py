"""Setup of the d^2-law case shared by the oracle and GPU pins: isothermal
droplet, zero gravity, no centripetal force, far-field boundaries, and the
quasi-steady Stefan reference rate with the cube's capacitance."""
import json
import math
import os

import workloads as W
from oracle import thermo as th

HERE = os.path.dirname(os.path.abspath(__file__))


def d2_case(n, T=300.0, L=4e-3, D0=1e-3):
    prm, _ = W.config("C1", g=(0.0, 0.0, 0.0), xi0=0.0, bc_mode=W.BC_FARFIELD, solve_energy=0,
                      T_amb=T, T_liq=T, tol=1e-10)
    prm = W.finalize(dict(prm, nx=n, ny=n, nz=n, h=L / n, x0=None))
    rho_G = th.gas_density(prm)
    ws = float(th.mass_fraction(th.equilibrium_y(T, prm), prm))
    B = ws / (1.0 - ws)
    Kd2 = 8.0 * rho_G * prm["D_v"] * math.log(1.0 + B) / prm["rho_L"]
    vs = prm["rho_L"] / rho_G * Kd2 / (4.0 * D0)          # Stefan velocity scale
    prm["dt"] = min(0.25 * prm["h"] / vs, 2e-4)
    cap = json.load(open(os.path.join(HERE, "golden", "cube_capacitance.json")))
    assert cap["L"] == L and cap["a"] == 0.5 * D0
    kappa = 1.0 - 1.0 / cap["ratio"]

    def box_ratio(a):          # C_box/C_inf for a sphere of radius a (image term scales with a)
        return 1.0 / (1.0 - kappa * a / cap["a"])

    def mdot_qs(a):
        return 4.0 * math.pi * rho_G * prm["D_v"] * a * math.log(1.0 + B) * box_ratio(a)

    return prm, dict(rho_G=rho_G, B=B, Kd2=Kd2, box_ratio=box_ratio, mdot_qs=mdot_qs, D0=D0)
