"""A/B of the liquid transport velocity on the CPU oracle (not collected by pytest).

Interface advection (Section 2.1, eq. 3) moves the liquid marker with the
velocity field.  The step can take either
  liquid_transport = 0: the full start-of-step face velocity u^n, or
  liquid_transport = 1: its discretely divergence-free part u^n - G phi
                        (D G phi = D u^n, the pressure's boundary kinds).
The Stefan expansion makes D u^n = mdot (1/rho_G - 1/rho_L) inside the
diffuse interface band, so with the full velocity the band's own dilatation
carries liquid outward through algebraic face fluxes.  This script runs both
variants of the oracle for 300 steps at 24^3 on two cases and records
alpha_max, the droplet volume and the d^2 slope:
  * the 32^3 configuration's physics (1 bar N2 at 773 K, 1.0 mm droplet,
    gravity, natural convection, dt 1e-5 s) on a 24^3 grid over the same 4 mm box;
  * the isothermal d^2-law case (300 K, 1 bar, no gravity, far field) at 24^3,
    whose slope is compared with the capacitance-corrected quasi-steady value.

    python tests/ab_liquid_transport.py      # ~3 min; writes tests/golden/ab_liquid_transport.json
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import workloads as W                    # noqa: E402
from oracle import step as S             # noqa: E402
from tests.d2_case import d2_case        # noqa: E402

STEPS = 300


def _run(prm, fields, steps):
    st = S.to_state(fields, prm)
    t, d2, amax, vol = [], [], [], []
    for k in range(steps):
        st, d = S.step(st, prm)
        t.append((k + 1) * prm["dt"])
        d2.append((6.0 * d["volume"] / math.pi) ** (2.0 / 3.0))
        amax.append(d["alpha_max"])
        vol.append(d["volume"])
    t, d2 = np.array(t), np.array(d2)
    half = steps // 2
    A = np.polyfit(t[half:], d2[half:], 1)
    resid = d2[half:] - np.polyval(A, t[half:])
    R2 = 1.0 - resid.var() / d2[half:].var()
    return dict(alpha_max=[amax[0], amax[steps // 3], amax[2 * steps // 3], amax[-1]],
                alpha_max_steps=[1, steps // 3 + 1, 2 * steps // 3 + 1, steps],
                volume_first=vol[0], volume_last=vol[-1], d2_slope=float(-A[0]), d2_R2=float(R2))


def main():
    out = {"steps": STEPS, "cases": {}}
    prm, run = W.scaled("C1", 24)
    f = W.initial_fields(prm, **run)
    prm_d2, ref = d2_case(24)
    f_d2 = W.initial_fields(prm_d2, D0=ref["D0"])
    for case, (p, fl) in {"c1_physics_24cubed": (prm, f), "d2_300K_24cubed": (prm_d2, f_d2)}.items():
        res = {}
        for lt in (0, 1):
            t0 = time.time()
            r = _run(dict(p, liquid_transport=lt), fl, STEPS)
            r["seconds"] = time.time() - t0
            if case.startswith("d2"):
                a_mid = 0.5 * math.sqrt((6.0 * r["volume_last"] / math.pi) ** (2.0 / 3.0))
                r["d2_slope_over_quasi_steady"] = r["d2_slope"] / (ref["Kd2"] * ref["box_ratio"](a_mid))
            res[f"liquid_transport_{lt}"] = r
            print(case, lt, json.dumps(r), flush=True)
        out["cases"][case] = res
    path = os.path.join(HERE, "golden", "ab_liquid_transport.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
