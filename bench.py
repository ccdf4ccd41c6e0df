"""Throughput of the VOF droplet-evaporation step on one MI355X.

Workload: 256^3 cells over an 8 mm box, 1.0 mm n-heptane droplet in 20 bar
nitrogen at 773 K, Peng-Robinson interface equilibrium, natural convection,
dt = 5e-6 s, seeded +-2% temperature noise.  A step is one full ds_step
(evaporation source, advection, energy/species/pressure solves, projection).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="grid cells per axis (default: the 256^3 workload)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--jacobi", action="store_true", help="Jacobi-PCG pressure solve instead of multigrid")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2005_02867_amd as ds

    prm, run = W.config("C3")
    if args.n != 256:
        prm, run = W.scaled("C3", args.n)
    prm = dict(prm, precision=0 if args.precision == "fp64" else 1, pressure_precond=0 if args.jacobi else 1)
    f = W.initial_fields(prm, **run)
    torch.cuda.set_device(0)
    g = ds.Grid(prm)
    g.set_fields(f)
    print(f"# warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        g.step(1)
    torch.cuda.synchronize()
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    iters = []
    for k in range(args.steps):
        g.step(1)
        d = g.diagnostics()
        iters.append((d["iters_T"], d["iters_omega"], d["iters_p"], d["refinements_p"]))
        print(f"# step {k} iters T/omega/p {iters[-1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    ms = (t1 - t0) * 1e3 / args.steps
    out = {
        "metric": "cell-steps/s at 256^3 (FP32+refine vs FP64), % HBM peak, adjoint/fwd cost",
        "value": ncell * args.steps / (t1 - t0),
        "unit": "cell-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64-refine",
        "data": "synthetic",
        "config": {"workload": f"droplet-evaporation step, {prm['nx']}^3 cells, 8 mm box, 20 bar, "
                               f"Peng-Robinson, natural convection", "cells": ncell,
                   "precision": args.precision, "iters_T_omega_p": iters},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
