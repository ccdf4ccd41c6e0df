"""Throughput of the VOF droplet-evaporation step on one MI355X.

Workload (the 256^3 configuration): 256^3 cells over an 8 mm box, one 1.0 mm
n-heptane droplet in 20 bar nitrogen at 773 K, Peng-Robinson interface
equilibrium, natural convection, dt = 5e-6 s, +-2% seeded temperature noise,
linear-solve tolerance 1e-10.  A step is one full ds_step: evaporation source,
liquid source and advection, energy / species / pressure solves, projection,
diagnostics.  Inputs are resident in HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` is the precision form (FP32 sweeps + FP64
refinement); the all-FP64 step is timed the same way and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
# HBM bytes per launch of the fine-level sweep from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE (separate runs of `bench.py --counters-pass`), each scaled by
# the ratio of known bytes to the counter's reading for a 1 GiB device copy in
# the same run; None until measured for the current kernel.
# Measured for the fine-level coloured sweep of the 256^3 workload: FETCH_SIZE
# 116872 KiB x 2.000 (the 1 GiB copy reads 524339 KiB) + WRITE_SIZE 65536 KiB x 1.000.
TRAFFIC_SMOOTH = (116871.575 * (1048576.0 / 524338.75) + 65536.0 * (1048576.0 / 1048576.0)) * 1024.0


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes per cell of the precision form's kernels (each array a
# kernel streams counted once per launch; FP64 state 8 B, FP32 solver arrays
# 4 B; a coarse level's arrays counted in cells of that level).
EXPLICIT_B = {            # FP64 stages, once per step
    "k_interface_scan": 20,      # alpha read; mraw, adj written
    "k_source": 32,              # alpha, mraw read; mdot, alpha1 written
    "k_div_setup": 32,           # u, v, w read; potential's right-hand side written
    "k_advect": 88,              # alpha1, omega, T, c, u, v, w, phi read; alpha', c', T' written
    "k_energy_setup": 80,        # alpha', T', mdot, u, v, w read; q, diag, b and FP32 q, diag written
    "k_species_setup": 88,       # ... and the warm start omega' written
    "k_species_update": 72,      # alpha', c', mdot, omega, u, v, w read; c, omega written
    "k_predictor": 64,           # alpha', xi, u, v, w read; u*, v*, w* written
    "k_pressure_setup": 80,      # alpha', mdot, u*, v*, w* read; q, diag, b and FP32 q, diag written
    "k_project": 88,             # alpha', p, u*, v*, w* read; u, v, w written; c, T, mdot read for the
                                 # step's diagnostics, taken in the same pass
}
RB_ZERO_B, RB_GEN_B, RB_PROLONG_B = 12, 16, 16.5    # coloured sweeps (r, q [, x, x_coarse] read; x written)
RESTRICT_B = 12.5                                   # r, x, q read; coarse r written
SMOOTH_TWO_B, SMOOTH_B, PROLONG_SMOOTH_B = 12, 16, 16.5
CG_OP_B, CG_OP_CQ_B, CG_UPDATE_B = 44, 40, 28       # FP64 CG with FP32 directions; residual update (+ FP32 r)
RESID64_B, AXPY_B = 36, 20
DIRECT_POTENTIAL_B = 5 * 16 + 16                    # five transform passes; residual check (phi, b read)
INNER_ITER_B = 32 + 24                              # FP32 CG operator + Neumann-polynomial residual update
ROUND_B = 16 + 12 + 24 + 40                         # round start, first z, correction, FP64 residual


def vcycle_bytes(n, const_q):
    """Bytes of one FP32 V-cycle per fine cell: coloured 3+3 sweeps on the
    fine level, damped Jacobi 4+4 on the levels down to 32^3, the levels that
    fit in one workgroup's LDS (16^3 and below) negligible."""
    # from x = 0, two from x, restriction; prolongation with a sweep, two from x
    # (a constant-coefficient level loads no q: 4 B less per sweep)
    fine = RB_ZERO_B + 2 * RB_GEN_B + RESTRICT_B + RB_PROLONG_B + 2 * RB_GEN_B - (24 if const_q else 0)
    coarse = 0.0
    m, frac = n // 2, 1.0 / 8.0
    while m > 16:
        coarse += frac * (SMOOTH_TWO_B + 2 * SMOOTH_B + RESTRICT_B + PROLONG_SMOOTH_B + 3 * SMOOTH_B)
        m //= 2
        frac /= 8.0
    return fine + coarse


def step_bytes_per_cell(n, d):
    """Algorithmic bytes per cell of one precision-form step of an n^3 grid,
    from the kernels' byte table and the step's iteration counts (d: the
    step's diagnostics: iterations of each solve, FP32 rounds of the energy
    and species solves)."""
    b = sum(EXPLICIT_B.values())
    vp, vphi = vcycle_bytes(n, False), vcycle_bytes(n, True)
    b += RESID64_B + vp + d["iters_p"] * (CG_OP_B + CG_UPDATE_B + vp) + AXPY_B
    if d["iters_phi"] == 0:      # the potential by the direct (diagonalised) solve
        b += DIRECT_POTENTIAL_B
    else:
        b += RESID64_B + vphi + d["iters_phi"] * (CG_OP_CQ_B + CG_UPDATE_B + vphi) + AXPY_B
    for it, rounds in ((d["iters_T"], d["rounds_T"]), (d["iters_omega"], d["rounds_omega"])):
        b += RESID64_B + rounds * ROUND_B + it * INNER_ITER_B
    return b


def timed_run(ds, torch, prm, fields, steps, warmup, replays=False):
    """Time `steps` steps after `warmup` (no kernel timing inside the timed
    region); with replays, afterwards time the pressure CG operator and the
    fine-level multigrid sweep replayed back to back on the live system."""
    g = ds.Grid(prm)
    g.set_fields(fields)
    for _ in range(warmup):
        g.step(1)
    iters, mdot, diags = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(1)
        d = g.diagnostics()
        iters.append([d["iters_T"], d["iters_omega"], d["iters_p"], d["refinements_p"], d["iters_phi"]])
        mdot.append(d["mdot_total"])
        diags.append(d)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = g.diagnostics()
    rep = g.time_operator_kernel(50) if replays else None
    rep_s = g.time_kernel(1, 50) if replays else None      # fine-level multigrid sweep
    del g
    torch.cuda.empty_cache()
    return dict(seconds=t1 - t0, iters=iters, replay=rep, replay_smooth=rep_s, volume=d["volume"], diag=d,
                diags=diags, mdot=mdot)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def adjoint_cost(ds, torch, W):
    """Differentiation workload (96^3 over 5 mm, 1 bar / 873 K, 100 steps):
    seconds of the forward run, of ds_forward_record and of the reverse sweep
    (ds_adjoint) with every state stored and with a checkpoint every 10 steps."""
    prm, run = W.config("C4")
    f = W.initial_fields(prm, **run)
    steps = run["steps"]
    out = {"workload": "96^3 over 5 mm, 1.0 mm droplet, 1 bar N2 at 873 K, natural convection, 100 steps of 1e-5 s, "
                       "FP64, J = droplet volume", "steps": steps}
    g = ds.Grid(prm)
    g.set_fields(f)
    g.step(2)                                  # warm-up (kernels loaded, batch sizes settled)
    g.set_fields(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    out["forward_s"] = time.perf_counter() - t0
    del g
    for ckpt in (1, 10):
        g = ds.Grid(prm)
        g.set_fields(f)
        t0 = time.perf_counter()
        g.forward_record(steps, ckpt)
        t1 = time.perf_counter()
        r = g.adjoint(1.0, fields=False)
        t2 = time.perf_counter()
        out[f"ckpt{ckpt}"] = {"record_s": t1 - t0, "reverse_s": t2 - t1,
                              "reverse_over_forward": (t2 - t1) / out["forward_s"],
                              "dV_dD_v": r["D_v"], "dV_ddh_ev": r["dh_ev"], "dV_dT_amb": r["T_amb"]}
        del g
        torch.cuda.empty_cache()
    return out


def other_configs(ds, torch, W, steps=5, warmup=2):
    """Throughput of the other configurations (parity-test cases; not the
    headline): FP64 and precision form, `steps` timed steps after `warmup`."""
    out = {}
    for name in ("C1", "C2", "C4", "C5"):
        prm, run = W.config(name)
        f = W.initial_fields(prm, **run)
        ncell = prm["nx"] * prm["ny"] * prm["nz"]
        res = {"cells": ncell}
        for label, prec in (("fp64", W.PREC_FP64), ("precision_form", W.PREC_MIXED)):
            g = ds.Grid(dict(prm, precision=prec))
            g.set_fields(f)
            g.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            d = g.diagnostics()
            res[label] = {"cell_steps_per_s": ncell * steps / dt, "ms_per_step": dt * 1e3 / steps,
                          "iters_T_omega_p_phi": [d["iters_T"], d["iters_omega"], d["iters_p"], d["iters_phi"]]}
            del g
            torch.cuda.empty_cache()
        out[name] = res
        log(f"  {name} {prm['nx']}^3: FP64 {res['fp64']['ms_per_step']:.2f} ms/step, precision form "
            f"{res['precision_form']['ms_per_step']:.2f} ms/step")
    return out


def adjoint_cost_384(ds, torch, W, steps=100, ckpt=20):
    """Adjoint cost at 384^3 (10 bar, Peng-Robinson, forced 1 m/s, precision
    form), the largest configuration's differentiation shape: reverse sweep
    over `steps` steps with a checkpoint every `ckpt` (100 and 20: a tape of
    about 125 GB), against the forward run of the same steps.  The steps start
    from the initial state (the configuration's 400 forward steps before the
    differentiated window only move the state)."""
    prm, run = W.config("C5")
    f = W.initial_fields(prm, **run)
    g = ds.Grid(prm)
    g.set_fields(f)
    g.step(1)
    g.set_fields(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    del g
    g = ds.Grid(prm)
    g.set_fields(f)
    del f
    tape = ds.tape_bytes(g.h, steps, ckpt)
    log(f"  384^3: forward {fwd:.2f} s for {steps} steps; recording with a {tape / 1e9:.0f} GB tape")
    t0 = time.perf_counter()
    g.forward_record(steps, ckpt)
    t1 = time.perf_counter()
    log(f"  recorded in {t1 - t0:.2f} s; reverse sweep")
    r = g.adjoint(1.0, fields=False)
    t2 = time.perf_counter()
    del g
    torch.cuda.empty_cache()
    return {"workload": f"384^3 over 10 mm, 2.0 mm droplet, 10 bar, Peng-Robinson, forced 1 m/s, precision form, "
                        f"{steps} steps from the initial state, checkpoint every {ckpt}",
            "steps": steps, "ckpt_every": ckpt, "tape_GB": tape / 1e9,
            "forward_s": fwd, "record_s": t1 - t0, "reverse_s": t2 - t1, "reverse_over_forward": (t2 - t1) / fwd,
            "dV_dD_v": r["D_v"], "dV_ddh_ev": r["dh_ev"], "dV_dT_amb": r["T_amb"]}


def cpu_baseline(prm, fields, jacobi_iters_p, sample_iters=8):
    """The CPU oracle (torch float64, host cores) on a bounded sample of the
    same workload: one oracle step from the initial state with its two
    pressure-form Jacobi-PCG solves (pressure and liquid-transport potential)
    stopped after `sample_iters` iterations each; the step time is the
    measured remaining time plus (iterations the two full Jacobi-PCG solves
    need, counted by the GPU's Jacobi-PCG on the same first step) times the
    measured oracle time per such iteration."""
    import torch
    from oracle import operators as O
    from oracle import step as S
    calls = []
    orig = O.pcg

    def pcg(op, b, x0, tol, maxit):
        is_p = op.m is None          # the pressure system has no Helmholtz term
        t = time.perf_counter()
        out = orig(op, b, x0, tol, sample_iters if is_p else maxit)
        calls.append((is_p, time.perf_counter() - t, out[1]))
        return out

    st = S.to_state(fields, prm)
    O.pcg = pcg
    try:
        t0 = time.perf_counter()
        S.step(st, prm)
        t1 = time.perf_counter()
    finally:
        O.pcg = orig
    tp = sum(t for p, t, _ in calls if p)
    ip = sum(i for p, _, i in calls if p)
    t_fixed = (t1 - t0) - tp
    t_iter = tp / max(ip, 1)
    t_step = t_fixed + jacobi_iters_p * t_iter
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    return {
        "value": ncell / t_step, "unit": "cell-steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
        "cpu": cpu_model(), "host_cpus": os.cpu_count(),
        "sample": (f"one oracle step of the {prm['nx']}^3 workload, pressure and potential Jacobi-PCG cut at {ip} "
                   f"iterations in total ({t1 - t0:.1f} s measured: {t_fixed:.1f} s outside those solves, "
                   f"{t_iter:.3f} s per iteration); step time = {t_fixed:.1f} s + {jacobi_iters_p} iterations (the "
                   f"count the same Jacobi-PCG solves take on the GPU) x {t_iter:.3f} s = {t_step:.0f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="cells per axis (256 = the benchmark workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-cost leg")
    ap.add_argument("--configs", action="store_true",
                    help="also time the other configurations (32^3 ... 384^3)")
    ap.add_argument("--no-adjoint-384", action="store_true",
                    help="skip the 384^3 adjoint leg (100 reverse steps, checkpoint every 20, ~125 GB tape)")
    ap.add_argument("--species-literal", action="store_true",
                    help="time the literal species form (the default; kept for older command lines)")
    ap.add_argument("--no-species-literal", action="store_true",
                    help="skip the leg that times the workload in the literal species form (saturated liquid, "
                         "central gradient at adj, no mdot source in the species equation) and compares its "
                         "evaporation rate with the conservative form's")
    ap.add_argument("--no-variable-gas", action="store_true",
                    help="skip the leg that times the workload with the variable-density gas (eq. 24 per cell, "
                         "eq. 7's compressibility term)")
    ap.add_argument("--no-geometric", action="store_true",
                    help="skip the leg that times the workload with the geometric interface advection")
    ap.add_argument("--counters-pass", action="store_true",
                    help="short run for hardware-counter passes: one step of the workload, 5 replayed launches of "
                         "the fine-level sweep, then 3 device copies of 1 GiB (the counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the step runs on one GPU; runs on several GPUs are not supported (the "
                                   "domain is not sharded)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2005_02867_amd as ds

    torch.cuda.set_device(0)
    prm, run = W.config("C3")
    if args.n != 256:
        prm, run = W.scaled("C3", args.n)
    fields = W.initial_fields(prm, **run)
    ncell = prm["nx"] * prm["ny"] * prm["nz"]

    if args.counters_pass:
        g = ds.Grid(dict(prm, precision=W.PREC_MIXED))
        g.set_fields(fields)
        g.step(1)
        r = g.time_kernel(1, 5)
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counters_pass": True, "smooth_avg_us": r["avg_us"], "smooth_bytes": r["bytes_per_launch"],
                          "copy_bytes": 1 << 30}))
        return
    log(f"precision form (FP32 multigrid and FP32 CG rounds, FP64 residuals): warmup {args.warmup}, timing {args.steps} steps")
    mixed = timed_run(ds, torch, dict(prm, precision=W.PREC_MIXED), fields, args.steps, args.warmup, replays=True)
    log(f"  {mixed['seconds'] * 1e3 / args.steps:.2f} ms/step, iters {mixed['iters'][-1]}")
    fp64 = None
    if not args.no_fp64:
        log(f"all-FP64: warmup {args.warmup}, timing {args.steps} steps")
        fp64 = timed_run(ds, torch, dict(prm, precision=W.PREC_FP64), fields, args.steps, args.warmup, replays=True)
        log(f"  {fp64['seconds'] * 1e3 / args.steps:.2f} ms/step, iters {fp64['iters'][-1]}")
    # the liquid-transport potential's share of the step: the same run with the
    # liquid moved by u^n itself (no potential setup and solve)
    log(f"precision form without the liquid-transport potential: warmup {args.warmup}, timing {args.steps} steps")
    nophi = timed_run(ds, torch, dict(prm, precision=W.PREC_MIXED, liquid_transport=0), fields, args.steps,
                      args.warmup)
    ms_mixed = mixed["seconds"] * 1e3 / args.steps
    ms_nophi = nophi["seconds"] * 1e3 / args.steps
    log(f"  {ms_nophi:.2f} ms/step")

    rs = mixed["replay_smooth"]
    rp = mixed["replay"]
    achieved = rs["bytes_per_launch"] / (rs["avg_us"] * 1e-6) / 1e9
    b_step = sum(step_bytes_per_cell(prm["nx"], d) for d in mixed["diags"]) / len(mixed["diags"])
    step_gbs = b_step * ncell / (ms_mixed * 1e-3) / 1e9
    roofline = {
        "kernel": "k_mg_rb_v<float,RB_GEN,false,256,false,false> (fine-level coloured (x-z red-black) sweep of the multigrid "
                  "preconditioner, FP32, reads r, x, q_coef, forms diag from q_coef, writes x: 16 B/cell; the "
                  "largest share of step time)",
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC_SMOOTH,
        "avg_us": rs["avg_us"], "bytes_per_launch": rs["bytes_per_launch"],
        "timing": f"HIP events around {rs['reps']} back-to-back launches on the live pressure system after the "
                  f"timed steps (stream of the launches)",
        "step_bytes_per_cell": b_step, "step_achieved": step_gbs, "step_frac": step_gbs / HBM_PEAK_GBS,
        "step_model": "algorithmic bytes of every kernel of the step (each array a kernel streams counted once per "
                      "launch) summed with the step's own iteration counts and FP32 rounds, over the measured "
                      "ms_per_step",
    }
    ach_op = rp["bytes_per_launch"] / (rp["avg_us"] * 1e-6) / 1e9
    roofline_op = {
        "kernel": "k_cg_dir_spmv_z32_v<false,512,false> (pressure CG operator of the precision form: p = z + beta p with z "
                  "and p in FP32, fused with q = A p and <p,q> in FP64, diag formed from q_coef; 28 B/cell)",
        "bound": "hbm", "achieved": ach_op, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach_op / HBM_PEAK_GBS,
        "avg_us": rp["avg_us"], "bytes_per_launch": rp["bytes_per_launch"],
    }
    out = {
        "metric": "cell-steps/s at 256^3 (FP32+refine vs FP64), % HBM peak, adjoint/fwd cost",
        "value": ncell * args.steps / mixed["seconds"],
        "unit": "cell-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mixed["seconds"] * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64-refine", "data": "synthetic",
        "config": {"workload": f"droplet-evaporation step, {prm['nx']}^3 cells over 8 mm, 20 bar N2 at 773 K, "
                               f"1.0 mm n-heptane droplet, Peng-Robinson equilibrium, natural convection, "
                               f"dt 5e-6 s, tol 1e-10", "cells": ncell,
                   "iters_T_omega_p_rounds_phi": mixed["iters"][-1]},
        "roofline": roofline,
        "roofline_cg_operator": roofline_op,
        "liquid_transport_potential": {
            "ms_per_step_without": ms_nophi, "ms_per_step_share": ms_mixed - ms_nophi,
            "iters_phi": mixed["iters"][-1][4],
            "note": "step time with the liquid moved by u^n itself (no potential setup and solve) against the "
                    "default step"},
    }
    if fp64:
        v64 = ncell * args.steps / fp64["seconds"]
        rp64 = fp64["replay"]
        out["fp64"] = {"value": v64, "ms_per_step": fp64["seconds"] * 1e3 / args.steps,
                       "iters_T_omega_p": fp64["iters"][-1],
                       "operator_kernel_us": rp64["avg_us"],
                       "operator_kernel_GBs": rp64["bytes_per_launch"] / (rp64["avg_us"] * 1e-6) / 1e9}
        out["speedup_mixed_vs_fp64"] = out["value"] / v64
        out["volume_rel_diff_mixed_vs_fp64"] = abs(mixed["volume"] - fp64["volume"]) / fp64["volume"]
    if args.species_literal or not args.no_species_literal:
        log(f"literal species form, precision form: warmup {args.warmup}, timing {args.steps} steps")
        lit = timed_run(ds, torch, dict(prm, precision=W.PREC_MIXED, species_form=1), fields, args.steps,
                        args.warmup)
        log(f"  {lit['seconds'] * 1e3 / args.steps:.2f} ms/step, iters {lit['iters'][-1]}")
        out["species_literal"] = {
            "value": ncell * args.steps / lit["seconds"], "ms_per_step": lit["seconds"] * 1e3 / args.steps,
            "iters_T_omega_p_rounds_phi": lit["iters"][-1],
            "mdot_total_kg_s": lit["mdot"], "mdot_total_conservative_kg_s": mixed["mdot"],
            "step_of_first_timed": args.warmup + 1,
        }
    if not args.no_variable_gas:
        log(f"variable-density gas, precision form: warmup {args.warmup}, timing {args.steps} steps")
        var = timed_run(ds, torch, dict(prm, precision=W.PREC_MIXED, gas_density=1), fields, args.steps,
                        args.warmup)
        log(f"  {var['seconds'] * 1e3 / args.steps:.2f} ms/step, iters {var['iters'][-1]}")
        out["variable_gas"] = {
            "value": ncell * args.steps / var["seconds"], "ms_per_step": var["seconds"] * 1e3 / args.steps,
            "iters_T_omega_p_rounds_phi": var["iters"][-1],
            "mdot_total_kg_s": var["mdot"], "mdot_total_ambient_gas_kg_s": mixed["mdot"],
            "volume_rel_diff_vs_ambient_gas": abs(var["volume"] - mixed["volume"]) / mixed["volume"],
            "note": "the same workload with rho_G from eq. 24 per cell (Peng-Robinson mixture) and eq. 7's "
                    "compressibility term; not the headline configuration, which states constant properties",
        }
    if not args.no_geometric:
        log(f"geometric interface advection, precision form: warmup {args.warmup}, timing {args.steps} steps")
        geo = timed_run(ds, torch, dict(prm, precision=W.PREC_MIXED, advection=1), fields, args.steps, args.warmup)
        log(f"  {geo['seconds'] * 1e3 / args.steps:.2f} ms/step, iters {geo['iters'][-1]}")
        out["geometric_advection"] = {
            "value": ncell * args.steps / geo["seconds"], "ms_per_step": geo["seconds"] * 1e3 / args.steps,
            "iters_T_omega_p_rounds_phi": geo["iters"][-1],
            "volume_rel_diff_vs_flux_limited": abs(geo["volume"] - mixed["volume"]) / mixed["volume"],
            "alpha_min": geo["diag"]["alpha_min"], "alpha_max": geo["diag"]["alpha_max"],
            "note": "the same workload with the liquid advected geometrically (a plane per surface cell, swept "
                    "face areas); not the headline configuration, which prescribes the flux-limited scheme",
        }
    if not args.no_adjoint:
        log("adjoint cost: 96^3, 100 steps")
        out["adjoint"] = adjoint_cost(ds, torch, W)
        log(f"  forward {out['adjoint']['forward_s']:.3f} s, reverse/forward "
            f"{out['adjoint']['ckpt1']['reverse_over_forward']:.2f} (every state stored), "
            f"{out['adjoint']['ckpt10']['reverse_over_forward']:.2f} (checkpoint every 10)")
    if not args.no_adjoint and not args.no_adjoint_384:
        log("adjoint cost at 384^3: 100 steps, checkpoint every 20")
        out["adjoint_384"] = adjoint_cost_384(ds, torch, W)
        log(f"  reverse/forward {out['adjoint_384']['reverse_over_forward']:.2f}")
    if args.configs:
        log("other configurations")
        out["other_configs"] = other_configs(ds, torch, W)
    if not args.no_cpu:
        log("GPU Jacobi-PCG step (pressure iteration count for the CPU extrapolation)")
        g = ds.Grid(dict(prm, precision=W.PREC_FP64, pressure_precond=0))
        g.set_fields(fields)
        g.step(1)
        dj = g.diagnostics()
        jac_iters = dj["iters_p"] + dj["iters_phi"]    # both pressure-form solves, as in the oracle
        del g
        torch.cuda.empty_cache()
        log(f"  {jac_iters} Jacobi-PCG iterations (pressure + liquid-transport potential); CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(prm, fields, jac_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
