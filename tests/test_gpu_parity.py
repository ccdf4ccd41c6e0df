"""GPU (HIP, gfx950) vs CPU oracle, through the C ABI.

FP64 path: every field after every step within 1e-9 relative (per-field
2-norm and element by element against the field's largest magnitude, both
sides solving to 1e-13); integer decisions (interface class, adj
association) bit-exact.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import step as S

pytestmark = pytest.mark.gpu

FIELDS = ("alpha", "T", "omega", "p", "u", "v", "w")
TOL = 1e-9


def _lib():
    import paper_2005_02867_amd as ds
    return ds


def _rel(a, b):
    a = torch.as_tensor(a, dtype=torch.float64).cpu()
    b = torch.as_tensor(b, dtype=torch.float64).cpu()
    nb = float(torch.linalg.vector_norm(b))
    d = float(torch.linalg.vector_norm(a - b))
    return d / nb if nb > 0 else d


def _rel_max(a, b):
    """max |a - b| / max |b| (absolute where b vanishes): the element-wise bar."""
    a = torch.as_tensor(a, dtype=torch.float64).cpu()
    b = torch.as_tensor(b, dtype=torch.float64).cpu()
    nb = float(b.abs().max()) if b.numel() else 0.0
    d = float((a - b).abs().max()) if b.numel() else 0.0
    return d / nb if nb > 0 else d


def _relx(a, b):
    return max(_rel(a, b), _rel_max(a, b))


def _compare(g_fields, st, where, tol=TOL, tol_max=None, fields=FIELDS):
    """Every field within tol relative, both in the 2-norm and element by
    element (max |a - b| <= tol max |b|), so errors confined to small-magnitude
    regions (the alpha band, omega near the droplet, faces at walls) show.
    tol_max: per-field element-wise bars where a case needs its own."""
    errs, bad = {}, {}
    for k in fields:
        e2, em = _rel(g_fields[k], st[k]), _rel_max(g_fields[k], st[k])
        errs[k] = max(e2, em)
        if not (e2 <= tol and em <= (tol_max or {}).get(k, tol)):
            bad[k] = (e2, em)
    assert not bad, f"{where}: {bad} (all: {errs})"
    return errs


def _grid_params(name="C1", n=(17, 19, 23), L=None, **kw):
    prm, run = W.config(name, **kw)
    h = prm["h"] if L is None else L / n[0]
    prm = W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], h=h, x0=None))
    return prm, run


def _run_both(prm, fields, steps, tol_solve=1e-13, check_each=True, tol_max=None):
    ds = _lib()
    prm = dict(prm, tol=tol_solve, tol_phi=tol_solve)
    print(f"case nx={prm['nx']} ny={prm['ny']} nz={prm['nz']} bc={prm['bc_mode']} eq={prm['eq_model']} "
          f"steps={steps}", flush=True)
    g = ds.Grid(prm)
    g.set_fields(fields)
    st = S.to_state(fields, prm)
    worst = {}
    for n in range(steps):
        g.step(1)
        st, d = S.step(st, prm)
        gd = g.diagnostics()
        if check_each or n == steps - 1:
            e = _compare(g.get_fields(), st, f"step {n}", tol_max=tol_max)
            for k, v in e.items():
                worst[k] = max(worst.get(k, 0.0), v)
            assert gd["n_interface"] == d["n_interface"], (gd["n_interface"], d["n_interface"])
            assert gd["K"] == pytest.approx(d["K"], rel=1e-11)
            assert gd["mdot_total"] == pytest.approx(d["mdot_total"], rel=1e-10, abs=1e-30)
            assert gd["volume"] == pytest.approx(d["volume"], rel=1e-12)
    return g, st, worst


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_step_parity_ragged_grid(mode):
    """Ragged 17x19x23 grid (several 256-thread ranges plus a tail), random
    droplet state with flow, 3 steps."""
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0)
    f = W.random_fields(prm, seed=7)
    _run_both(prm, f, steps=3)


def test_step_parity_c1_twenty_steps():
    """Configuration C1 (32^3, natural convection, ideal equilibrium), every
    step of the 20-step run."""
    prm, run = W.config("C1")
    f = W.initial_fields(prm, **run)
    g, st, worst = _run_both(prm, f, steps=run["steps"])
    print("worst relative errors over 20 steps:", worst)


def test_step_parity_peng_robinson():
    """Non-ideal equilibrium (20 bar, Peng-Robinson) on a 24^3 cut of C3."""
    prm, run = W.scaled("C3", 24)
    prm = dict(prm, precision=0)
    f = W.initial_fields(prm, D0=1e-3, seed=1, T_noise=0.02)
    _run_both(prm, f, steps=3)


def test_interface_decisions_bit_exact():
    """Interface class and the int -> adj association agree exactly; the raw
    source agrees to rounding."""
    ds = _lib()
    from oracle import interface as I, thermo as th
    prm, _ = _grid_params(n=(24, 26, 28), L=24 * 1.25e-4)
    f = W.random_fields(prm, seed=3)
    g = ds.Grid(prm)
    g.set_fields(f)
    total, mdot = g.evaporation_rate(return_field=True)
    st = S.to_state(f, prm)
    geo = I.geometry(st["alpha"], prm)
    rho_G = th.gas_density(prm)
    mraw = I.raw_evaporation(st["alpha"], st["T"], st["omega"], st["u"], st["v"], st["w"], geo, prm, rho_G)
    adj_gpu = g.internal(ds.FIELD_ADJ).cpu().numpy().astype(np.int64)
    expect = np.full(adj_gpu.shape, -2, dtype=np.int64)
    ic = geo["icells"].numpy()
    a = st["alpha"].numpy()
    eps = prm["eps_int"]
    band = (a > eps) & (a < 1 - eps)
    expect[band] = -1
    flat = lambda ijk: (ijk[:, 0] * prm["ny"] + ijk[:, 1]) * prm["nz"] + ijk[:, 2]
    found = geo["found"].numpy()
    expect[ic[found, 0], ic[found, 1], ic[found, 2]] = flat(geo["adj"].numpy()[found])
    assert np.array_equal(adj_gpu, expect)
    assert _relx(g.internal(ds.FIELD_MDOT_RAW), mraw) < 1e-12
    mdot_o, K = I.redistribute(mraw, st["alpha"])
    assert _relx(mdot, mdot_o) < 1e-12
    assert total == pytest.approx(prm["h"] ** 3 * float(mdot_o.sum()), rel=1e-12)


def test_solve_pressure_static_droplet():
    """One projection from rest with the centripetal force only."""
    ds = _lib()
    prm, run = W.config("C1", g=(0.0, 0.0, 0.0), evaporation=0, solve_energy=0, tol=1e-13, tol_phi=1e-13)
    f = W.initial_fields(prm, D0=1e-3)
    g = ds.Grid(prm)
    g.set_fields(f)
    it, res = g.solve_pressure()
    assert res <= 1e-13
    new, d = S.step(S.to_state(f, prm), prm)
    out = g.get_fields()
    assert _relx(out["p"], new["p"]) < TOL
    for k in "uvw":
        assert _relx(out[k], new[k]) < 1e-8


def test_determinism_bitwise():
    ds = _lib()
    prm, run = W.config("C1")
    f = W.initial_fields(prm, **run)
    outs = []
    for _ in range(2):
        g = ds.Grid(prm)
        g.set_fields(f)
        g.step(3)
        outs.append(g.get_fields())
    for k in FIELDS:
        assert torch.equal(outs[0][k], outs[1][k]), k


def test_error_paths():
    ds = _lib()
    prm, run = W.config("C1")
    f = W.initial_fields(prm, **run)
    g = ds.Grid(prm)
    with pytest.raises(ds.DSError) as e:
        g.step(1)
    assert e.value.code == ds.DS_ERR_STATE
    g2 = ds.Grid(dict(prm, maxit=1))
    g2.set_fields(f)
    with pytest.raises(ds.NotConverged):
        g2.step(1)
    assert g2.diagnostics()["converged"] == 0
    bad = dict(f)
    bad["T"] = bad["T"].copy()
    bad["T"][3, 4, 5] = float("nan")
    g3 = ds.Grid(prm)
    with pytest.raises(ds.DSError) as e:
        g3.set_fields(bad)
    assert e.value.code == ds.DS_ERR_NONFINITE
    with pytest.raises(ds.DSError):
        ds.create_grid(1, 4, 4, prm)


def test_step_parity_jacobi_pressure():
    """The plain Jacobi-PCG pressure path agrees with the oracle as well."""
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, pressure_precond=0)
    f = W.random_fields(prm, seed=11)
    _run_both(prm, f, steps=2)


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_step_parity_384_thread_row_blocks(precision):
    """48x48x96 grid: a fine-level z-row is 48 FP64 or 24 FP32 vectors, so
    the multigrid CG's stencil kernels run 384-thread blocks of whole rows,
    sharing y neighbours through LDS, and restrict in marching form.  Random
    state with flow, 2 steps, both sides solving to 1e-13."""
    prm, _ = _grid_params(n=(48, 48, 96), L=48 * 1.25e-4, precision=precision)
    f = W.random_fields(prm, seed=5)
    _run_both(prm, f, steps=2)


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_step_parity_coloured_vcycle_sweeps(monkeypatch, precision):
    """The V-cycle's coloured (x-z red-black) sweeps, which by default only
    levels with long marching chunks take (the 256^3 fine level), forced on
    every level that allows them: C1 (32^3, z-rows of 8 or 16 vectors), 5
    steps against the oracle, both sides solving to 1e-13."""
    monkeypatch.setenv("DSVOF_MG_RB_MINPLANES", "1")
    prm, run = W.config("C1", precision=precision)
    f = W.initial_fields(prm, **run)
    g, st, worst = _run_both(prm, f, steps=5)
    print("worst relative errors:", worst, "iterations p/phi:", g.diagnostics()["iters_p"],
          g.diagnostics()["iters_phi"])


@pytest.mark.parametrize("n", [(16, 8, 512), (16, 16, 96)])
def test_step_parity_coloured_sweeps_rows_across_waves(monkeypatch, n):
    """Coloured sweeps (FP32 V-cycle of the precision form) on levels whose
    z-rows span or straddle 64-lane waves (rows of 128 and of 24 vectors),
    where a wave's edge lanes take their z neighbours from the adjacent
    thread through LDS; forced on every level that allows them, 3 steps
    against the oracle, both sides solving to 1e-13."""
    precision = W.PREC_MIXED
    monkeypatch.setenv("DSVOF_MG_RB_MINPLANES", "1")
    prm, _ = _grid_params(n=n, L=n[0] * 1.25e-4, precision=precision)
    f = W.random_fields(prm, seed=9)
    _run_both(prm, f, steps=3)


@pytest.mark.parametrize("n", [(32, 32, 32), (48, 48, 96)])
def test_graph_replays_bitwise_equal_to_eager(monkeypatch, n):
    """The precision form's multigrid CG replays pairs of iterations as HIP
    graphs: every field after every step bit-identical to running the same
    kernels one launch at a time (several solves per step, so each graph is
    replayed many times, with eager work and synchronisations in between)."""
    ds = _lib()
    prm, run = _grid_params(n=n, L=n[0] * 1.25e-4, precision=W.PREC_MIXED)
    f = W.random_fields(prm, seed=3)
    out = {}
    for gr in ("0", "1"):
        monkeypatch.setenv("DSVOF_GRAPHS", gr)
        g = ds.Grid(prm)
        g.set_fields(f)
        out[gr] = []
        for step in range(4):
            g.step(1)
            out[gr].append((g.get_fields(), g.diagnostics()))
        del g
    for step in range(4):
        (fa, da), (fb, db) = out["0"][step], out["1"][step]
        for k in FIELDS:
            assert torch.equal(torch.as_tensor(fa[k]), torch.as_tensor(fb[k])), (step, k)
        assert da["iters_p"] == db["iters_p"] and da["iters_phi"] == db["iters_phi"]
    print("iterations p/phi per step:", [(d["iters_p"], d["iters_phi"]) for _, d in out["1"]])


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_neumann_preconditioner_same_solution_fewer_iterations(monkeypatch, precision):
    """Energy and species on vectorised grids use the first-order Neumann
    polynomial of the Jacobi splitting as preconditioner: the same discrete
    solution as plain Jacobi (both solving to 1e-13), in fewer iterations
    (C1, 3 steps)."""
    ds = _lib()
    prm, run = W.config("C1", precision=precision)
    prm = dict(prm, tol=1e-13, tol_phi=1e-13)
    f = W.initial_fields(prm, **run)
    out = {}
    for nm in (0, 1):
        monkeypatch.setenv("DSVOF_NEUMANN", str(nm))
        g = ds.Grid(prm)
        g.set_fields(f)
        g.step(3)
        out[nm] = (g.get_fields(), g.diagnostics())
        del g
    for k in FIELDS:
        # two solvers each converged to 1e-13: kappa tol apart (2-norm, and 10x that element-wise)
        assert _rel(out[1][0][k], out[0][0][k]) <= 1e-11, k
        assert _rel_max(out[1][0][k], out[0][0][k]) <= 1e-10, k
    d0, d1 = out[0][1], out[1][1]
    print("iterations T/omega, Jacobi:", d0["iters_T"], d0["iters_omega"], "Neumann:", d1["iters_T"], d1["iters_omega"])
    assert d1["iters_omega"] < d0["iters_omega"] and d1["iters_T"] <= d0["iters_T"]


@pytest.mark.parametrize("precond", [1, 0])
def test_step_parity_mixed_precision_refined(precond):
    """Precision form to 1e-13 reaches the FP64 discrete solution: same 1e-9
    bar against the oracle on C1, 10 steps.  Multigrid pressure: FP64 CG with
    the FP32 V-cycle; Jacobi pressure (and the energy and species systems):
    FP32 CG rounds with FP64 residuals and updates."""
    prm, run = W.config("C1", precision=W.PREC_MIXED, pressure_precond=precond)
    f = W.initial_fields(prm, **run)
    g, st, worst = _run_both(prm, f, steps=10)
    d = g.diagnostics()
    assert d["iters_p"] > 0
    if precond == 0:
        assert d["refinements_p"] >= 1


def test_precision_form_volume_after_200_steps():
    """Precision form at the configuration tolerance (1e-10): droplet volume
    after 200 steps within 1e-6 relative of the FP64 GPU path (96^3 cut of
    the 20 bar Peng-Robinson case)."""
    ds = _lib()
    prm, run = W.scaled("C3", 96)
    f = W.initial_fields(prm, **run)
    vols = {}
    for prec in (W.PREC_FP64, W.PREC_MIXED):
        print(f"precision {prec}: 200 steps at 96^3", flush=True)
        g = ds.Grid(dict(prm, precision=prec))
        g.set_fields(f)
        g.step(200)
        vols[prec] = g.droplet_volume()
        d = g.diagnostics()
        rel = abs(d["fuel_mass"] - d["fuel_mass_before"] + d["B_L"] + d["B_v"]) / d["fuel_mass_before"]
        assert rel <= 1e-10, rel
    rel = abs(vols[W.PREC_MIXED] - vols[W.PREC_FP64]) / vols[W.PREC_FP64]
    print("volume FP64", vols[W.PREC_FP64], "mixed", vols[W.PREC_MIXED], "rel", rel)
    assert rel <= 1e-6


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FARFIELD])
def test_step_parity_literal_species_form(mode):
    """Literal species form (saturated liquid, central grad(omega) at adj, no
    mdot source in eq. 9) on the ragged 17x19x23 grid with flow, 3 steps,
    every field and the fuel mass against the oracle."""
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, bc_mode=mode, species_form=1)
    f = W.random_fields(prm, seed=13)
    g, st, worst = _run_both(prm, f, steps=3)
    gd = g.diagnostics()
    st_o = S.to_state(f, dict(prm, tol=1e-13, tol_phi=1e-13))
    for _ in range(3):
        st_o, d = S.step(st_o, dict(prm, tol=1e-13, tol_phi=1e-13))
    assert gd["fuel_mass"] == pytest.approx(d["fuel_mass"], rel=1e-10)
    assert gd["fuel_mass_before"] == pytest.approx(d["fuel_mass_before"], rel=1e-10)
    print("worst relative errors:", worst)


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_step_parity_literal_species_peng_robinson(precision):
    """Literal species form with the Peng-Robinson equilibrium assigned to
    every liquid cell (20 bar, a 24^3 cut of the 256^3 workload's box with a
    2 mm droplet, six cells across: a three-cell droplet has only diagonal
    adj cells, whose face neighbours miss the liquid), 3 steps, both
    precision forms."""
    prm, run = W.scaled("C3", 24)
    prm = dict(prm, precision=precision, species_form=1)
    f = W.initial_fields(prm, D0=2e-3, seed=2, T_noise=0.02)
    _run_both(prm, f, steps=3)


def test_literal_species_evaporation_rate_and_assignment():
    """ds_evaporation_rate in the literal form: the liquid's omega equals the
    oracle's saturation values (gas cells untouched), the raw source and
    mdot agree to rounding, adj decisions bit-exact."""
    ds = _lib()
    from oracle import interface as I, thermo as th
    prm, _ = _grid_params(n=(24, 26, 28), L=24 * 1.25e-4, species_form=1)
    f = W.random_fields(prm, seed=4)
    g = ds.Grid(prm)
    g.set_fields(f)
    total, mdot = g.evaporation_rate(return_field=True)
    rho_G = th.gas_density(prm)
    st = S.assign_liquid_saturation(S.to_state(f, prm), prm, rho_G)
    liquid = st["alpha"] > prm["eps_gas"]
    assert bool(liquid.any())
    om_g = torch.as_tensor(g.get_fields()["omega"], dtype=torch.float64).cpu()
    assert _relx(om_g[liquid], st["omega"][liquid]) < 1e-13
    assert torch.equal(om_g[~liquid], torch.as_tensor(f["omega"], dtype=torch.float64)[~liquid])
    geo = I.geometry(st["alpha"], prm)
    mraw = I.raw_evaporation(st["alpha"], st["T"], st["omega"], st["u"], st["v"], st["w"], geo, prm, rho_G)
    assert _relx(g.internal(ds.FIELD_MDOT_RAW), mraw) < 1e-12
    mdot_o, K = I.redistribute(mraw, st["alpha"])
    assert _relx(mdot, mdot_o) < 1e-12
    assert total == pytest.approx(prm["h"] ** 3 * float(mdot_o.sum()), rel=1e-12)


def test_literal_species_form_rejected_by_the_adjoint():
    ds = _lib()
    prm, run = W.config("C1", species_form=1)
    f = W.initial_fields(prm, **run)
    g = ds.Grid(prm)
    g.set_fields(f)
    tape = torch.empty(ds.tape_bytes(g.h, 2, 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(ds.DSError) as e:
        ds.forward_record(g.h, 2, 1, tape)
    assert e.value.code == ds.DS_ERR_ARG


def test_step_parity_literal_species_droplet_at_the_wall():
    """Literal species form with the droplet's band reaching the x- wall
    (24^3, centre 0.6 mm from it): adj cells on the box face take the
    zero-gradient ghost in the central difference, and marches that leave
    the box give no source.  3 steps against the oracle."""
    n = 24
    h = 1.25e-4
    prm, _ = W.config("C1", species_form=1)
    prm = W.finalize(dict(prm, nx=n, ny=n, nz=n, h=h, x0=(0.6e-3, n * h / 2, n * h / 2)))
    f = W.initial_fields(prm, D0=1.0e-3, seed=3, T_noise=0.01)
    _run_both(prm, f, steps=3)


def test_step_parity_literal_species_without_evaporation():
    """Literal species form with evaporation off: nothing is assigned to the
    liquid and there is no source; 2 steps against the oracle."""
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, species_form=1, evaporation=0)
    f = W.random_fields(prm, seed=17)
    _run_both(prm, f, steps=2)


def test_step_parity_zero_species_right_hand_side_precision_form():
    """No evaporation and no vapour: the species system's right-hand side is
    exactly zero, so its solve returns x = 0 (and r = 0) from the start; in
    the precision form the first FP32 round is enqueued without a host test
    and must leave omega at zero.  3 steps of C1 against the oracle."""
    prm, run = W.config("C1", precision=W.PREC_MIXED, evaporation=0)
    f = W.initial_fields(prm, **run)
    assert float(np.abs(f["omega"]).max()) == 0.0
    g, st, worst = _run_both(prm, f, steps=3)
    assert float(g.get_fields()["omega"].abs().max()) == 0.0


@pytest.mark.parametrize("n,fill,form", [((12, 13, 14), 0.0, 0), ((12, 13, 14), 1.0, 0), ((12, 13, 14), 1.0, 1),
                                         ((2, 3, 5), None, 0), ((2, 2, 2), None, 0)])
def test_step_parity_degenerate_inputs(n, fill, form):
    """Degenerate inputs: no liquid anywhere (no interface cell, K = 0), the
    box full of liquid (theta at its floor everywhere; liquid leaves through
    the open faces, both species forms), and the smallest grids (every
    kernel on its non-vectorised path).  2 steps against the oracle."""
    prm, _ = _grid_params(n=n, L=n[0] * 1.25e-4, species_form=form)
    f = W.random_fields(prm, seed=21)
    if fill is not None:
        f["alpha"] = np.full_like(f["alpha"], fill)
    # all liquid: theta sits at its floor 1e-8 in every cell, so the species system's
    # diagonal is 1e8 times smaller than in gas and omega = c/(rho_G theta) magnifies the
    # rounding of c 1e8-fold cell by cell; omega and c (the conserved variable, compared
    # below) get an element-wise bar of 1e-8, the 2-norm keeps 1e-9
    full = fill == 1.0
    g, st, _ = _run_both(prm, f, steps=2, tol_max={"omega": 1e-8} if full else None)
    ds = _lib()
    c = g.internal(ds.FIELD_C)
    assert _rel(c, st["c"]) <= TOL and _rel_max(c, st["c"]) <= (1e-8 if full else TOL)


def test_constant_coefficient_sweep_matches_the_loading_sweep(monkeypatch):
    """The liquid-transport potential's coloured sweeps take its constant q
    (1/dt rounded to FP32, the value its array holds) from a register: the
    same arithmetic as loading it.  C1 in the precision form with coloured
    sweeps on every level that takes them, 3 steps with and without
    (DSVOF_CONST_Q=0): equal potential iteration counts, fields within 1e-13."""
    ds = _lib()
    monkeypatch.setenv("DSVOF_MG_RB_MINPLANES", "1")
    monkeypatch.setenv("DSVOF_PHI_DIRECT", "0")       # the potential by its multigrid CG
    prm, run = W.config("C1", precision=W.PREC_MIXED)
    f = W.initial_fields(prm, **run)
    out = []
    for cq in ("1", "0"):
        monkeypatch.setenv("DSVOF_CONST_Q", cq)
        g = ds.Grid(dict(prm, tol=1e-13, tol_phi=1e-13))
        g.set_fields(f)
        its = []
        for _ in range(3):
            g.step(1)
            its.append(g.diagnostics()["iters_phi"])
        out.append((g.get_fields(), its))
    assert out[0][1] == out[1][1], (out[0][1], out[1][1])
    assert out[0][1][-1] > 0           # the multigrid CG ran (the first step starts from rest: no work)
    for k in FIELDS:
        assert _rel(out[0][0][k], out[1][0][k]) <= 1e-13, k
        assert _rel_max(out[0][0][k], out[1][0][k]) <= 1e-12, k


def test_step_parity_round_tests_on_the_host(monkeypatch):
    """The energy and species FP32 rounds with their start and inner solves
    tested on the host (DSVOF_ROUND_TEST=0, the schedule before one test per
    round): C1 in the precision form, 5 steps against the oracle."""
    monkeypatch.setenv("DSVOF_ROUND_TEST", "0")
    prm, run = W.config("C1", precision=W.PREC_MIXED)
    f = W.initial_fields(prm, **run)
    _run_both(prm, f, steps=5)


def test_step_parity_forced_convection_64cubed():
    """A 64^3 cut of the forced-convection configuration (6 mm box, 1.5 mm
    droplet, 0.5 m/s inflow at z-, gravity on, ideal equilibrium, dt 5e-6 s):
    every field after each of 20 steps against the oracle, both at 1e-13."""
    prm, run = W.scaled("C2", 64)
    f = W.initial_fields(prm, **run)
    g, st, worst = _run_both(prm, f, steps=20)
    d = g.diagnostics()
    print("worst relative errors over 20 steps:", worst, "max |w|", float(st["w"].abs().max()))
    assert d["mdot_total"] > 0 and float(st["w"].abs().max()) >= 0.5


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_step_parity_direct_potential_grid(mode):
    """A ragged grid whose extents the potential's direct solve takes
    (24x32x18), random droplet state with flow, 3 steps against the oracle."""
    prm, _ = _grid_params(n=(24, 32, 18), L=24 * 1.25e-4, bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0)
    f = W.random_fields(prm, seed=21)
    g, st, worst = _run_both(prm, f, steps=3)
    assert g.diagnostics()["iters_phi"] == 0


@pytest.mark.parametrize("mode", [W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD])
def test_step_parity_viscous(mode):
    """Implicit viscous momentum (div mu (grad v + grad v^T) of eqs. 5 and 30,
    mu mixed by eq. 31): the ragged 17x19x23 grid with a random droplet state
    and flow, 3 steps against the oracle in the three boundary modes."""
    prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4, bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0,
                          viscous=1)
    f = W.random_fields(prm, seed=31)
    g, st, worst = _run_both(prm, f, steps=3)
    d = g.diagnostics()
    print("viscous iterations", d["iters_visc"], "residual", d["res_visc"])
    assert d["iters_visc"] > 0 and d["res_visc"] <= 1e-13


def test_step_parity_viscous_precision_form_32cubed():
    """The 32^3 configuration with viscosity in the precision form (the viscous
    solve itself FP64), 5 steps against the oracle; the adjoint rejects the
    viscous step."""
    ds = _lib()
    prm, run = W.config("C1", viscous=1, precision=W.PREC_MIXED)
    f = W.initial_fields(prm, **run)
    g, st, worst = _run_both(prm, f, steps=5)
    print("worst relative errors over 5 steps:", worst)
    with pytest.raises(ds.DSError) as e:
        g.forward_record(2, 1)
    assert e.value.code == ds.DS_ERR_ARG


@pytest.mark.parametrize("case", ["ragged", "C1"])
def test_step_diagnostics_match_the_fields(case):
    """The step's closing diagnostics, computed in the projection's pass,
    against the same quantities taken from the state the step leaves, summed
    with torch in FP64: h^3 sum(alpha) (and the handle's own volume reduction,
    a separate kernel), h^3 sum(rho_L alpha + c) and h^3 sum(mdot) to 1e-12,
    alpha's extremes exactly; three steps on a ragged grid and of the C1
    droplet."""
    ds = _lib()
    if case == "ragged":
        prm, _ = _grid_params(n=(17, 19, 23), L=17 * 1.25e-4)
        f = W.random_fields(prm, seed=21)
    else:
        prm, run = W.config("C1")
        f = W.initial_fields(prm, **run)
    print(f"step diagnostics against the fields: {case}", flush=True)
    g = ds.Grid(prm)
    g.set_fields(f)
    h3 = prm["h"] ** 3
    for n in range(3):
        g.step(1)
        d = g.diagnostics()
        a = g.get_fields()["alpha"].double()
        c = g.internal(ds.FIELD_C)
        mdot = g.internal(ds.FIELD_MDOT)
        assert d["volume"] == pytest.approx(h3 * float(a.sum()), rel=1e-12), n
        assert d["volume"] == pytest.approx(g.droplet_volume(), rel=1e-13), n
        assert d["fuel_mass"] == pytest.approx(h3 * float((prm["rho_L"] * a + c).sum()), rel=1e-12), n
        assert d["mdot_total"] == pytest.approx(h3 * float(mdot.sum()), rel=1e-12,
                                                abs=1e-12 * h3 * float(mdot.abs().sum())), n
        assert d["alpha_min"] == float(a.min()) and d["alpha_max"] == float(a.max()), n
