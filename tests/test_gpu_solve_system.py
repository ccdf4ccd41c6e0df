"""The step's linear systems solved one at a time through ds_solve_system.

* 8^3, every system (pressure eq. 7, energy eq. 8, species eq. 9, the
  liquid-transport potential) in the three boundary modes: the GPU solve of
  A x = b matches numpy.linalg.solve on the matrix assembled column by column
  from the oracle's matrix-free operator for the same state, to 1e-12.
* 17x19x23 (ragged: several tiles and a tail), FP64 and the precision form:
  the GPU solve at tol 1e-13 matches the oracle's PCG solve at 1e-15, to
  1e-10 (2-norm and element-wise), from a zero start and from a warm start
  (the solution perturbed by 10%); the residual reported is the true one.
* The state is untouched: fields are bitwise unchanged, and a step afterwards
  equals the step of a handle that never solved a system, bit for bit.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O
from oracle import step as S
from oracle import thermo as th

pytestmark = pytest.mark.gpu

MODES = (W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD)


def _lib():
    import paper_2005_02867_amd as ds
    return ds


def _prm(n, mode, **kw):
    prm, _ = W.config("C1", bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0, **kw)
    return W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], h=1.25e-4, x0=None))


def _oracle_ops(prm, f):
    """The operators the step assembles, with the state's alpha as alpha'."""
    st = S.to_state(f, prm)
    rho_G = th.gas_density(prm)
    ab, rho, cp, k, theta = S.properties(st["alpha"], prm, rho_G)
    U = [st["u"], st["v"], st["w"]]
    h, dt = prm["h"], prm["dt"]
    ds = _lib()
    return {
        ds.SYS_PRESSURE: O.pressure_operator(1.0 / rho, prm),
        ds.SYS_ENERGY: O.scalar_system(rho * cp / dt, k, 1 / h ** 2, 2 * prm["k_G"] / h ** 2, prm["T_amb"], U, prm)[0],
        ds.SYS_SPECIES: O.scalar_system(rho_G * theta / dt, theta, rho_G * prm["D_v"] / h ** 2,
                                        2 * rho_G * prm["D_v"] / h ** 2, 0.0, U, prm)[0],
        ds.SYS_POTENTIAL: O.pressure_operator(torch.full_like(rho, 1.0 / dt), prm),
    }


def _dense(op, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for j in range(n):
        e = torch.zeros(n, dtype=torch.float64)
        e[j] = 1.0
        A[:, j] = op.apply(e.reshape(shape)).ravel().numpy()
    return A


def _err(a, b):
    a = torch.as_tensor(a, dtype=torch.float64).cpu().ravel()
    b = torch.as_tensor(b, dtype=torch.float64).cpu().ravel()
    return max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)),
               float((a - b).abs().max() / b.abs().max()))


@pytest.mark.parametrize("mode", MODES)
def test_dense_solve_8cubed(mode):
    ds = _lib()
    prm = _prm((8, 8, 8), mode, tol=1e-14, tol_phi=1e-14)
    f = W.random_fields(prm, seed=3)
    print(f"8^3 mode {mode}: dense solves", flush=True)
    g = ds.Grid(prm)
    g.set_fields(f)
    rng = np.random.default_rng(9)
    shape = (8, 8, 8)
    for which, op in _oracle_ops(prm, f).items():
        A = _dense(op, shape)
        b = rng.standard_normal(512)
        x_ref = np.linalg.solve(A, b)
        x, it, res = g.solve_system(which, torch.tensor(b).reshape(shape))
        e = _err(x, x_ref)
        print(f"  system {which}: {it} iterations, residual {res:.2e}, error vs dense {e:.2e}")
        # the potential takes the direct (diagonalised) solve at 8^3: no iterations
        assert (it == 0 if which == ds.SYS_POTENTIAL else it > 0) and res <= 1e-14
        assert e < 1e-12, (which, e)


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
@pytest.mark.parametrize("mode", MODES)
def test_ragged_grid_against_oracle_pcg(mode, prec):
    ds = _lib()
    prm = _prm((17, 19, 23), mode, tol=1e-13, tol_phi=1e-13, precision=prec)
    f = W.random_fields(prm, seed=5)
    print(f"17x19x23 mode {mode} precision {prec}", flush=True)
    g = ds.Grid(prm)
    g.set_fields(f)
    rng = np.random.default_rng(1)
    shape = (17, 19, 23)
    for which, op in _oracle_ops(prm, f).items():
        b = torch.tensor(rng.standard_normal(shape))
        x_ref, it_ref, res_ref, ok = O.pcg(op, b, torch.zeros(shape, dtype=torch.float64), 1e-15, 20000)
        assert ok
        for start in ("zero", "warm"):
            # warm: the solution perturbed by 10% per cell, like a step's warm start
            x0 = None if start == "zero" else x_ref * (1.0 + 0.1 * torch.tensor(rng.uniform(-1, 1, shape)))
            x, it, res = g.solve_system(which, b, x0)
            e = _err(x, x_ref)
            r_true = float(torch.linalg.vector_norm(b - op.apply(x.cpu())) / torch.linalg.vector_norm(b))
            print(f"  system {which} ({start} start): {it} iterations (oracle {it_ref}), residual {res:.2e} "
                  f"(oracle's recomputation {r_true:.2e}), error {e:.2e}")
            assert it >= 0 and res <= 1e-13
            assert abs(res - r_true) <= 0.1 * max(res, r_true) + 1e-15   # the reported residual is the true one
            assert e < 1e-10, (which, start, e)


def test_far_start_reports_true_residual():
    """A start 1e11 times the solution (energy system: x ~ b dt/(rho cp)):
    the recursively updated residual meets the tolerance, the true one cannot
    (rounding of the first residual, ~eps ||A x0||); the call reports the true
    residual and DS_ERR_NOT_CONVERGED, or converges for real."""
    ds = _lib()
    prm = _prm((17, 19, 23), W.BC_NATURAL, tol=1e-13, tol_phi=1e-13)
    f = W.random_fields(prm, seed=5)
    g = ds.Grid(prm)
    g.set_fields(f)
    rng = np.random.default_rng(1)
    shape = (17, 19, 23)
    op = _oracle_ops(prm, f)[ds.SYS_ENERGY]
    b = torch.tensor(rng.standard_normal(shape))
    x0 = torch.tensor(rng.standard_normal(shape))
    try:
        x, it, res = g.solve_system(ds.SYS_ENERGY, b, x0)
        converged = True
    except ds.NotConverged as e:
        converged = False
        print("not converged:", e)
    if converged:
        r_true = float(torch.linalg.vector_norm(b - op.apply(x.cpu())) / torch.linalg.vector_norm(b))
        print("converged: reported", res, "true", r_true)
        assert res <= 1e-13 and abs(res - r_true) <= 0.1 * max(res, r_true) + 1e-15


def test_state_untouched_by_system_solves():
    ds = _lib()
    prm = _prm((17, 19, 23), W.BC_NATURAL, tol=1e-13, tol_phi=1e-13)
    f = W.random_fields(prm, seed=8)
    g = ds.Grid(prm)
    g.set_fields(f)
    ref = ds.Grid(prm)
    ref.set_fields(f)
    before = {k: v.clone() for k, v in g.get_fields().items()}
    rng = np.random.default_rng(2)
    for which in (ds.SYS_PRESSURE, ds.SYS_ENERGY, ds.SYS_SPECIES, ds.SYS_POTENTIAL):
        g.solve_system(which, torch.tensor(rng.standard_normal((17, 19, 23))))
    after = g.get_fields()
    for k in before:
        assert torch.equal(before[k], after[k]), k
    g.step(1)
    ref.step(1)
    a, b = g.get_fields(), ref.get_fields()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    with pytest.raises(ds.DSError) as e:
        g.solve_system(7, torch.zeros((17, 19, 23)))
    assert e.value.code == ds.DS_ERR_ARG


@pytest.mark.parametrize("mode", MODES)
def test_potential_direct_solve_against_oracle(mode):
    """The liquid-transport potential on grids whose extents allow the direct
    (diagonalised) solve: 24x32x18 (radices 3, 2, 4; the forced inlet mirrors
    z to 36) and 96x64x48.  The direct solve reports 0 iterations, its true
    residual is at rounding level, and it matches the oracle's PCG at 1e-15."""
    ds = _lib()
    rng = np.random.default_rng(4)
    for n in ((24, 32, 18), (96, 64, 48)):
        prm = _prm(n, mode, tol=1e-13, tol_phi=1e-13)
        f = W.random_fields(prm, seed=6)
        print(f"{n} mode {mode}: direct potential solve", flush=True)
        g = ds.Grid(prm)
        g.set_fields(f)
        op = _oracle_ops(prm, f)[ds.SYS_POTENTIAL]
        b = torch.tensor(rng.standard_normal(n))
        x_ref, it_ref, _, ok = O.pcg(op, b, torch.zeros(n, dtype=torch.float64), 1e-15, 40000)
        assert ok
        x, it, res = g.solve_system(ds.SYS_POTENTIAL, b)
        e = _err(x, x_ref)
        print(f"  iterations {it} (oracle {it_ref}), residual {res:.2e}, error {e:.2e}")
        assert it == 0 and res <= 1e-13
        assert e < 1e-10


@pytest.mark.parametrize("mode", MODES)
def test_potential_direct_and_multigrid_steps_agree(mode, monkeypatch):
    """Three steps on a grid the direct solve takes, once with it and once with
    the multigrid CG (DSVOF_PHI_DIRECT=0, read when the handle is created),
    both at 1e-13: every field agrees to 1e-10 (2-norm and element-wise)."""
    ds = _lib()
    prm = _prm((24, 32, 18), mode, tol=1e-13, tol_phi=1e-13)
    f = W.random_fields(prm, seed=12)
    out, iters = [], []
    for direct in ("1", "0"):
        monkeypatch.setenv("DSVOF_PHI_DIRECT", direct)
        g = ds.Grid(prm)
        g.set_fields(f)
        g.step(3)
        out.append(g.get_fields())
        iters.append(g.diagnostics()["iters_phi"])
    print("potential iterations, direct / multigrid:", iters)
    assert iters[0] == 0 and iters[1] > 0
    for k in out[0]:
        assert _err(out[0][k], out[1][k]) < 1e-10, k


@pytest.mark.parametrize("mode", MODES)
def test_potential_direct_solve_many_groups(mode, monkeypatch):
    """128x128x96: more line groups per pass (768 along x and y, 1024 z-line
    blocks; 1536 for the forced inlet's mirrored z) than the direct solve's
    persistent workgroups, so each workgroup transforms several groups with
    the next one's loads in flight.  0 iterations, the true residual (the
    FP64 operator, not the transforms) at rounding level, and the solution
    equal to the multigrid CG's (DSVOF_PHI_DIRECT=0, residual 1e-13) to 1e-8:
    the CG's error is bounded by its residual times the condition number,
    about (2 N / pi)^2 = 6.6e3 here."""
    ds = _lib()
    n = (128, 128, 96)
    prm = _prm(n, mode, tol=1e-13, tol_phi=1e-13)
    f = W.random_fields(prm, seed=8)
    b = torch.tensor(np.random.default_rng(5).standard_normal(n))
    out = []
    for direct in ("1", "0"):
        monkeypatch.setenv("DSVOF_PHI_DIRECT", direct)
        print(f"{n} mode {mode}: potential, direct solve {direct}", flush=True)
        g = ds.Grid(prm)
        g.set_fields(f)
        x, it, res = g.solve_system(ds.SYS_POTENTIAL, b)
        print(f"  iterations {it}, residual {res:.2e}")
        assert res <= 1e-13
        assert (it == 0) == (direct == "1")
        out.append(x)
        del g
    assert _err(out[0], out[1]) < 1e-8


@pytest.mark.parametrize("mode", MODES)
def test_species_warm_start_correction(mode, monkeypatch):
    """ds_step starts the species solve from omega' plus the previous step's
    solve correction (omega~ - omega'); DSVOF_EXTRAP=0 starts from omega'
    alone.  Five steps of the C1 droplet (a forced or far-field box in the
    other modes) at tolerance 1e-13 both ways: every field agrees to 1e-9
    (2-norm and element-wise), and the corrected start takes no more species
    iterations in total."""
    ds = _lib()
    prm, run = W.config("C1", bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0, tol=1e-13, tol_phi=1e-13)
    f = W.initial_fields(prm, **run)
    out, its = [], []
    for ex in ("1", "0"):
        monkeypatch.setenv("DSVOF_EXTRAP", ex)
        g = ds.Grid(prm)
        g.set_fields(f)
        n_it = 0
        for _ in range(5):
            g.step(1)
            n_it += g.diagnostics()["iters_omega"]
        out.append(g.get_fields())
        its.append(n_it)
    print(f"mode {mode}: species iterations over 5 steps, corrected / plain start: {its}")
    assert its[0] <= its[1]
    for k in out[0]:
        assert _err(out[0][k], out[1][k]) < 1e-9, k


@pytest.mark.parametrize("precision", [W.PREC_MIXED, W.PREC_FP64])
@pytest.mark.parametrize("case", ["C1-natural", "C1-forced", "C1-farfield", "C2-64"])
def test_overlapped_pressure_is_bit_identical(case, precision, monkeypatch):
    """With the multigrid pressure, ds_step runs the predictor and the
    pressure solve on a second stream, on the pressure's own arrays, while the
    energy and species solves run on the caller's stream (DSVOF_OVERLAP=0: all
    on one stream, on the shared arrays); with the direct potential solve the
    potential runs on the second stream too, beside the evaporation source.
    The stages touch disjoint data, so five steps give every field bit for
    bit the same, with the same iteration counts, budget terms (B_L, B_v,
    fuel mass) and potential residual, in both precision forms; the 64^3 cut
    of the forced-convection configuration takes several batches of pressure
    iterations per step."""
    ds = _lib()
    name, tag = case.split("-")
    if name == "C1":
        mode = {"natural": W.BC_NATURAL, "forced": W.BC_FORCED, "farfield": W.BC_FARFIELD}[tag]
        prm, run = W.config("C1", bc_mode=mode, w_in=0.2 if mode == W.BC_FORCED else 0.0, precision=precision)
        f = W.initial_fields(prm, **run)
    else:
        prm, run = W.config("C2", precision=precision)
        prm = W.finalize(dict(prm, nx=64, ny=64, nz=64, h=6e-3 / 64, x0=None))
        f = W.initial_fields(prm, D0=run["D0"])
    out, its = [], []
    for ov in ("1", "0"):
        monkeypatch.setenv("DSVOF_OVERLAP", ov)
        print(f"{case} precision {precision}: overlap {ov}", flush=True)
        g = ds.Grid(prm)
        g.set_fields(f)
        n_it = []
        for _ in range(5):
            g.step(1)
            d = g.diagnostics()
            n_it.append((d["iters_T"], d["iters_omega"], d["iters_p"], d["B_L"], d["B_v"], d["fuel_mass"],
                         d["iters_phi"], d["res_phi"]))
        out.append({k: v.cpu() for k, v in g.get_fields().items()})
        its.append(n_it)
        del g
    print("iterations T/omega/p, B_L, B_v, fuel mass, potential iterations and residual per step, overlapped:",
          its[0])
    assert its[0] == its[1]
    # the potential's residual is reported (the first step's u^0 = 0 gives b = 0 and a zero residual)
    res_phi = [t[-1] for t in its[0]]
    assert all(0.0 <= r <= prm["tol_phi"] for r in res_phi) and max(res_phi) > 0.0, res_phi
    for k in out[0]:
        assert torch.equal(out[0][k], out[1][k]), k
