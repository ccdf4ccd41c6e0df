"""Pins of the liquid transport velocity (interface advection, Section 2.1, eq. 3).

The oracle moves the liquid marker with U_s = U - G phi, the discretely
divergence-free part of the face velocities, where D G phi = D U with the
pressure's boundary kinds: phi = 0 half a cell outside open faces, no flux
through walls and the forced inlet.  The pins below fix it independently of
the oracle's own operators:
* a Helmholtz split built by hand, U = U_df + G psi with U_df divergence-free
  (integer stream function, exact in binary) and G written out here with the
  boundary kinds above, must come back as U_s = U_df and phi = psi -- a sign
  error, a transposed face, or a wrong boundary kind (zero gradient instead of
  the phi = 0 ghost) moves phi away from psi;
* the discrete divergence of U_s vanishes to the solve tolerance;
* a divergence-free U is returned unchanged, bit for bit;
* wall and inlet normal velocities are never touched.
Each runs in all three boundary modes on a ragged grid.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import momentum as M

MODES = (W.BC_NATURAL, W.BC_FORCED, W.BC_FARFIELD)


def _prm(mode, n=(9, 10, 11)):
    prm, _ = W.config("C1", bc_mode=mode, w_in=0.25 if mode == W.BC_FORCED else 0.0)
    return W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], x0=None))


def _div(u, v, w, h):
    """Discrete divergence, written out: (sum of outflows)/h per cell."""
    return ((u[1:] - u[:-1]) + (v[:, 1:] - v[:, :-1]) + (w[:, :, 1:] - w[:, :, :-1])) / h


def _stream_field(shape, seed, w0):
    """Divergence-free faces: an integer stream function in the x-y plane
    (zero on the lateral box faces, so no flow through them) plus a uniform
    w0 through every z-plane; scaled by 2^-10 so every sum is exact."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    psi = rng.integers(-8, 9, (nx + 1, ny + 1, nz)).astype(np.float64)
    psi[0], psi[-1], psi[:, 0], psi[:, -1] = 0.0, 0.0, 0.0, 0.0
    s = 2.0 ** -10
    u = s * (psi[:, 1:, :] - psi[:, :-1, :])
    v = -s * (psi[1:, :, :] - psi[:-1, :, :])
    w = np.full((nx, ny, nz + 1), w0)
    return [torch.tensor(a) for a in (u, v, w)]


def _open_faces(mode):
    """(axis, side) -> face is open (phi = 0 ghost); the others carry no flux."""
    out = {}
    for a in range(3):
        for s in range(2):
            if mode == W.BC_FARFIELD:
                out[(a, s)] = True
            elif a < 2:
                out[(a, s)] = False                      # outer walls
            else:
                out[(a, s)] = (s == 1) or mode == W.BC_NATURAL   # z+ outlet; z- open unless forced inlet
    return out


def _grad(psi, h, mode):
    """Face gradient of a cell potential: interior (psi_R - psi_L)/h; open box
    faces against psi = 0 at h/2 outside; walls and inlet 0."""
    opn = _open_faces(mode)
    out = []
    for a in range(3):
        p = torch.movedim(psi, a, 0)
        g = torch.zeros((p.shape[0] + 1,) + tuple(p.shape[1:]), dtype=torch.float64)
        g[1:-1] = (p[1:] - p[:-1]) / h
        if opn[(a, 0)]:
            g[0] = (p[0] - 0.0) / (0.5 * h)
        if opn[(a, 1)]:
            g[-1] = (0.0 - p[-1]) / (0.5 * h)
        out.append(torch.movedim(g, 0, a))
    return out


@pytest.mark.parametrize("mode", MODES)
def test_helmholtz_split_recovered(mode):
    prm = _prm(mode)
    shape = (prm["nx"], prm["ny"], prm["nz"])
    h = prm["h"]
    Udf = _stream_field(shape, 3, prm["w_in"] if mode == W.BC_FORCED else 0.125)
    rng = np.random.default_rng(7)
    psi = torch.tensor(rng.uniform(-1, 1, shape)) * 1e-5
    G = _grad(psi, h, mode)
    U = [Udf[a] + G[a] for a in range(3)]
    assert float(_div(*Udf, h).abs().max()) == 0.0
    Us, phi, it = M.solenoidal_part(U, prm, tol=1e-14)
    assert it > 0
    scale = max(float(g.abs().max()) for g in G)
    for a in range(3):
        err = float((Us[a] - Udf[a]).abs().max()) / scale
        assert err < 1e-11, (a, err)
    assert float((phi - psi).abs().max()) / float(psi.abs().max()) < 1e-11


@pytest.mark.parametrize("mode", MODES)
def test_divergence_of_transport_velocity_vanishes(mode):
    prm = _prm(mode)
    f = W.random_fields(prm, seed=11)
    U = [torch.tensor(f[k]) for k in ("u", "v", "w")]
    h = prm["h"]
    d0 = float(_div(*U, h).abs().max())
    assert d0 > 0.0
    Us, phi, it = M.solenoidal_part(U, prm, tol=1e-13)
    d1 = float(_div(*Us, h).abs().max())
    assert d1 <= 1e-12 * d0, (d1, d0)
    # idempotent: the divergence-free part of U_s is U_s
    Us2, _, _ = M.solenoidal_part(Us, prm, tol=1e-13)
    for a in range(3):
        assert float((Us2[a] - Us[a]).abs().max()) <= 1e-11 * float(Us[a].abs().max())


@pytest.mark.parametrize("mode", MODES)
def test_divergence_free_field_unchanged_bitwise(mode):
    prm = _prm(mode)
    shape = (prm["nx"], prm["ny"], prm["nz"])
    U = _stream_field(shape, 5, prm["w_in"] if mode == W.BC_FORCED else -0.0625)
    assert float(_div(*U, prm["h"]).abs().max()) == 0.0
    Us, phi, it = M.solenoidal_part(U, prm, tol=1e-13)
    assert it == 0 and float(phi.abs().max()) == 0.0
    for a in range(3):
        assert torch.equal(Us[a], U[a])


@pytest.mark.parametrize("mode", MODES)
def test_wall_and_inlet_normal_faces_untouched(mode):
    prm = _prm(mode)
    f = W.random_fields(prm, seed=4)
    U = [torch.tensor(f[k]) for k in ("u", "v", "w")]
    Us, _, _ = M.solenoidal_part(U, prm, tol=1e-13)
    opn = _open_faces(mode)
    n_fixed = 0
    for a in range(3):
        Ua, Sa = torch.movedim(U[a], a, 0), torch.movedim(Us[a], a, 0)
        for s, idx in ((0, 0), (1, -1)):
            if not opn[(a, s)]:
                assert torch.equal(Sa[idx], Ua[idx])
                n_fixed += 1
            else:
                assert not torch.equal(Sa[idx], Ua[idx])     # open faces take the correction
    assert n_fixed == {W.BC_NATURAL: 4, W.BC_FORCED: 5, W.BC_FARFIELD: 0}[mode]
    if mode == W.BC_FORCED:
        assert bool((Us[2][:, :, 0] == prm["w_in"]).all())
