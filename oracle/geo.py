"""Geometric interface advection (Section 2.1, eq. 3: the paper advects alpha
with isoAdvector, a geometric scheme).

Test infrastructure: the CPU oracle only.

Reading (advection = 1).  The paper names the scheme and gives none of its
steps; the isoAdvector idea is taken with a planar interface per cell:
* surface cells are those with tol < alpha < 1 - tol, tol = 1e-8;
* in a surface cell the interface is the plane n.x = s (cell-local
  coordinates, corner at the origin, x in [0, h]^3), n = -grad(alpha)/
  |grad(alpha)| from central differences (a ghost outside the box repeats
  its neighbour, so a box face does not tilt the plane), so that the liquid
  is n.x <= s; s makes the liquid volume alpha h^3 (bisection on the exact
  volume function);
* during the step the plane moves along n with the normal speed U_n = U_c.n
  of the cell-centre velocity (the mean of the cell's two face velocities
  per axis): s(t) = s + U_n t;
* the liquid volume through a face in the step is U_f times the time
  integral over the step of the face area the donor (upwind) cell's plane
  submerges (isoAdvector's face flux); a donor that is not a surface cell
  gives U_f h^2 dt alpha; inflow through a box face carries no liquid;
* alpha' = alpha1 - (1/h^3) sum of the outgoing minus incoming volumes (no
  bounding step: the update stays exactly conservative).
Exact integration: the submerged area of a face is quadratic in the plane
offset between the offsets at which the plane passes the face's corners, and
the cut volume of a cell cubic between those of its corners; both are
integrated piecewise with Simpson's rule, which is exact for quadratics.
With |grad(alpha)| = 0 a surface cell gives U_f h^2 dt alpha.
"""
from __future__ import annotations

import numpy as np
import torch

SURF_TOL = 1e-8


def face_area(sig, a, b, h):
    """Area of {(y, z) in [0, h]^2 : a y + b z <= sig} for a >= b >= 0."""
    sig, a, b = np.broadcast_arrays(np.asarray(sig, float), np.asarray(a, float), np.asarray(b, float))
    out = np.empty(sig.shape)
    flat = a < 1e-12                  # plane parallel to the face
    out[flat] = np.where(sig[flat] > 0.0, h * h, 0.0)
    one = ~flat & (b == 0.0)
    out[one] = h * np.clip(sig[one] / a[one], 0.0, h)
    two = ~flat & ~one
    s2, a2, b2 = sig[two], a[two], b[two]
    zA = np.clip((s2 - a2 * h) / b2, 0.0, h)   # below zA the whole y-row is submerged
    zB = np.clip(s2 / b2, 0.0, h)              # above zB nothing is
    out[two] = h * zA + (zB - zA) * (s2 - 0.5 * b2 * (zA + zB)) / a2
    return out


def face_area_n(sig, ny, nz, h):
    """Area of {(y, z) in [0, h]^2 : ny y + nz z <= sig} for any signs."""
    sig = np.asarray(sig, float) - np.minimum(ny, 0.0) * h - np.minimum(nz, 0.0) * h
    p, q = np.abs(ny), np.abs(nz)
    return face_area(sig, np.maximum(p, q), np.minimum(p, q), h)


def _simpson_pieces(f, t0, t1, breaks):
    """Integral of f over [t0, t1] (arrays), f quadratic between the sorted
    break points (columns of `breaks`, clipped into [t0, t1])."""
    pts = np.concatenate([t0[:, None], np.clip(breaks, t0[:, None], t1[:, None]), t1[:, None]], axis=1)
    pts = np.sort(pts, axis=1)
    total = np.zeros(t0.shape)
    for k in range(pts.shape[1] - 1):
        lo, hi = pts[:, k], pts[:, k + 1]
        w = hi - lo
        total += w / 6.0 * (f(lo) + 4.0 * f(0.5 * (lo + hi)) + f(hi))
    return total


def cell_volume(s, n, h):
    """Volume of {x in [0, h]^3 : n.x <= s} (n: (..., 3), any signs)."""
    s = np.asarray(s, float)
    n = np.asarray(n, float)
    sp = s - np.minimum(n, 0.0).sum(axis=-1) * h
    c = np.sort(np.abs(n), axis=-1)[..., ::-1]          # c1 >= c2 >= c3 >= 0
    c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2]
    # V = int_0^h A(sp - c1 x; c2, c3) dx, A quadratic between the x where
    # sp - c1 x crosses 0, c3 h, c2 h, (c2 + c3) h
    sp1, c1f, c2f, c3f = (x.reshape(-1) for x in np.broadcast_arrays(sp, c1, c2, c3))
    brk = np.stack([(sp1 - v) / c1f for v in (0.0 * c1f, c3f * h, c2f * h, (c2f + c3f) * h)], axis=1)
    f = lambda x: face_area(sp1 - c1f * x, c2f, c3f, h)
    zero = np.zeros(sp1.shape)
    V = _simpson_pieces(f, zero, zero + h, brk)
    # a plane normal to an axis: the face area is a step in x; a slab
    slab = c2f < 1e-12
    V[slab] = h * h * np.clip(sp1[slab] / c1f[slab], 0.0, h)
    return V.reshape(np.shape(sp))


def plane_offset(alpha, n, h, iters=200):
    """s with cell_volume(s, n, h) = alpha h^3 (bisection)."""
    alpha = np.asarray(alpha, float)
    n = np.asarray(n, float)
    lo = np.minimum(n, 0.0).sum(axis=-1) * h
    hi = np.maximum(n, 0.0).sum(axis=-1) * h
    target = alpha * h ** 3
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.all((mid == lo) | (mid == hi)):
            break
        up = cell_volume(mid, n, h) > target
        hi = np.where(up, mid, hi)
        lo = np.where(up, lo, mid)
    return 0.5 * (lo + hi)


def swept_area(sig0, un, ny, nz, h, dt):
    """int_0^dt of the submerged area of a face whose plane offset (in the
    face's coordinates) moves as sig0 + un t."""
    sig0, un, ny, nz = (np.asarray(x, float) for x in (sig0, un, ny, nz))
    sh = sig0 - np.minimum(ny, 0.0) * h - np.minimum(nz, 0.0) * h
    p, q = np.abs(ny), np.abs(nz)
    a, b = np.maximum(p, q), np.minimum(p, q)
    moving = un != 0.0
    brk = np.full(sig0.shape + (4,), -1.0)                # outside [0, dt]: ignored
    for k, v in enumerate((0.0 * a, b * h, a * h, (a + b) * h)):
        brk[moving, k] = (v[moving] - sh[moving]) / un[moving]
    f = lambda t: face_area(sh + un * t, a, b, h)
    zero = np.zeros(sig0.shape)
    out = _simpson_pieces(f, zero, zero + dt, brk)
    # a plane parallel to the face: the face is wholly submerged while the offset is positive
    flat = a < 1e-12
    if flat.any():
        s0, u = sh[flat], un[flat]
        tc = np.where(u != 0.0, -s0 / np.where(u != 0.0, u, 1.0), 0.0)
        wet = np.where(u > 0.0, dt - np.clip(tc, 0.0, dt), np.where(u < 0.0, np.clip(tc, 0.0, dt),
                                                                     np.where(s0 > 0.0, dt, 0.0)))
        out[flat] = h * h * wet
    return out


def _grad(alpha, h):
    a = torch.nn.functional.pad(alpha[None, None], (1, 1, 1, 1, 1, 1), mode="replicate")[0, 0].numpy()
    gx = (a[2:, 1:-1, 1:-1] - a[:-2, 1:-1, 1:-1]) / (2.0 * h)
    gy = (a[1:-1, 2:, 1:-1] - a[1:-1, :-2, 1:-1]) / (2.0 * h)
    gz = (a[1:-1, 1:-1, 2:] - a[1:-1, 1:-1, :-2]) / (2.0 * h)
    return np.stack([gx, gy, gz], axis=-1)


def reconstruct(alpha, h):
    """Planes of the surface cells: (mask, n (nx,ny,nz,3), s)."""
    a = alpha.numpy()
    g = _grad(alpha, h)
    gm = np.sqrt((g * g).sum(axis=-1))
    surf = (a > SURF_TOL) & (a < 1.0 - SURF_TOL) & (gm > 0.0)
    n = np.zeros(a.shape + (3,))
    n[surf] = -g[surf] / gm[surf][:, None]
    s = np.zeros(a.shape)
    s[surf] = plane_offset(a[surf], n[surf], h)
    return surf, n, s


def liquid_face_volumes(alpha, U, prm, planes=None):
    """Liquid volume through every face during dt, signed along +axis, for
    face velocities U (3 arrays, box faces included).  Returns 3 arrays."""
    h, dt = prm["h"], prm["dt"]
    a = alpha.numpy()
    surf, n, s = reconstruct(alpha, h) if planes is None else planes
    Un = [u.numpy() for u in U]
    uc = np.stack([0.5 * (Un[0][1:] + Un[0][:-1]), 0.5 * (Un[1][:, 1:] + Un[1][:, :-1]),
                   0.5 * (Un[2][:, :, 1:] + Un[2][:, :, :-1])], axis=-1)
    unrm = (uc * n).sum(axis=-1)   # normal speed of the plane (surface cells)
    out = []
    for ax in range(3):
        uf = np.moveaxis(Un[ax], ax, 0)            # (n_ax + 1, ...)
        am = np.moveaxis(a, ax, 0)
        sm = np.moveaxis(surf, ax, 0)
        nm = np.moveaxis(n, ax, 0)
        ssm = np.moveaxis(s, ax, 0)
        unm = np.moveaxis(unrm, ax, 0)
        N = am.shape[0]
        dV = np.zeros(uf.shape)
        # donor of face f: cell f-1 (flow in +ax) or f (flow in -ax); box inflow carries none
        for f in range(N + 1):
            u = uf[f]
            fwd = u > 0.0
            lo_ok = f >= 1
            hi_ok = f <= N - 1
            don = np.where(fwd, f - 1, f)
            valid = np.where(fwd, lo_ok, hi_ok) & (u != 0.0)
            if not valid.any():
                continue
            d = np.clip(don, 0, N - 1)
            idx = np.indices(u.shape)
            ad = np.where(valid, am[d, idx[0], idx[1]], 0.0)
            sd = np.where(valid, sm[d, idx[0], idx[1]], False)
            vol = u * h * h * dt * ad
            if sd.any():
                nn = nm[d, idx[0], idx[1]][sd]       # (m, 3): the normals' components in grid-axis order
                n_ax = nn[:, ax]
                oth = [q for q in range(3) if q != ax]
                xf = np.where(fwd[sd], h, 0.0)      # the face is the donor's high (flow +) or low side
                sig0 = ssm[d, idx[0], idx[1]][sd] - n_ax * xf
                sw = swept_area(sig0, unm[d, idx[0], idx[1]][sd], nn[:, oth[0]], nn[:, oth[1]], h, dt)
                vol[sd] = u[sd] * sw
            dV[f] = np.where(valid, vol, 0.0)
        out.append(torch.as_tensor(np.moveaxis(dV, 0, ax), dtype=torch.float64))
    return out


def advect(alpha1, U, prm):
    """alpha' and the liquid volume that left the box during dt."""
    h = prm["h"]
    dV = liquid_face_volumes(alpha1, U, prm)
    div = (dV[0][1:] - dV[0][:-1]) + (dV[1][:, 1:] - dV[1][:, :-1]) + (dV[2][:, :, 1:] - dV[2][:, :, :-1])
    out_box = (dV[0][-1].sum() - dV[0][0].sum()) + (dV[1][:, -1].sum() - dV[1][:, 0].sum()) + \
              (dV[2][:, :, -1].sum() - dV[2][:, :, 0].sum())
    return alpha1 - div / h ** 3, out_box, dV
