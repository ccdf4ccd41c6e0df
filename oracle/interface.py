"""Interface geometry and evaporation source (paper Section 2.4).

Test infrastructure: the CPU oracle only.

Readings of the paper taken here (each listed in the design notes):
* |grad alpha| (eq. 15) from central differences of alpha, with alpha = 0
  outside the box (alpha = 0 on every boundary, boundary-condition table).
* "Interface cells" (where |grad alpha| is nonzero, text after eq. 16) are the
  cells with eps < alpha < 1 - eps.  Gas cells have alpha <= eps.
* The association of each interface cell with "the closest gas cell along the
  interface normal" (text after eq. 16, algorithm unspecified in the paper):
  march s = 1, 2, ..., s_max cell lengths along n = -grad alpha/|grad alpha|
  from the cell centre; the target cell is floor(i + 1/2 + s n_i) per axis;
  the first target with alpha <= eps is adj.  Leaving the box or running out
  of steps leaves the cell without adj (no source).  Evaluated in index
  units with every product and sum rounded separately, in this order.
* Flux at adj (eqs. 12-14) for the binary fuel/N2 gas: the mole-fraction
  form of eq. 12 equals Fick's law -rho_G D grad(omega) for two species, so
  j.n = rho_G D (omega_sat - omega_adj)/d + rho_G omega_adj (v_adj . n), with
  d the distance between the interface and adj cell centres, omega_sat the
  saturation value at the interface cell temperature (Section 2.5) and
  v_adj the cell-centred average of the staggered velocities at adj.
* eq. 17: mdot_raw = (j.n) |grad alpha|_int, positive for evaporation.
* eqs. 19-21: mdot = K f(alpha) mdot_raw with f = sqrt(alpha(1-alpha)) and K
  the ratio of the two volume integrals (sums over all cells); K = 0 when the
  denominator vanishes.
* Literal species form (species_form = 1, Section 2.5 after eq. 23): the
  saturation value is assigned to the whole liquid (every cell with
  alpha > eps_gas, the cells the adj march passes over) and the diffusive
  part of j.n at adj is -rho_G D (grad omega)_adj . n, grad omega by central
  differences of that field with zero-gradient ghosts outside the box.
The geometry stays differentiable in alpha (|grad alpha| and the normal);
classes, the march and adj are integer decisions and carry no derivative.
"""
from __future__ import annotations

import torch

from . import thermo

GAS, INTERFACE, LIQUID = 0, 1, 2


def central_differences(alpha):
    """alpha(i+1) - alpha(i-1) per axis (index units), zero ghosts."""
    a = torch.nn.functional.pad(alpha[None, None], (1, 1, 1, 1, 1, 1), value=0.0)[0, 0]
    dx = a[2:, 1:-1, 1:-1] - a[:-2, 1:-1, 1:-1]
    dy = a[1:-1, 2:, 1:-1] - a[1:-1, :-2, 1:-1]
    dz = a[1:-1, 1:-1, 2:] - a[1:-1, 1:-1, :-2]
    return dx, dy, dz


def geometry(alpha, prm):
    """Classes, |grad alpha|, normals and the interface -> adj association.

    Returns a dict with
      cls      (nx,ny,nz) int: GAS / INTERFACE / LIQUID
      gradmag  (nx,ny,nz) |grad alpha| in 1/m
      icells   (m,3) int64 indices of interface cells with a nonzero gradient
      normal   (m,3) unit normal n = -grad alpha/|grad alpha|
      adj      (m,3) int64 indices of adj (-1 rows where none was found)
      dist     (m,) centre distance int -> adj in m (0 where none)
    """
    eps = prm["eps_int"]
    eps_gas = prm.get("eps_gas", eps)
    h = prm["h"]
    shape = alpha.shape
    dx, dy, dz = central_differences(alpha)
    sq = (dx * dx + dy * dy) + dz * dz
    # sqrt written so that a zero gradient has a zero (not NaN) derivative
    norm = torch.where(sq > 0.0, torch.sqrt(torch.where(sq > 0.0, sq, torch.ones_like(sq))),
                       torch.zeros_like(sq))
    gradmag = norm / (2.0 * h)
    cls = torch.full(shape, INTERFACE, dtype=torch.int64)
    cls[alpha <= eps] = GAS
    cls[alpha >= 1.0 - eps] = LIQUID
    sel = (cls == INTERFACE) & (norm > 0.0)
    icells = torch.nonzero(sel)
    nrm = norm[sel]
    normal = torch.stack([-dx[sel] / nrm, -dy[sel] / nrm, -dz[sel] / nrm], dim=1)
    m = icells.shape[0]
    adj = torch.full((m, 3), -1, dtype=torch.int64)
    found = torch.zeros(m, dtype=torch.bool)
    stopped = torch.zeros(m, dtype=torch.bool)
    base = icells.to(torch.float64) + 0.5
    upper = torch.tensor(shape, dtype=torch.int64)
    for s in range(1, prm["s_max"] + 1):
        target = torch.floor(base + float(s) * normal).to(torch.int64)
        inside = ((target >= 0) & (target < upper)).all(dim=1)
        active = ~found & ~stopped
        stopped |= active & ~inside
        t = torch.where(inside[:, None], target, torch.zeros_like(target))
        is_gas = alpha[t[:, 0], t[:, 1], t[:, 2]] <= eps_gas
        hit = active & inside & is_gas
        adj[hit] = target[hit]
        found |= hit
    diff = (adj - icells).to(torch.float64)
    dist = torch.where(found, h * torch.sqrt((diff * diff).sum(dim=1)), torch.zeros(m, dtype=torch.float64))
    return dict(cls=cls, gradmag=gradmag, icells=icells, normal=normal, adj=adj,
                found=found, dist=dist)


def cell_velocity(u, v, w):
    """Cell-centred average of the staggered face velocities."""
    return 0.5 * (u[:-1] + u[1:]), 0.5 * (v[:, :-1] + v[:, 1:]), 0.5 * (w[:, :, :-1] + w[:, :, 1:])


def liquid_saturation(alpha, T, omega, prm):
    """omega with the saturation value omega_sat(T) assigned to every liquid
    cell (alpha > eps_gas), as the paper's species equation takes it (Section
    2.5, after eq. 23); gas cells keep their value."""
    liquid = alpha > prm["eps_gas"]
    out = omega.clone()
    if bool(liquid.any()):
        out[liquid] = thermo.saturation_omega(T[liquid], prm)
    return out


def omega_gradient(omega, h):
    """Central-difference grad(omega) per axis, zero-gradient ghosts outside
    the box (a ghost takes its neighbouring cell's value)."""
    o = torch.nn.functional.pad(omega[None, None], (1, 1, 1, 1, 1, 1), mode="replicate")[0, 0]
    gx = (o[2:, 1:-1, 1:-1] - o[:-2, 1:-1, 1:-1]) / (2.0 * h)
    gy = (o[1:-1, 2:, 1:-1] - o[1:-1, :-2, 1:-1]) / (2.0 * h)
    gz = (o[1:-1, 1:-1, 2:] - o[1:-1, 1:-1, :-2]) / (2.0 * h)
    return gx, gy, gz


def raw_evaporation(alpha, T, omega, u, v, w, geo, prm, rho_G, D_v=None):
    """mdot_raw (kg m^-3 s^-1) on the grid; zero off the interface (eq. 17).

    species_form 1 (literal): omega must already hold the liquid's saturation
    values (liquid_saturation); the diffusive flux at adj is then
    -rho_G D (grad omega)_adj . n instead of the two-point difference."""
    D = prm["D_v"] if D_v is None else D_v
    mraw = torch.zeros_like(alpha)
    ic, adj, found = geo["icells"], geo["adj"], geo["found"]
    if ic.shape[0] == 0 or not bool(found.any()):
        return mraw
    ic = ic[found]
    aj = adj[found]
    n = geo["normal"][found]
    d = geo["dist"][found]
    T_int = T[ic[:, 0], ic[:, 1], ic[:, 2]]
    w_sat = thermo.saturation_omega(T_int, prm)
    w_adj = omega[aj[:, 0], aj[:, 1], aj[:, 2]]
    if isinstance(rho_G, torch.Tensor) and rho_G.dim() == 3:   # variable gas: rho_G at adj
        rho_G = rho_G[aj[:, 0], aj[:, 1], aj[:, 2]]
    uc, vc, wc = cell_velocity(u, v, w)
    vn = (uc[aj[:, 0], aj[:, 1], aj[:, 2]] * n[:, 0] + vc[aj[:, 0], aj[:, 1], aj[:, 2]] * n[:, 1]
          + wc[aj[:, 0], aj[:, 1], aj[:, 2]] * n[:, 2])
    if prm.get("species_form", 0) == 1:
        gx, gy, gz = omega_gradient(omega, prm["h"])
        gn = (gx[aj[:, 0], aj[:, 1], aj[:, 2]] * n[:, 0] + gy[aj[:, 0], aj[:, 1], aj[:, 2]] * n[:, 1]
              + gz[aj[:, 0], aj[:, 1], aj[:, 2]] * n[:, 2])
        jn = -rho_G * D * gn + rho_G * w_adj * vn
    else:
        jn = rho_G * D * (w_sat - w_adj) / d + rho_G * w_adj * vn
    gm = geo["gradmag"][ic[:, 0], ic[:, 1], ic[:, 2]]
    mraw = mraw.index_put((ic[:, 0], ic[:, 1], ic[:, 2]), jn * gm)
    return mraw


def redistribute(mraw, alpha):
    """Eqs. 19-21: mdot = K f(alpha) mdot_raw, K preserving the volume integral."""
    q = torch.clamp(alpha * (1.0 - alpha), min=0.0)
    f = torch.where(q > 0.0, torch.sqrt(torch.where(q > 0.0, q, torch.ones_like(q))), torch.zeros_like(q))
    S1 = mraw.sum()
    S2 = (f * mraw).sum()
    if float(S2) == 0.0:
        return torch.zeros_like(mraw), torch.zeros((), dtype=torch.float64)
    K = S1 / S2
    return K * f * mraw, K
