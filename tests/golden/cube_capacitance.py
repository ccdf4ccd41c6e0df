"""Capacitance of a sphere (radius a) centred in a grounded cube (side L),
relative to the same sphere in free space.  Written to cube_capacitance.json.

Independent of the method, the oracle and the GPU library: a second-order
finite-difference Laplace solve (scipy) with phi = 1 on cells inside the
sphere and phi = 0 half a cell outside the cube, the charge taken as the flux
through the cube walls, averaged over several grids (the staircase sphere
makes single grids scatter by ~2%).  The quasi-steady evaporation rate of a
droplet in this box is the free-space rate times this ratio.

    python tests/golden/cube_capacitance.py
"""
import json
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def capacitance_ratio(n, a, L):
    h = L / n
    x = (np.arange(n) + 0.5) * h - L / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    inside = (np.sqrt(X ** 2 + Y ** 2 + Z ** 2) <= a).ravel()
    N = n ** 3
    idx = np.arange(N).reshape(n, n, n)
    rows, cols = [], []
    diag = np.zeros(N)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        s, d = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        rows += [s, d]
        cols += [d, s]
        np.add.at(diag, s, 1.0)
        np.add.at(diag, d, 1.0)
        for e in (0, n - 1):
            sl = [slice(None)] * 3
            sl[ax] = e
            np.add.at(diag, idx[tuple(sl)].ravel(), 2.0)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = sp.csr_matrix((-np.ones(r.size), (r, c)), shape=(N, N)) + sp.diags(diag)
    out = ~inside
    rhs = -(A[out][:, inside] @ np.ones(inside.sum()))
    phi_o, info = spla.cg(A[out][:, out], rhs, rtol=1e-11, maxiter=50000)
    assert info == 0
    phi = np.ones(N)
    phi[out] = phi_o
    P = phi.reshape(n, n, n)
    Q = 0.0
    for ax in range(3):
        for e in (0, n - 1):
            sl = [slice(None)] * 3
            sl[ax] = e
            Q += (2.0 * P[tuple(sl)] * h).sum()
    return Q / (4.0 * np.pi) / a


if __name__ == "__main__":
    a, L = 0.5e-3, 4e-3
    grids = (48, 64, 80, 96)
    vals = [capacitance_ratio(n, a, L) for n in grids]
    # converged value: the finest grid (successive grids change it by < 0.2%)
    out = dict(a=a, L=L, grids=list(grids), ratios=[float(v) for v in vals], ratio=float(vals[-1]),
               last_change=float(abs(vals[-1] - vals[-2])))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_capacitance.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(out)
