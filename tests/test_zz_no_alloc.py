"""The entry point for callers that cannot allocate: ds_droplet_volume_noalloc
(handle-free liquid volume of a caller's alpha array, the library's own
file-scope scratch for the reduction) against ds_droplet_volume of a handle
holding the same alpha, on two calls in a row, the second with a smaller grid;
oversize grids and bad arguments are rejected before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2005_02867_amd as ds
    return ds


def _case(n, seed):
    prm, _ = W.config("C1")
    prm = W.finalize(dict(prm, nx=n[0], ny=n[1], nz=n[2], x0=None))
    return prm, W.random_fields(prm, seed=seed)


def test_noalloc_volume_matches_handle_volume_twice():
    ds = _lib()
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    for n, seed in (((40, 36, 44), 1), ((17, 19, 23), 2)):     # the second call on a smaller grid
        prm, f = _case(n, seed)
        print(f"grid {n}: handle volume vs no-allocation volume", flush=True)
        g = ds.Grid(prm)
        g.set_fields(f)
        v_handle = g.droplet_volume()
        a = torch.tensor(f["alpha"], dtype=torch.float64, device="cuda")
        ds.droplet_volume_noalloc(a, prm["h"], out)
        torch.cuda.synchronize()
        v = float(out.item())
        print("  handle", v_handle, "no-allocation", v)
        assert v == v_handle                       # same reduction order: bit for bit
        assert v == pytest.approx(prm["h"] ** 3 * float(np.sum(f["alpha"])), rel=1e-13)
        del g


def test_noalloc_rejects_oversize_and_bad_arguments():
    ds = _lib()
    a = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    lib = ds._lib
    # 2048^3 cells exceeds the maximum: rejected before anything is launched
    rc = lib.ds_droplet_volume_noalloc(C.c_void_p(a.data_ptr()), 2048, 2048, 2048, C.c_double(1e-4),
                                       C.c_void_p(out.data_ptr()), None)
    assert rc == ds.DS_ERR_ARG
    assert "exceeds the maximum" in lib.ds_last_error(None).decode()
    rc = lib.ds_droplet_volume_noalloc(C.c_void_p(a.data_ptr()), 0, 2, 2, C.c_double(1e-4),
                                       C.c_void_p(out.data_ptr()), None)
    assert rc == ds.DS_ERR_ARG
    rc = lib.ds_droplet_volume_noalloc(None, 2, 2, 2, C.c_double(1e-4), C.c_void_p(out.data_ptr()), None)
    assert rc == ds.DS_ERR_ARG
    # a valid call afterwards still works and clears the message
    a2 = torch.full((2, 2, 2), 0.5, dtype=torch.float64, device="cuda")
    ds.droplet_volume_noalloc(a2, 1e-4, out)
    torch.cuda.synchronize()
    assert float(out.item()) == pytest.approx(8 * 0.5 * 1e-12, rel=1e-15)
    assert lib.ds_last_error(None).decode() == ""
