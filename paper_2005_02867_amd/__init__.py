"""MI355X (gfx950) VOF droplet-evaporation step: Python binding of libdsvof.

The binding marshals arguments only: every step of the method runs in the
HIP kernels of ``libdsvof.so`` (built in-tree by ``build.py``).  PyTorch
supplies device memory (the caller-owned workspace and field tensors) and the
current HIP stream.  Importing this module without the built library raises.

Functions mirror the C ABI in ``include/dsvof.h`` (without the ``ds_``
prefix); ``Grid`` bundles a handle with its workspace.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsvof.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_02867_amd.build`")
_lib = C.CDLL(LIB_PATH)

DS_OK, DS_ERR_ARG, DS_ERR_HIP, DS_ERR_NOT_CONVERGED, DS_ERR_NONFINITE, DS_ERR_STATE = 0, -1, -2, -3, -4, -5
(FIELD_MDOT_RAW, FIELD_MDOT, FIELD_ALPHA1, FIELD_C, FIELD_USTAR, FIELD_VSTAR, FIELD_WSTAR, FIELD_ADJ,
 FIELD_RHO_G) = range(9)
EXPORTS = ("ds_create_grid", "ds_destroy_grid", "ds_workspace_bytes", "ds_set_fields", "ds_get_fields",
           "ds_step", "ds_solve_pressure", "ds_evaporation_rate", "ds_droplet_volume", "ds_get_diagnostics",
           "ds_get_internal", "ds_last_error", "ds_set_kernel_timing", "ds_get_kernel_timing",
           "ds_time_operator_kernel", "ds_tape_bytes", "ds_forward_record", "ds_adjoint",
           "ds_get_adjoint_iterations", "ds_time_kernel", "ds_solve_system", "ds_droplet_volume_noalloc")
KERNEL_CG_OPERATOR, KERNEL_MG_SMOOTH = 0, 1
SYS_PRESSURE, SYS_ENERGY, SYS_SPECIES, SYS_POTENTIAL = 0, 1, 2, 3


class Params(C.Structure):
    _fields_ = [
        ("h", C.c_double), ("dt", C.c_double), ("p", C.c_double), ("T_amb", C.c_double),
        ("rho_L", C.c_double), ("cp_L", C.c_double), ("k_L", C.c_double),
        ("cp_G", C.c_double), ("k_G", C.c_double), ("D_v", C.c_double), ("dh_ev", C.c_double),
        ("M_v", C.c_double), ("M_G", C.c_double), ("g", C.c_double * 3),
        ("xi0", C.c_double), ("Df", C.c_double), ("r_fib", C.c_double), ("w_in", C.c_double),
        ("x0", C.c_double * 3),
        ("Tc", C.c_double), ("Pc", C.c_double), ("acentric", C.c_double),
        ("Tc_G", C.c_double), ("Pc_G", C.c_double), ("acentric_G", C.c_double), ("kij", C.c_double),
        ("T_ref", C.c_double), ("p_ref", C.c_double), ("eps_int", C.c_double), ("eps_gas", C.c_double),
        ("theta_min", C.c_double),
        ("tol", C.c_double), ("tol_phi", C.c_double),
        ("s_max", C.c_int), ("maxit", C.c_int), ("eq_model", C.c_int), ("bc_mode", C.c_int),
        ("precision", C.c_int), ("solve_energy", C.c_int), ("evaporation", C.c_int), ("pressure_precond", C.c_int),
        ("liquid_transport", C.c_int), ("species_form", C.c_int), ("viscous", C.c_int),
        ("mu_L", C.c_double), ("mu_G", C.c_double), ("gas_density", C.c_int), ("advection", C.c_int),
    ]


class Diagnostics(C.Structure):
    _fields_ = [
        ("K", C.c_double), ("mdot_total", C.c_double), ("volume", C.c_double), ("fuel_mass", C.c_double),
        ("fuel_mass_before", C.c_double), ("B_L", C.c_double), ("B_v", C.c_double),
        ("alpha_min", C.c_double), ("alpha_max", C.c_double),
        ("res_T", C.c_double), ("res_omega", C.c_double), ("res_p", C.c_double), ("rho_G", C.c_double),
        ("iters_T", C.c_int), ("iters_omega", C.c_int), ("iters_p", C.c_int),
        ("n_interface", C.c_int), ("converged", C.c_int), ("refinements_p", C.c_int),
        ("iters_phi", C.c_int), ("res_phi", C.c_double), ("rounds_T", C.c_int), ("rounds_omega", C.c_int),
        ("iters_visc", C.c_int), ("res_visc", C.c_double),
    ]


_P = C.c_void_p
_lib.ds_create_grid.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(Params), C.POINTER(_P)]
_lib.ds_destroy_grid.argtypes = [_P]
_lib.ds_workspace_bytes.argtypes = [_P]
_lib.ds_workspace_bytes.restype = C.c_size_t
_lib.ds_set_fields.argtypes = [_P] + [_P] * 7 + [_P, C.c_size_t, _P]
_lib.ds_get_fields.argtypes = [_P] + [_P] * 7 + [_P]
_lib.ds_step.argtypes = [_P, C.c_int, _P]
_lib.ds_solve_pressure.argtypes = [_P, _P, C.POINTER(C.c_int), C.POINTER(C.c_double)]
_lib.ds_solve_system.argtypes = [_P, C.c_int, _P, _P, _P, C.POINTER(C.c_int), C.POINTER(C.c_double)]
_lib.ds_evaporation_rate.argtypes = [_P, C.POINTER(C.c_double), _P, _P]
_lib.ds_droplet_volume.argtypes = [_P, C.POINTER(C.c_double), _P]
_lib.ds_get_diagnostics.argtypes = [_P, C.POINTER(Diagnostics)]
_lib.ds_get_internal.argtypes = [_P, C.c_int, _P, C.c_size_t, _P]
_lib.ds_set_kernel_timing.argtypes = [_P, C.c_int]
_lib.ds_get_kernel_timing.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.POINTER(C.c_double)]
_lib.ds_time_operator_kernel.argtypes = [_P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), _P]
_lib.ds_tape_bytes.argtypes = [_P, C.c_int, C.c_int]
_lib.ds_tape_bytes.restype = C.c_size_t
_lib.ds_forward_record.argtypes = [_P, C.c_int, C.c_int, _P, C.c_size_t, _P]
_lib.ds_adjoint.argtypes = [_P, C.c_double, C.POINTER(C.c_double)] + [_P] * 6 + [_P]
_lib.ds_get_adjoint_iterations.argtypes = [_P, C.POINTER(C.c_int)]
_lib.ds_time_kernel.argtypes = [_P, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), _P]
_lib.ds_droplet_volume_noalloc.argtypes = [_P, C.c_int, C.c_int, C.c_int, C.c_double, _P, _P]
_lib.ds_last_error.argtypes = [_P]
_lib.ds_last_error.restype = C.c_char_p


class DSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dsvof error {code}: {msg}")
        self.code = code


class NotConverged(DSError):
    pass


def _check(handle, code, handle_free=False):
    if code == DS_OK:
        return
    msg = _lib.ds_last_error(handle).decode() if (handle or handle_free) else ""
    raise (NotConverged if code == DS_ERR_NOT_CONVERGED else DSError)(code, msg)


def make_params(prm: dict) -> Params:
    P = Params()
    for name, ctype in Params._fields_:
        if name in ("pressure_precond", "liquid_transport"):
            val = prm.get(name, 1)
        elif name in ("species_form", "viscous", "gas_density", "advection"):
            val = prm.get(name, 0)
        elif name in ("mu_L", "mu_G"):
            val = prm.get(name, 0.0)
        elif name == "eps_gas":
            val = prm.get(name, prm["eps_int"])
        elif name == "tol_phi":
            val = prm.get(name, prm["tol"])
        else:
            val = prm[name]
        if name in ("g", "x0"):
            setattr(P, name, (C.c_double * 3)(*[float(x) for x in val]))
        else:
            setattr(P, name, int(val) if ctype is C.c_int else float(val))
    return P


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("fields must be contiguous float64 CUDA tensors")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------ C-ABI mirrors
def create_grid(nx, ny, nz, prm: dict):
    h = _P()
    P = make_params(prm)
    code = _lib.ds_create_grid(int(nx), int(ny), int(nz), C.byref(P), C.byref(h))
    if code != DS_OK:
        raise DSError(code, "ds_create_grid rejected the parameters")
    return h


def destroy_grid(h):
    _check(None, _lib.ds_destroy_grid(h))


def workspace_bytes(h) -> int:
    return int(_lib.ds_workspace_bytes(h))


def set_fields(h, alpha, T, omega, u, v, w, p, workspace):
    _check(h, _lib.ds_set_fields(h, _dptr(alpha), _dptr(T), _dptr(omega), _dptr(u), _dptr(v), _dptr(w),
                                 _dptr(p), C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream()))


def get_fields(h, alpha=None, T=None, omega=None, u=None, v=None, w=None, p=None):
    _check(h, _lib.ds_get_fields(h, _dptr(alpha), _dptr(T), _dptr(omega), _dptr(u), _dptr(v), _dptr(w),
                                 _dptr(p), _stream()))


def step(h, nsteps=1):
    _check(h, _lib.ds_step(h, int(nsteps), _stream()))


def solve_pressure(h):
    it = C.c_int()
    res = C.c_double()
    _check(h, _lib.ds_solve_pressure(h, _stream(), C.byref(it), C.byref(res)))
    return it.value, res.value


def solve_system(h, which, rhs, x):
    """x: initial guess in, solution out (device float64 cell tensors)."""
    it = C.c_int()
    res = C.c_double()
    _check(h, _lib.ds_solve_system(h, int(which), _dptr(rhs), _dptr(x), _stream(), C.byref(it), C.byref(res)))
    return it.value, res.value


def evaporation_rate(h, mdot_out=None):
    v = C.c_double()
    _check(h, _lib.ds_evaporation_rate(h, C.byref(v), _dptr(mdot_out), _stream()))
    return v.value


def droplet_volume(h):
    v = C.c_double()
    _check(h, _lib.ds_droplet_volume(h, C.byref(v), _stream()))
    return v.value


def droplet_volume_noalloc(alpha, h, out):
    """h^3 sum(alpha) of a device float64 cell tensor (nx, ny, nz) into the
    device float64 tensor out[0]; no handle, nothing allocated, asynchronous."""
    if alpha.dim() != 3 or alpha.dtype != torch.float64 or not alpha.is_contiguous():
        raise ValueError("alpha: a contiguous float64 (nx, ny, nz) tensor")
    if out.dtype != torch.float64 or out.numel() < 1:
        raise ValueError("out: a float64 tensor of at least one element")
    nx, ny, nz = alpha.shape
    _check(None, _lib.ds_droplet_volume_noalloc(_dptr(alpha), nx, ny, nz, float(h), _dptr(out), _stream()),
           handle_free=True)


def get_diagnostics(h) -> dict:
    d = Diagnostics()
    _check(h, _lib.ds_get_diagnostics(h, C.byref(d)))
    return {name: getattr(d, name) for name, _ in Diagnostics._fields_}


def get_internal(h, which, out):
    _check(h, _lib.ds_get_internal(h, int(which), _dptr(out), out.numel(), _stream()))


def set_kernel_timing(h, enable=True):
    _check(h, _lib.ds_set_kernel_timing(h, 1 if enable else 0))


def get_kernel_timing(h):
    avg = C.c_double()
    cnt = C.c_longlong()
    nb = C.c_double()
    _check(h, _lib.ds_get_kernel_timing(h, C.byref(avg), C.byref(cnt), C.byref(nb)))
    return dict(avg_us=avg.value, launches=cnt.value, bytes_per_launch=nb.value)


def time_operator_kernel(h, reps=50):
    us = C.c_double()
    nb = C.c_double()
    _check(h, _lib.ds_time_operator_kernel(h, int(reps), C.byref(us), C.byref(nb), _stream()))
    return dict(avg_us=us.value, bytes_per_launch=nb.value, reps=int(reps))


def tape_bytes(h, nsteps, ckpt_every=1) -> int:
    return int(_lib.ds_tape_bytes(h, int(nsteps), int(ckpt_every)))


def forward_record(h, nsteps, ckpt_every, tape):
    _check(h, _lib.ds_forward_record(h, int(nsteps), int(ckpt_every), C.c_void_p(tape.data_ptr()), tape.numel(),
                                     _stream()))


def adjoint(h, dJ_dV=1.0, dalpha0=None, dT0=None, domega0=None, du0=None, dv0=None, dw0=None):
    g = (C.c_double * 3)()
    _check(h, _lib.ds_adjoint(h, float(dJ_dV), g, _dptr(dalpha0), _dptr(dT0), _dptr(domega0), _dptr(du0),
                              _dptr(dv0), _dptr(dw0), _stream()))
    return [g[0], g[1], g[2]]


def get_adjoint_iterations(h):
    it = (C.c_int * 4)()
    _check(h, _lib.ds_get_adjoint_iterations(h, it))
    return dict(p=it[0], omega=it[1], T=it[2], phi=it[3])


def time_kernel(h, which, reps=50):
    us = C.c_double()
    nb = C.c_double()
    _check(h, _lib.ds_time_kernel(h, int(which), int(reps), C.byref(us), C.byref(nb), _stream()))
    return dict(avg_us=us.value, bytes_per_launch=nb.value, reps=int(reps))


# ------------------------------------------------------------ convenience
class Grid:
    """A handle plus its torch-allocated workspace on the current CUDA device."""

    def __init__(self, prm: dict, device="cuda"):
        self.prm = dict(prm)
        self.nx, self.ny, self.nz = int(prm["nx"]), int(prm["ny"]), int(prm["nz"])
        self.device = torch.device(device)
        self.h = create_grid(self.nx, self.ny, self.nz, prm)
        nbytes = workspace_bytes(self.h)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nbytes]
        self._raw = raw

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ds_destroy_grid(h)
            self.h = None

    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return dict(alpha=(nx, ny, nz), T=(nx, ny, nz), omega=(nx, ny, nz), p=(nx, ny, nz),
                    u=(nx + 1, ny, nz), v=(nx, ny + 1, nz), w=(nx, ny, nz + 1))

    def set_fields(self, fields: dict):
        t = {}
        for k, shp in self.shapes().items():
            x = torch.as_tensor(fields[k], dtype=torch.float64).to(self.device).contiguous()
            if tuple(x.shape) != shp:
                raise ValueError(f"{k}: shape {tuple(x.shape)} != {shp}")
            t[k] = x
        set_fields(self.h, t["alpha"], t["T"], t["omega"], t["u"], t["v"], t["w"], t["p"], self.workspace)
        torch.cuda.current_stream().synchronize()

    def get_fields(self) -> dict:
        out = {k: torch.empty(s, dtype=torch.float64, device=self.device) for k, s in self.shapes().items()}
        get_fields(self.h, **out)
        return out

    def step(self, nsteps=1):
        step(self.h, nsteps)

    def solve_pressure(self):
        return solve_pressure(self.h)

    def solve_system(self, which, rhs, x0=None):
        """Solve one implicit system of the step on the current state; returns
        (x, iterations, relative residual)."""
        shp = (self.nx, self.ny, self.nz)
        b = torch.as_tensor(rhs, dtype=torch.float64).to(self.device).reshape(shp).contiguous()
        x = (torch.zeros(shp, dtype=torch.float64, device=self.device) if x0 is None else
             torch.as_tensor(x0, dtype=torch.float64).to(self.device).reshape(shp).clone())
        it, res = solve_system(self.h, which, b, x)
        return x, it, res

    def evaporation_rate(self, return_field=False):
        if return_field:
            m = torch.empty((self.nx, self.ny, self.nz), dtype=torch.float64, device=self.device)
            return evaporation_rate(self.h, m), m
        return evaporation_rate(self.h)

    def droplet_volume(self):
        return droplet_volume(self.h)

    def diagnostics(self):
        return get_diagnostics(self.h)

    def set_kernel_timing(self, enable=True):
        set_kernel_timing(self.h, enable)

    def kernel_timing(self):
        return get_kernel_timing(self.h)

    def time_operator_kernel(self, reps=50):
        return time_operator_kernel(self.h, reps)

    def time_kernel(self, which, reps=50):
        return time_kernel(self.h, which, reps)

    def forward_record(self, nsteps, ckpt_every=1):
        """Run nsteps steps storing the tape for adjoint() (allocated here, on
        the grid's device, and kept until the next record)."""
        nbytes = tape_bytes(self.h, nsteps, ckpt_every)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._tape_raw = raw
        self.tape = raw[off:off + nbytes]
        forward_record(self.h, nsteps, ckpt_every, self.tape)

    def adjoint(self, dJ_dV=1.0, fields=True):
        """dJ/d(D_v, dh_ev, T_amb) for J = dJ_dV * droplet volume after the
        recorded run, and (fields=True) dJ/d(initial alpha, T, omega, u, v, w)."""
        out = None
        if fields:
            out = {k: torch.empty(sh, dtype=torch.float64, device=self.device)
                   for k, sh in self.shapes().items() if k != "p"}
            g = adjoint(self.h, dJ_dV, out["alpha"], out["T"], out["omega"], out["u"], out["v"], out["w"])
        else:
            g = adjoint(self.h, dJ_dV)
        return dict(D_v=g[0], dh_ev=g[1], T_amb=g[2], fields=out)

    def adjoint_iterations(self):
        return get_adjoint_iterations(self.h)

    def internal(self, which):
        s = self.shapes()
        shp = {FIELD_USTAR: s["u"], FIELD_VSTAR: s["v"], FIELD_WSTAR: s["w"]}.get(which, s["alpha"])
        out = torch.empty(shp, dtype=torch.float64, device=self.device)
        get_internal(self.h, which, out)
        return out


class DropletVolume(torch.autograd.Function):
    """V_N = h^3 sum(alpha) after `steps` steps of the library's step, as a
    differentiable function of (D_v, dh_ev, T_amb) and the initial fields
    alpha0, T0, omega0, u0, v0, w0 (float64 CUDA tensors; p0 only warm-starts).

    The forward runs ds_forward_record; the backward runs the library's
    reverse sweep (ds_adjoint).  Use through droplet_volume_after()."""

    @staticmethod
    def forward(ctx, D_v, dh_ev, T_amb, alpha0, T0, omega0, u0, v0, w0, p0, prm, steps, ckpt_every):
        q = dict(prm, D_v=float(D_v), dh_ev=float(dh_ev), T_amb=float(T_amb))
        g = Grid(q, device=alpha0.device)
        g.set_fields(dict(alpha=alpha0.detach(), T=T0.detach(), omega=omega0.detach(), u=u0.detach(),
                          v=v0.detach(), w=w0.detach(), p=p0.detach()))
        g.forward_record(int(steps), int(ckpt_every))
        V = g.droplet_volume()
        ctx.g = g
        return torch.tensor(V, dtype=torch.float64, device=alpha0.device)

    @staticmethod
    def backward(ctx, gV):
        r = ctx.g.adjoint(float(gV), fields=True)
        f = r["fields"]
        dev = f["alpha"].device
        scal = [torch.tensor(r[k], dtype=torch.float64, device=dev) for k in ("D_v", "dh_ev", "T_amb")]
        ctx.g = None
        return (*scal, f["alpha"], f["T"], f["omega"], f["u"], f["v"], f["w"], None, None, None, None)


def droplet_volume_after(prm, fields, steps, D_v, dh_ev, T_amb, ckpt_every=1):
    """Differentiable droplet volume after `steps` steps (see DropletVolume).
    D_v, dh_ev, T_amb: 0-d float64 tensors (may require grad); fields: dict of
    float64 CUDA tensors alpha, T, omega, u, v, w, p."""
    return DropletVolume.apply(D_v, dh_ev, T_amb, fields["alpha"], fields["T"], fields["omega"], fields["u"],
                               fields["v"], fields["w"], fields["p"], prm, steps, ckpt_every)
