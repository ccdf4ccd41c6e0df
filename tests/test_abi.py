"""The C-ABI library loads on the CPU host, exports every symbol the header
declares, and its structs have the layout the Python binding assumes.  No
compute calls (no GPU here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsvof.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ds_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2005_02867_amd as ds
    lib = C.CDLL(ds.LIB_PATH)
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ds.EXPORTS)


def test_struct_layout_matches_binding(tmp_path):
    import paper_2005_02867_amd as ds
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    lines.append('printf("params %zu\\n", sizeof(ds_params));')
    lines.append('printf("diag %zu\\n", sizeof(ds_diagnostics));')
    for name, _ in ds.Params._fields_:
        lines.append(f'printf("P.{name} %zu\\n", offsetof(ds_params, {name}));')
    for name, _ in ds.Diagnostics._fields_:
        lines.append(f'printf("D.{name} %zu\\n", offsetof(ds_diagnostics, {name}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split(" ") for line in out if line)
    assert int(got["params"]) == C.sizeof(ds.Params)
    assert int(got["diag"]) == C.sizeof(ds.Diagnostics)
    for name, _ in ds.Params._fields_:
        assert int(got[f"P.{name}"]) == getattr(ds.Params, name).offset, name
    for name, _ in ds.Diagnostics._fields_:
        assert int(got[f"D.{name}"]) == getattr(ds.Diagnostics, name).offset, name


def test_create_grid_rejects_bad_arguments_before_touching_the_device():
    import workloads as W
    import paper_2005_02867_amd as ds
    prm, _ = W.config("C1")
    for bad in (dict(prm, h=0.0), dict(prm, dt=-1.0), dict(prm, eps_int=0.7), dict(prm, bc_mode=5),
                dict(prm, maxit=0), dict(prm, tol=0.0)):
        with pytest.raises(ds.DSError) as e:
            ds.create_grid(8, 8, 8, bad)
        assert e.value.code == ds.DS_ERR_ARG
    with pytest.raises(ds.DSError):
        ds.create_grid(1, 8, 8, prm)
