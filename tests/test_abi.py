"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, its structs match the binding's layout, and host-side
validation rejects bad problems before touching the GPU."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1912_03106_amd import _abi
from workload import config, polar_mesh
from workload.configs import LevelSpec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgrit.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    assert set(declared_functions()) == set(_abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True)
    exported = {line.split()[-1] for line in nm.stdout.splitlines() if " T " in line}
    assert set(declared_functions()) <= exported


STRUCTS = {"mgrit_mesh": _abi.Mesh, "mgrit_physics": _abi.Physics, "mgrit_problem": _abi.Problem,
           "mgrit_params": _abi.Params, "mgrit_stats": _abi.Stats,
           "mgrit_train_params": _abi.TrainParams, "mgrit_train_stats": _abi.TrainStats}


def test_struct_layout_matches_header(tmp_path):
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgrit.h"', "int main(void){"]
    for cname, py in STRUCTS.items():
        src.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            src.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src.append("return 0;}")
    c_file = tmp_path / "layout.c"
    c_file.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(c_file), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for line in out.splitlines():
        cname, field, val = line.split()
        py = STRUCTS[cname]
        got = C.sizeof(py) if field == "size" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)


def test_default_params():
    L = _abi.lib()
    p = _abi.Params()
    L.mgrit_default_params(C.byref(p))
    assert (p.m, p.gamma, p.precision, p.restriction) == (16, 1, _abi.FP64, _abi.R_NORMALIZED)
    assert p.tol == 1e-8 and p.warm_start == 1 and p.pcg_max_iter > 0


def test_strerror_names_every_status():
    L = _abi.lib()
    for code in _abi.STATUS:
        assert L.mgrit_strerror(code)
    assert L.mgrit_strerror(-100) == b"unknown status"


def _solver(cfg, **kw):
    from paper_1912_03106_amd.solver import Solver
    return Solver(cfg, **kw)


def _status_of(fn):
    with pytest.raises(_abi.MgritError) as e:
        fn()
    return e.value.name


def test_host_validation_not_nested():
    cfg = config("cfg1")
    cfg.meshes = [LevelSpec(16, 128), LevelSpec(8, 32)]
    assert _status_of(lambda: _solver(cfg)) == "NOT_NESTED"


def test_host_validation_bad_arguments():
    cfg = config("cfg1", m=1)
    assert _status_of(lambda: _solver(cfg)) == "INVALID_ARGUMENT"
    cfg = config("cfg1", n_steps=1000)        # not divisible by m
    assert _status_of(lambda: _solver(cfg)) == "INVALID_ARGUMENT"


def test_host_validation_clockwise_triangle():
    cfg = config("cfg1")
    meshes = [polar_mesh(16, 128), polar_mesh(16, 128)]
    meshes[0].tri = meshes[0].tri[:, [0, 2, 1]].copy()
    assert _status_of(lambda: _solver(cfg, meshes=meshes)) == "INVALID_ARGUMENT"


def test_host_validation_node_out_of_range():
    cfg = config("cfg1")
    meshes = [polar_mesh(16, 128), polar_mesh(16, 128)]
    meshes[1].tri = meshes[1].tri.copy()
    meshes[1].tri[5, 1] = meshes[1].n_nodes + 3
    assert _status_of(lambda: _solver(cfg, meshes=meshes)) == "INVALID_ARGUMENT"


def test_host_validation_nonfinite_coordinate():
    cfg = config("cfg1")
    meshes = [polar_mesh(16, 128), polar_mesh(16, 128)]
    meshes[0].xy = meshes[0].xy.copy()
    meshes[0].xy[7, 0] = np.nan
    assert _status_of(lambda: _solver(cfg, meshes=meshes)) in ("NONFINITE", "INVALID_ARGUMENT")


@pytest.mark.parametrize("bad", [dict(pcg_prefetch=3), dict(warm_start=3), dict(residual_eta=1.0),
                                 dict(residual_eta=-1e-3), dict(pcg_rows_narrow=48),
                                 dict(compact_fraction=1.0), dict(compact_columns=-1),
                                 dict(pcg_kernel=5), dict(pcg_tol_eta=-1.0)])
def test_host_validation_solver_parameters(bad):
    """Every mgrit_params check runs before the first HIP call."""
    assert _status_of(lambda: _solver(config("cfg1"), **bad)) == "INVALID_ARGUMENT"


def test_default_params_of_the_cg_loop():
    L = _abi.lib()
    p = _abi.Params()
    L.mgrit_default_params(C.byref(p))
    assert (p.pcg_check_every, p.compact_columns, p.compact_fraction) == (4, 64, 0.9)
    assert (p.pcg_prefetch, p.pcg_rows_narrow, p.residual_eta, p.pcg_tol_eta) == (0, 0, 0.0, 0.0)
