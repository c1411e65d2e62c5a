"""The C ABI library loads and exports every symbol include/suppcg.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "suppcg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1807_10151_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1807_10151_amd import build
        build.build()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_solver_calls():
    names = declared_functions()
    for must in ("sp_project", "sp_backproject", "sp_precond_apply", "sp_tv_perturb",
                 "sp_suppcg_solve"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1807_10151_amd import _lib
    assert set(declared_functions()) <= set(_lib.exported_symbols())


def test_version_and_null_context(lib):
    from paper_1807_10151_amd import _lib
    L = _lib.load()
    assert L.sp_version().decode().startswith("suppcg")
    g = _lib.sp_geometry(4, 4, 1.0, 4, 0.0, -1.0, 5, 1.0, 0.0)
    assert L.sp_project(None, ctypes.byref(g), None, None) == _lib.SP_ERR_ARG
    assert L.sp_ctx_destroy(None) == _lib.SP_ERR_ARG
    assert L.sp_last_error(None) == b"null context"


def test_struct_layouts_match_header(tmp_path):
    # sizes and field offsets from the C compiler against the ctypes mirror
    from paper_1807_10151_amd import _lib
    structs = {"sp_geometry": _lib.sp_geometry, "sp_tv_params": _lib.sp_tv_params,
               "sp_precond": _lib.sp_precond, "sp_solve_params": _lib.sp_solve_params,
               "sp_trace": _lib.sp_trace, "sp_batch_trace": _lib.sp_batch_trace}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "suppcg.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = dict(line.split() for line in out if line.strip())
    for name, cls in structs.items():
        assert int(want[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(want[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
