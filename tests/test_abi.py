"""The C-ABI library loads, exports every symbol the header declares, and its
argument validation works without a GPU (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hermite.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hermite_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1104_2700_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_hot_path():
    names = _declared()
    for need in ("hermite_select_block", "hermite_predict", "hermite_force_jerk",
                 "hermite_correct", "hermite_init_dt", "hermite_step", "hermite_run",
                 "hermite_energy", "hermite_autotune"):
        assert need in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_errors_without_touching_a_device(lib):
    lib.hermite_last_error.restype = ctypes.c_char_p
    # null context is rejected before any HIP call
    lib.hermite_force_jerk.restype = ctypes.c_int
    rc = lib.hermite_force_jerk(None, None, None, None, None, 0, ctypes.c_double(0.0),
                                0, None, None, None, None)
    assert rc == -1
    assert b"null context" in lib.hermite_last_error()
    lib.hermite_create.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    rc = lib.hermite_create(0, None)
    assert rc == -1
    lib.hermite_destroy.argtypes = [ctypes.c_void_p]
    assert lib.hermite_destroy(None) == 0
    lib.hermite_check_finite.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.hermite_check_finite(None, None, None) == -1


def test_binding_names_match_header():
    """Every C entry point has a ctypes signature in the binding."""
    import importlib
    from paper_1104_2700_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    herm = importlib.import_module("paper_1104_2700_amd.hermite")
    for n in _declared():
        if n == "hermite_last_error":
            continue
        assert n in herm._SIGS, n


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the C layout of include/hermite.h
    (size and every field offset, as the host C compiler lays them out)."""
    import subprocess
    from paper_1104_2700_amd import hermite as H
    structs = {"hermite_state": H.CState, "hermite_dt_params": H.CDtParams,
               "hermite_clusters": H.CClusters, "hermite_tuning": H.CTuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hermite.h"',
             'int main(void) {']
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
