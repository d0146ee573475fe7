"""CPU checks of the C ABI: the library loads and exports every entry point
that include/grca.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2605_10457_amd import grca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "grca.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(grca_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_three_core_calls():
    names = _declared()
    for core in ("grca_scene_update", "grca_sensor_config", "grca_cast"):
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(grca.LIB_PATH):
        pytest.skip("libgrca.so not built")
    lib = ctypes.CDLL(grca.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(grca.exported_symbols()) == _declared()


def test_binding_signatures_load():
    if not os.path.exists(grca.LIB_PATH):
        pytest.skip("libgrca.so not built")
    lib = grca.load()
    assert lib.grca_cast.restype is ctypes.c_int


def test_header_is_plain_c(tmp_path):
    """include/grca.h must compile as C99 (no C++ in the public ABI)."""
    import subprocess
    src = tmp_path / "use_abi.c"
    src.write_text('#include "grca.h"\n'
                   'int probe(grca_context* c) {\n'
                   '  grca_sensor_desc d; grca_options o; grca_stats s; (void)d; (void)s;\n'
                   '  return (int)grca_get_options(c, &o) + (int)GRCA_MISS_TRI;\n}\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-c",
                        "-I", os.path.join(ROOT, "include"), str(src), "-o",
                        str(tmp_path / "use_abi.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
