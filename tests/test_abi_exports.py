"""The C-ABI library loads and exports every entry point include/dd.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd.h")
LIB = os.path.join(ROOT, "paper_1612_06424_amd", "libdd.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    syms = declared_symbols()
    for name in ["dd_apply_dirac", "dd_block_solve", "dd_factorized_propagator", "dd_pion_correlator",
                 "dd_block_solve_backward", "dd_create", "dd_destroy", "dd_last_error"]:
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_binding_covers_every_symbol():
    import paper_1612_06424_amd.dd as dd
    assert sorted(dd.EXPORTS) == declared_symbols()


@pytest.mark.parametrize("compiler,std,lang", [("gcc", "c99", "c"), ("g++", "c++17", "c++")])
def test_header_is_plain_c_and_cpp(compiler, std, lang):
    """include/dd.h is a C header (the boundary takes no C++ or torch types): it compiles on
    its own as C99 and as C++17 without warnings."""
    import shutil
    import subprocess
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    hdr = os.path.join(ROOT, "include", "dd.h")
    subprocess.check_call([compiler, "-fsyntax-only", f"-std={std}", "-Wall", "-Wextra", "-Werror", "-x", lang, hdr])
