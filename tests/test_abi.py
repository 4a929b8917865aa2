"""The C ABI: every function declared in include/ilh.h is exported by libilh.so and bound
by the Python binding (load only; no compute call without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ilh.h")
LIB = os.path.join(ROOT, "paper_2609_16424_amd", "libilh.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ilh_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_documented_calls():
    names = declared()
    for n in ["ilh_create", "ilh_destroy", "ilh_residual", "ilh_jvp", "ilh_jvp_lin", "ilh_force", "ilh_force_jvp",
              "ilh_mass_v_solve", "ilh_mass_e_inv", "ilh_implicit_step", "ilh_mlp_forward", "ilh_mlp_backward"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libilh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ilh_[a-z0-9_]+)", out))
    assert set(declared()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libilh.so not built")
def test_binding_covers_the_header():
    from paper_2609_16424_amd import _lib
    assert set(declared()) == set(_lib.SIGNATURES)
    lib = _lib.load()
    for n in declared():
        assert getattr(lib, n).argtypes is not None or getattr(lib, n).restype is None


def test_product_path_has_no_oracle_import():
    """The package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_2609_16424_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
