"""The C-ABI library loads and exports every symbol the header declares (CPU:
no compute calls, no GPU needed)."""
import ctypes
import os
import re

from paper_1403_5044_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "shipwave.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shipwave_\w+)\s*\(", text)))


def test_header_declares_the_paper_calls():
    names = _declared()
    for n in ("shipwave_residual", "shipwave_jvp", "shipwave_precond_build_banded",
              "shipwave_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert sorted(_lib.SIGNATURES) == _declared()


def test_abi_version_and_error_string():
    lib = _lib.load()
    assert lib.shipwave_abi_version() == 1
    assert isinstance(lib.shipwave_last_error(), bytes)


def test_struct_layouts_match_the_header():
    assert ctypes.sizeof(_lib.SwProblem) == 8 + 24 + 40
    assert ctypes.sizeof(_lib.SwParams) == 40
    assert ctypes.sizeof(_lib.SwSolveOpts) == 8 + 8 * 4 + 8 + 8 + 8
