"""The C-ABI library loads and exports every function include/ba.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_path():
    names = _declared()
    for n in ("ba_create", "ba_destroy", "ba_linearize", "ba_form_rcs", "ba_pcg_solve",
              "ba_back_substitute", "ba_lm_step", "ba_project", "ba_status_str", "ba_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2307_08383_amd import ba
    if not os.path.exists(ba.LIB_PATH):
        from paper_2307_08383_amd import build
        build.build()
    lib = ctypes.CDLL(ba.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert set(ba.SIGNATURES) == set(_declared())


def test_status_strings_without_gpu():
    from paper_2307_08383_amd import ba
    assert ba.ba_status_str(ba.BA_OK) == "ok"
    assert "converge" in ba.ba_status_str(ba.BA_ERR_NOT_CONVERGED)
