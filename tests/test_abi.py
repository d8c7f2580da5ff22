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


def _documented_param_layout():
    """(name, shape) list of the network parameters as include/ba.h documents
    them (the block after "in the order"), with "3 x (...)" expanded."""
    src = open(os.path.join(ROOT, "include", "ba.h")).read()
    body = src.split("in the order", 1)[1].split("(row-major", 1)[0]
    body = re.sub(r"\s*\*\s*", " ", body)
    body = re.sub(r"\(factorised head,.*?\)", "", body, flags=re.S)
    out = []
    for rep, group in re.findall(r"(?:(\d+) x \(([^)]*)\))", body):
        for _ in range(int(rep)):
            for name, dims in re.findall(r"([A-Za-z_]+)((?:\[\d+\])+)", group):
                out.append((name, tuple(int(d) for d in re.findall(r"\d+", dims))))
        body = body.replace(f"{rep} x ({group})", "@LAYERS@", 1)
    pre, post = body.split("@LAYERS@")
    ent = lambda s: [(n, tuple(int(d) for d in re.findall(r"\d+", ds)))
                     for n, ds in re.findall(r"([A-Za-z_0-9]+)((?:\[\d+\])+)", s)]
    return ent(pre) + out + ent(post)


def test_documented_network_layout_matches_library_and_reference():
    """The header's parameter list has the library's parameter count and the
    shapes, in order, of the CPU reference network."""
    import numpy as np
    from oracle import gnn_ref
    from paper_2307_08383_amd import ba
    doc = _documented_param_layout()
    n_doc = sum(int(np.prod(s)) for _, s in doc)
    assert n_doc == ba.ba_gnn_param_count()
    ref = [tuple(s) for _, s in gnn_ref.PARAM_SHAPES]
    assert [s for _, s in doc] == ref
    assert [n for n, _ in doc][-5:] == ["Wo1", "bo1", "Wo2", "bo2", "ao"]
    assert f"{n_doc:,} values in all" in open(os.path.join(ROOT, "include", "ba.h")).read()
