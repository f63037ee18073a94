"""CPU checks of the boundary: the built library loads and exports every entry point that
include/sph.h declares (no compute call: this container has no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_stage_calls():
    names = declared("sph.h")
    for f in ("sph_build_cells", "sph_density", "sph_stress_rate", "sph_forces", "sph_step"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2107_07315_amd import sph
    if not os.path.exists(sph.LIB_PATH):
        pytest.skip("libsph.so not built")
    lib = ctypes.CDLL(sph.LIB_PATH)
    missing = [f for f in declared("sph.h") if not hasattr(lib, f)]
    assert not missing, missing
    assert set(sph.EXPORTED) <= set(declared("sph.h"))


def test_binding_structs_match_header_field_order():
    from paper_2107_07315_amd import sph
    txt = open(os.path.join(ROOT, "include", "sph.h")).read()
    body = txt[txt.index("typedef struct {\n  int32_t kernel;"):]
    body = body[: body.index("} sph_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.replace("typedef struct {", "").split(";"):
        decl = decl.strip()
        if not decl:
            continue
        if decl.startswith("const "):
            decl = decl[len("const "):]
        names = decl.split(None, 1)[1]
        for nm in names.split(","):
            fields.append(nm.strip().lstrip("*").strip())
    assert [f for f, _ in sph.SphParams._fields_] == fields


def test_status_string_without_gpu():
    from paper_2107_07315_amd import sph
    if not os.path.exists(sph.LIB_PATH):
        pytest.skip("libsph.so not built")
    lib = ctypes.CDLL(sph.LIB_PATH)
    lib.sph_status_string.restype = ctypes.c_char_p
    assert lib.sph_status_string(5) == b"SPH_E_NGB_CAPACITY"
