"""CPU checks of the C ABI library: it loads, and it exports every function
that include/frpmg.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2202_09733_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "frpmg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:fr_status|void|const char \*|size_t|int)\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_parses():
    names = _declared_functions()
    assert "fr_residual" in names and "gmres_solve_stage" in names and len(names) >= 12


@pytest.mark.skipif(not os.path.exists(capi.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(capi.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(capi.EXPORTS) == _declared_functions()


def test_struct_layouts_match_header_field_order():
    txt = open(os.path.join(ROOT, "include", "frpmg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    for cname, pyst in [("stage_params", capi.StageParams), ("pmg_params", capi.PmgParams),
                        ("stage_stats", capi.StageStats), ("fr_mesh_desc", capi.MeshDesc)]:
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", txt).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"\[.*?\]", "", decl)
            parts = decl.replace("*", " ").split()
            names = " ".join(parts[1:]).split(",") if len(parts) > 1 else []
            if parts[0] == "const":
                names = " ".join(parts[2:]).split(",")
            fields += [n.strip() for n in names if n.strip()]
        assert fields == [f[0] for f in pyst._fields_], (cname, fields)
