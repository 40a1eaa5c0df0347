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


def test_integer_constants_match_header():
    """Every integer #define of the header that the binding mirrors (under
    its name with or without the FR_ prefix) has the same value; the step
    tableaux and the stage cap are among them."""
    txt = open(os.path.join(ROOT, "include", "frpmg.h")).read()
    defs = dict(re.findall(r"^#define\s+(FR_\w+)\s+(-?\d+)\b", txt, flags=re.M))
    seen = []
    for name, val in defs.items():
        for py in (name, name[3:]):
            if hasattr(capi, py):
                assert getattr(capi, py) == int(val), (name, getattr(capi, py), val)
                seen.append(name)
                break
    for need in ["FR_TAB_ESDIRK2", "FR_TAB_ROW2", "FR_TAB_ESDIRK3", "FR_TAB_ROW3", "FR_TAB_ESDIRK4",
                 "FR_TAB_ROW4", "FR_MAX_STEP_STAGES"]:
        assert need in seen, need


TABS = {"esdirk2": capi.TAB_ESDIRK2, "esdirk3": capi.TAB_ESDIRK3, "esdirk4": capi.TAB_ESDIRK4,
        "row2": capi.TAB_ROW2, "row3": capi.TAB_ROW3, "row4": capi.TAB_ROW4}


@pytest.mark.skipif(not os.path.exists(capi.LIB_PATH), reason="library not built")
@pytest.mark.parametrize("name", list(TABS))
def test_step_tableaux_match_the_oracle(name):
    """The coefficients of the library's full time steps (a host call) equal
    the oracle's tableaux, which its own tests pin to the order conditions."""
    import numpy as np
    from oracle import stepping as S
    t = capi.step_tableau(TABS[name])
    if name.startswith("esdirk"):
        ref = S.ESDIRK_TABLEAUX[name]()
        assert not t["rosenbrock"] and t["stages"] == len(ref.b)
        assert abs(t["gamma"] - ref.gamma) <= 1e-15
        assert np.allclose(t["A"], ref.A, rtol=0, atol=2e-15)
    else:
        ref = S.ROW_TABLEAUX[name]()
        s = len(ref.b)
        assert t["rosenbrock"] and t["stages"] == s
        assert abs(t["gamma"] - ref.gamma) <= 1e-15
        lo = np.tril(np.ones((s, s)), -1).astype(bool)
        scale = max(1.0, np.abs(ref.cm).max())
        assert np.allclose(np.array(t["a"])[lo], ref.a[lo], rtol=0, atol=1e-14)
        assert np.allclose(np.array(t["c"])[lo], ref.cm[lo], rtol=0, atol=1e-14 * scale)
        assert not np.any(np.array(t["a"])[~lo]) and not np.any(np.array(t["c"])[~lo])
        assert np.allclose(t["m"], ref.m, rtol=0, atol=1e-14)


def test_step_tableau_rejects_unknown():
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(capi.FRError):
        capi.step_tableau(6)
