"""The C-ABI library builds for gfx950, loads without a GPU and exports every
entry point declared in include/afmpb.h (no compute calls here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afmpb.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char \*|afmpb_status )\s*(afmpb_\w+)\(", text,
                                 re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("afmpb_create", "afmpb_set_molecule", "afmpb_matvec", "afmpb_solve",
                     "afmpb_destroy", "afmpb_matvec_dev", "afmpb_debug_tree"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1710_06316_amd as A
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libafmpb.so not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (afmpb_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = A.lib()
    for n in _declared():
        assert hasattr(L, n)
    assert set(A.ABI_FUNCTIONS) == set(_declared())


def test_default_params_without_gpu():
    import paper_1710_06316_amd as A
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libafmpb.so not built")
    p = A.afmpb_default_params()
    assert (p.eps_p, p.eps_s, p.kappa, p.order_p, p.leaf_cap) == (2.0, 80.0, 0.1, 8, 64)
    assert (p.restart, p.max_restarts, p.near_eta, p.rel_tol) == (80, 5, 4.0, 1e-6)
    # implementation choices default to automatic
    assert (p.m2l_layout, p.rhs_fmm, p.overlap, p.wx_expand) == (0, 0, 0, 0)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1710_06316_amd as A
    monkeypatch.setattr(A, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(A, "_lib", None)
    with pytest.raises(RuntimeError, match="not found"):
        A.lib()


def _struct_fields(name):
    """Member names of `typedef struct { ... } name;` in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    names = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        first, *rest = decl.split(",")
        names.append(re.findall(r"\w+", first)[-1])
        names += [re.findall(r"\w+", r)[-1] for r in rest]
    return names


@pytest.mark.parametrize("name", ["afmpb_params", "afmpb_solve_info", "afmpb_tree_sizes",
                                  "afmpb_tree_view"])
def test_binding_structs_follow_the_header(name):
    """The ctypes mirrors of the parameter and result structs list the
    header's members in the header's order (a missing or reordered member
    would shift every later field across the boundary)."""
    import paper_1710_06316_amd as A
    cls = getattr(A, name)
    assert [f for f, _ in cls._fields_] == _struct_fields(name)
