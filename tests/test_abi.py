"""The C-ABI library loads and exports every function include/ddamg.h declares
(no device calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ddamg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dd_create", "dd_setup", "dd_solve", "dd_destroy", "dd_last_error", "dd_apply"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1303_1377_amd import LIB_PATH

    assert os.path.exists(LIB_PATH), "libddamg.so not built"
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_params_are_table1():
    import paper_1303_1377_amd as G

    p = G.default_params()
    assert p.levels == 2 and p.n_tv[0] == 20 and p.nu == 2 and p.n_inv == 6
    assert list(p.agg[0]) == [4, 4, 4, 4] and list(p.sap[0]) == [4, 4, 4, 4]
    assert p.mr_steps[0] == 4 and p.coarse_restart == 30 and abs(p.coarse_tol - 5e-2) < 1e-15
    assert p.outer_restart == 25
    assert p.max_rhs == 1


def test_package_import_does_not_need_the_device():
    import paper_1303_1377_amd as G

    assert callable(G.Solver)


def _enum_values(prefix):
    src = open(os.path.join(ROOT, "include", "ddamg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b%s([A-Z0-9_]+)\s*=\s*(\d+)" % prefix, src)}


def test_binding_constants_match_the_header():
    """The binding passes operators, kernel classes and schedule flags as
    plain integers: its tables must hold the header's values."""
    import paper_1303_1377_amd as G

    ops = _enum_values("DD_OP_")
    assert ops == G.OPS
    sched = _enum_values("DD_SCHED_")
    assert sched == G.SCHED
    kcls = _enum_values("DD_K_")
    n = kcls.pop("NCLASS")
    assert n == len(G.KERNEL_CLASSES)
    assert sorted(kcls.values()) == list(range(n))
    for name, v in kcls.items():
        assert G.KERNEL_CLASSES[v] == name.lower(), (name, v)
