"""The C-ABI library loads on the host and exports every function that
include/ddsolve.h declares (no compute call: there may be no GPU)."""
import ctypes
import os
import re

import paper_2109_10687_amd as dd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ddsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_]\w*\s+)+\**\s*([A-Za-z_]\w*)\s*\(", src, re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dirac_apply", "sap_precondition", "bicgstab_solve", "dd_create", "dd_destroy",
                     "dd_load_gauge", "dd_last_error"):
        assert required in names
    assert sorted(dd.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    L = dd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_create_rejects_bad_geometry_without_gpu():
    # geometry is checked before any device call
    p = dd.Params(dims=(8, 8, 8, 6), kappa=0.12, csw=1.0, block=(4, 4, 4, 4))  # 6 is not a multiple of 2*4
    try:
        dd.dd_create(p, stream=0)
    except dd.DDError as e:
        assert e.status == -2
    else:
        raise AssertionError("expected DD_ERR_GEOMETRY")
    p = dd.Params(dims=(16, 8, 8, 8), kappa=0.12, csw=1.0, block=(8, 4, 4, 4))  # 512 sites > one workgroup
    try:
        dd.dd_create(p, stream=0)
    except dd.DDError as e:
        assert e.status == -2
    else:
        raise AssertionError("expected DD_ERR_GEOMETRY")
    p = dd.Params(dims=(8, 8, 8, 8), kappa=0.12, csw=1.0, block=(4, 3, 4, 4))  # not a power of two
    try:
        dd.dd_create(p, stream=0)
    except dd.DDError as e:
        assert e.status == -2
    else:
        raise AssertionError("expected DD_ERR_GEOMETRY")


def test_create_rejects_bad_gcr_cycle_without_gpu():
    p = dd.Params(dims=(8, 8, 8, 8), kappa=0.12, csw=1.0, gcr_nkv=17)
    try:
        dd.dd_create(p, stream=0)
    except dd.DDError as e:
        assert e.status == -1
    else:
        raise AssertionError("expected DD_ERR_ARG")
