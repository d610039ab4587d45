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


def test_new_entry_points_reject_null_handles_without_gpu():
    L = dd.lib()
    vp = ctypes.c_void_p
    null = vp(0)
    d = ctypes.c_double(0)
    info = dd.binding._Info()
    assert L.dirac_apply_batch(null, null, null, 12, dd.DD_F32, dd.DD_OP_A) == -1
    assert L.dirac_apply_packed_f16in(null, null, null) == -1
    assert L.bicgstab_solve_batch(null, null, null, 12, 1e-10, 10, 0, ctypes.byref(info)) == -1
    assert L.bicgstab_solve_dagger(null, null, null, 1e-10, 10, dd.DD_SOLVE_MIXED, ctypes.byref(info)) == -1
    assert L.dd_force(null, null, ctypes.byref(d), null, null, 0) == -1
    assert L.dd_spinor_norm2(null, null, ctypes.byref(d)) == -1
    assert L.dd_set_csw(null, 1.0) == -1
    assert L.dd_batch_set_variant(null, 0) == -1
    assert L.dd_batch_tuning(null, 12, None, None, 0) == -1
    assert L.dirac_apply_multi(null, None, None) == -1
    assert L.bicgstab_solve_multi(null, None, None, 1e-10, 10, None) == -1
    assert L.dd_multi_load_gauge(null, 0, null) == -1
    assert L.dd_multi_context(null, 0) is None
    assert L.dd_multi_last_error(null) == b"null handle"
    assert L.dd_destroy(null) == 0 and L.dd_multi_destroy(null) == 0
    n = ctypes.c_int(-1)
    assert L.dd_solve_history(null, 0, None, 0, ctypes.byref(n)) == -1


def struct_fields(name):
    """Field names of `typedef struct { ... } name;` in the header, in order."""
    src = open(os.path.join(ROOT, "include", "ddsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            fields += [re.sub(r"\[.*?\]", "", v).strip().lstrip("*") for v in decl.split(None, 1)[1].split(",")]
    return fields


def test_binding_structs_follow_the_header():
    """The ctypes mirrors of dd_params and dd_solve_info list the header's fields in its order."""
    assert [f for f, _ in dd.binding._Params._fields_] == struct_fields("dd_params")
    assert [f for f, _ in dd.binding._Info._fields_] == struct_fields("dd_solve_info")


def test_debug_flags_follow_the_header():
    src = open(os.path.join(ROOT, "include", "ddsolve.h")).read()
    defs = dict(re.findall(r"#define (DD_DEBUG_\w+)\s+(\d+)", src))
    assert defs == {"DD_DEBUG_ZERO_OMEGA_F16": str(dd.DD_DEBUG_ZERO_OMEGA_F16),
                    "DD_DEBUG_ZERO_OMEGA_F32": str(dd.DD_DEBUG_ZERO_OMEGA_F32)}


def test_batch_variant_names():
    names = [dd.dd_batch_variant_name(v) for v in range(13)]
    assert all(n and n != "?" for n in names) and len(set(names)) == 13
    assert any("mfma" in n for n in names) and any("vector" in n for n in names) and any("resident" in n for n in names)
    assert dd.dd_batch_variant_name(-1) == "?" and dd.dd_batch_variant_name(13) == "?"


def test_multi_create_checks_every_lattice_without_gpu():
    ok = dd.Params(dims=(8, 8, 8, 8), kappa=0.12, csw=1.0, block=(4, 4, 4, 4))
    bad = dd.Params(dims=(8, 8, 8, 6), kappa=0.12, csw=1.0, block=(4, 4, 4, 4))
    L = dd.lib()
    out = ctypes.c_void_p()
    arr = (dd.binding._Params * 1)(bad.c())
    assert L.dd_multi_create(arr, 1, None, ctypes.byref(out)) == -2 and not out.value
    assert L.dd_multi_create(arr, 0, None, ctypes.byref(out)) == -1
    arr2 = (dd.binding._Params * 2)(bad.c(), ok.c())
    assert L.dd_multi_create(arr2, 2, None, ctypes.byref(out)) == -2 and not out.value
