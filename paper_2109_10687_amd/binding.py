"""ctypes binding of libddsolve.so (include/ddsolve.h), argument marshalling only.

The functions carry the C names.  Fields are torch tensors on the GPU in the
canonical layout (complex128):

  gauge   U[mu][t][z][y][x][3][3]        (mu = 0..3 is the paper's mu = 1..4)
  spinor  psi[t][z][y][x][colour][spin]

Every step of the solver runs in the HIP library.  There is no fallback: if
libddsolve.so is missing or fails to load, every call raises.
"""
import contextlib
import ctypes
import math
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddsolve.so")
LIB_RACE_PATH = os.path.join(HERE, "libddsolve_racecheck.so")

DD_F64, DD_F32, DD_F16 = 0, 1, 2
DD_OP_D, DD_OP_A, DD_OP_DDAG = 0, 1, 2
DD_SOLVE_F64_PLAIN, DD_SOLVE_F32_SAP, DD_SOLVE_MIXED, DD_SOLVE_MIXED_GCR, DD_SOLVE_FGMRES = 0, 1, 2, 3, 4
DD_DEBUG_ZERO_OMEGA_F16, DD_DEBUG_ZERO_OMEGA_F32 = 1, 2
(DD_KT_DIRAC_F64, DD_KT_DIRAC_F32, DD_KT_DIRAC_F16IN, DD_KT_DIRAC_F16, DD_KT_SAP, DD_KT_BLAS, DD_KT_FORCE,
 DD_KT_DIRAC_MRHS, DD_KT_DIRAC_MULTI) = range(9)
KERNEL_CLASSES = {"dirac_f64": DD_KT_DIRAC_F64, "dirac_f32": DD_KT_DIRAC_F32, "dirac_f16in": DD_KT_DIRAC_F16IN,
                  "dirac_f16": DD_KT_DIRAC_F16, "sap": DD_KT_SAP, "blas": DD_KT_BLAS, "force": DD_KT_FORCE,
                  "dirac_mrhs": DD_KT_DIRAC_MRHS, "dirac_multi": DD_KT_DIRAC_MULTI}
DD_BATCH_INNER_SAP, DD_BATCH_INNER_PLAIN = 0, 1

STATUS = {0: "DD_OK", 1: "DD_NOT_CONVERGED", 2: "DD_BREAKDOWN", -1: "DD_ERR_ARG", -2: "DD_ERR_GEOMETRY",
          -3: "DD_ERR_HIP", -4: "DD_ERR_NOMEM", -5: "DD_ERR_NONFINITE", -6: "DD_ERR_CLOVER_NOT_PD",
          -7: "DD_ERR_STATE"}

EXPORTS = ["dd_create", "dd_destroy", "dd_load_gauge", "dirac_apply", "sap_precondition", "bicgstab_solve",
           "dd_last_error", "dd_field_bytes", "dd_pack_spinor", "dd_unpack_spinor", "dirac_apply_packed",
           "dirac_apply_packed_f16in", "dd_timing_enable", "dd_timing_query", "bicgstab_solve_dagger", "dd_spinor_norm2", "dd_set_csw",
           "dd_force", "dirac_apply_batch", "dd_batch_set_variant", "dd_batch_tuning", "dd_batch_variant_name",
           "bicgstab_solve_batch", "dd_multi_create", "dd_multi_destroy", "dd_multi_last_error", "dd_multi_context",
           "dd_multi_load_gauge", "dirac_apply_multi", "bicgstab_solve_multi", "dd_solve_history",
           "dd_force_noalloc", "sap_precondition_batch",
           "sap_precondition_amsap"]


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("block", ctypes.c_int * 4), ("kappa", ctypes.c_double),
                ("csw", ctypes.c_double), ("phase_re", ctypes.c_double * 4), ("phase_im", ctypes.c_double * 4),
                ("n_sap", ctypes.c_int), ("n_jac", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("inner_maxiter", ctypes.c_int), ("gcr_nkv", ctypes.c_int), ("sap_fp16_arith", ctypes.c_int),
                ("stall_window", ctypes.c_int), ("sap_fused_tail", ctypes.c_int), ("fgmres_nkv", ctypes.c_int),
                ("no_fallback", ctypes.c_int), ("debug_flags", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("iters_outer", ctypes.c_int), ("iters_inner_total", ctypes.c_int),
                ("relres_true", ctypes.c_double), ("relres_inner_last", ctypes.c_double),
                ("seconds", ctypes.c_double), ("status_detail", ctypes.c_int), ("status", ctypes.c_int),
                ("precision_level", ctypes.c_int)]


_LIB = None


def lib():
    """Load libddsolve.so; raises when it has not been built."""
    global _LIB
    if _LIB is None:
        _LIB = _load(LIB_PATH)
    return _LIB


@contextlib.contextmanager
def use_library(path):
    """Route every call of this module to another build of the library (the LDS race-check
    build, LIB_RACE_PATH) inside the with block; contexts made there belong to that build."""
    global _LIB
    saved = lib()
    _LIB = _load(path)
    try:
        yield _LIB
    finally:
        _LIB = saved


def _load(path):
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build() "
                           "or python paper_2109_10687_amd/build.py")
    L = ctypes.CDLL(path)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "dd_create": (i, [ctypes.POINTER(_Params), vp, ctypes.POINTER(vp)]),
        "dd_destroy": (i, [vp]),
        "dd_load_gauge": (i, [vp, vp]),
        "dirac_apply": (i, [vp, vp, vp, i, i]),
        "sap_precondition": (i, [vp, vp, vp, i]),
        "sap_precondition_amsap": (i, [vp, vp, vp, i]),
        "bicgstab_solve": (i, [vp, vp, vp, d, i, i, ctypes.POINTER(_Info)]),
        "dd_last_error": (ctypes.c_char_p, [vp]),
        "dd_solve_history": (i, [vp, i, ctypes.POINTER(d), i, ctypes.POINTER(i)]),
        "dd_field_bytes": (ll, [vp, i]),
        "dd_pack_spinor": (i, [vp, vp, vp, i]),
        "dd_unpack_spinor": (i, [vp, vp, vp, i]),
        "dirac_apply_packed": (i, [vp, vp, vp, i, i]),
        "dirac_apply_packed_f16in": (i, [vp, vp, vp]),
        "dd_timing_enable": (i, [vp, i]),
        "dd_timing_query": (i, [vp, i, ctypes.POINTER(ll), ctypes.POINTER(d), ctypes.POINTER(d),
                                ctypes.POINTER(d)]),
        "bicgstab_solve_dagger": (i, [vp, vp, vp, d, i, i, ctypes.POINTER(_Info)]),
        "dd_spinor_norm2": (i, [vp, vp, ctypes.POINTER(d)]),
        "dd_set_csw": (i, [vp, d]),
        "dd_force": (i, [vp, vp, ctypes.POINTER(d), vp, vp, i]),
        "dd_force_noalloc": (i, [vp, vp, ctypes.POINTER(d), vp, vp, i]),
        "dirac_apply_batch": (i, [vp, vp, vp, i, i, i]),
        "dd_batch_set_variant": (i, [vp, i]),
        "sap_precondition_batch": (i, [vp, vp, vp, i]),
        "dd_batch_tuning": (i, [vp, i, ctypes.POINTER(i), ctypes.POINTER(d), i]),
        "dd_batch_variant_name": (ctypes.c_char_p, [i]),
        "bicgstab_solve_batch": (i, [vp, vp, vp, i, d, i, i, ctypes.POINTER(_Info)]),
        "dd_multi_create": (i, [ctypes.POINTER(_Params), i, vp, ctypes.POINTER(vp)]),
        "dd_multi_destroy": (i, [vp]),
        "dd_multi_last_error": (ctypes.c_char_p, [vp]),
        "dd_multi_context": (vp, [vp, i]),
        "dd_multi_load_gauge": (i, [vp, i, vp]),
        "dirac_apply_multi": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "bicgstab_solve_multi": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), d, i, ctypes.POINTER(_Info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


@dataclass
class Params:
    """dd_params: dims = (Lx, Ly, Lz, Lt); block = SAP block extents."""
    dims: tuple
    kappa: float
    csw: float
    block: tuple = (4, 4, 4, 4)
    phases: tuple = (1.0, 1.0, 1.0, -1.0)
    n_sap: int = 4
    n_jac: int = 4
    inner_tol: float = 1e-6
    inner_maxiter: int = 2000
    gcr_nkv: int = 16
    sap_fp16_arith: int = 1
    stall_window: int = 200
    sap_fused_tail: int = 0
    fgmres_nkv: int = 4
    no_fallback: int = 0
    debug_flags: int = 0

    def c(self):
        p = _Params()
        for mu in range(4):
            p.dims[mu] = int(self.dims[mu])
            p.block[mu] = int(self.block[mu])
            ph = complex(self.phases[mu])
            p.phase_re[mu] = ph.real
            p.phase_im[mu] = ph.imag
        p.kappa = float(self.kappa)
        p.csw = float(self.csw)
        p.n_sap = int(self.n_sap)
        p.n_jac = int(self.n_jac)
        p.inner_tol = float(self.inner_tol)
        p.inner_maxiter = int(self.inner_maxiter)
        p.gcr_nkv = int(self.gcr_nkv)
        p.sap_fp16_arith = int(self.sap_fp16_arith)
        p.stall_window = int(self.stall_window)
        p.sap_fused_tail = int(self.sap_fused_tail)
        p.fgmres_nkv = int(self.fgmres_nkv)
        p.no_fallback = int(self.no_fallback)
        p.debug_flags = int(self.debug_flags)
        return p

    @property
    def volume(self):
        return math.prod(self.dims)

    @property
    def shape(self):
        Lx, Ly, Lz, Lt = self.dims
        return (Lt, Lz, Ly, Lx)


def _check(ctx, st):
    if st < 0:
        raise DDError(st, lib().dd_last_error(ctx).decode())
    return st


def _dev(t, shape=None, what="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _c128(t, shape, what):
    if t.dtype != torch.complex128:
        raise TypeError(f"{what} must be complex128")
    return _dev(t, shape, what)


# ------------------------------------------------------------------ C names

def dd_create(params, stream=None):
    """Create a context bound to `stream` (default: torch's current stream)."""
    if stream is None:
        stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    out = ctypes.c_void_p()
    p = params.c()
    st = lib().dd_create(ctypes.byref(p), h, ctypes.byref(out))
    if st < 0:
        raise DDError(st, "dd_create failed")
    return out


def dd_destroy(ctx):
    return lib().dd_destroy(ctx)


def dd_load_gauge(ctx, U, shape):
    return _check(ctx, lib().dd_load_gauge(ctx, _c128(U, (4,) + shape + (3, 3), "gauge field")))


def dirac_apply(ctx, out, inp, prec, op, shape):
    sp = shape + (3, 4)
    return _check(ctx, lib().dirac_apply(ctx, _c128(out, sp, "out"), _c128(inp, sp, "in"), prec, op))


def sap_precondition(ctx, x, b, prec, shape):
    sp = shape + (3, 4)
    return _check(ctx, lib().sap_precondition(ctx, _c128(x, sp, "x"), _c128(b, sp, "b"), prec))


def _info_dict(info):
    """dd_solve_info as a dict; "status" is the C side's status of that solve, by name."""
    d = {k: getattr(info, k) for k, _ in _Info._fields_}
    d["status"] = STATUS[d["status"]]
    return d


def sap_precondition_amsap(ctx, ax, b, prec, shape):
    sp = shape + (3, 4)
    return _check(ctx, lib().sap_precondition_amsap(ctx, _c128(ax, sp, "ax"), _c128(b, sp, "b"), prec))


def bicgstab_solve(ctx, x, b, tol, maxiter, mode, shape):
    sp = shape + (3, 4)
    info = _Info()
    st = _check(ctx, lib().bicgstab_solve(ctx, _c128(x, sp, "x"), _c128(b, sp, "b"), float(tol), int(maxiter),
                                          int(mode), ctypes.byref(info)))
    return st, _info_dict(info)


def dd_solve_history(ctx, which):
    """Residual history of the last single-field solve: which = 0 the true FP64 residual per outer
    pass (and at the start), 1 the recursive inner residual per inner iteration."""
    n = ctypes.c_int(0)
    _check(ctx, lib().dd_solve_history(ctx, int(which), None, 0, ctypes.byref(n)))
    buf = (ctypes.c_double * max(n.value, 1))()
    _check(ctx, lib().dd_solve_history(ctx, int(which), buf, n.value, ctypes.byref(n)))
    return [buf[k] for k in range(n.value)]


def bicgstab_solve_dagger(ctx, x, b, tol, maxiter, mode, shape):
    sp = shape + (3, 4)
    info = _Info()
    st = _check(ctx, lib().bicgstab_solve_dagger(ctx, _c128(x, sp, "x"), _c128(b, sp, "b"), float(tol),
                                                 int(maxiter), int(mode), ctypes.byref(info)))
    return st, _info_dict(info)


def dd_spinor_norm2(ctx, x, shape):
    out = ctypes.c_double(0)
    _check(ctx, lib().dd_spinor_norm2(ctx, _c128(x, shape + (3, 4), "x"), ctypes.byref(out)))
    return out.value


def dd_set_csw(ctx, csw):
    return _check(ctx, lib().dd_set_csw(ctx, float(csw)))


def dd_force(ctx, out, psi, chi, su3, shape, want_dcsw=True):
    """Fills out (gradient W^dagger per link, or the su(3) force); returns dL/dc_SW (None if not asked)."""
    sp = shape + (3, 4)
    d = ctypes.c_double(0)
    _check(ctx, lib().dd_force(ctx, _c128(out, (4,) + shape + (3, 3), "out"), ctypes.byref(d) if want_dcsw else None,
                               _c128(psi, sp, "psi"), _c128(chi, sp, "chi"), int(su3)))
    return d.value if want_dcsw else None


def dd_force_noalloc(ctx, out, psi, chi, su3, shape, want_dcsw=True):
    """dd_force with the work field in the library's fixed device array (no allocation)."""
    sp = shape + (3, 4)
    d = ctypes.c_double(0)
    _check(ctx, lib().dd_force_noalloc(ctx, _c128(out, (4,) + shape + (3, 3), "out"),
                                       ctypes.byref(d) if want_dcsw else None, _c128(psi, sp, "psi"),
                                       _c128(chi, sp, "chi"), int(su3)))
    return d.value if want_dcsw else None


def dirac_apply_batch(ctx, out, inp, nrhs, prec, op, shape):
    sp = (nrhs,) + shape + (3, 4)
    return _check(ctx, lib().dirac_apply_batch(ctx, _c128(out, sp, "out"), _c128(inp, sp, "in"), int(nrhs), prec, op))


def sap_precondition_batch(ctx, x, b, nrhs, shape):
    sp = (nrhs,) + shape + (3, 4)
    return _check(ctx, lib().sap_precondition_batch(ctx, _c128(x, sp, "x"), _c128(b, sp, "b"), int(nrhs)))


def dd_batch_set_variant(ctx, variant):
    return _check(ctx, lib().dd_batch_set_variant(ctx, int(variant)))


def dd_batch_tuning(ctx, nrhs):
    """(variant in use, autotuner ms per variant) for tiles of nrhs right-hand sides."""
    v = ctypes.c_int(-1)
    n = 16
    ms = (ctypes.c_double * n)()
    _check(ctx, lib().dd_batch_tuning(ctx, int(nrhs), ctypes.byref(v), ms, n))
    return v.value, [m for m in ms]


def dd_batch_variant_name(variant):
    return lib().dd_batch_variant_name(int(variant)).decode()


def bicgstab_solve_batch(ctx, x, b, nrhs, tol, maxiter, inner, shape):
    sp = (nrhs,) + shape + (3, 4)
    infos = (_Info * nrhs)()
    st = _check(ctx, lib().bicgstab_solve_batch(ctx, _c128(x, sp, "x"), _c128(b, sp, "b"), int(nrhs), float(tol),
                                                int(maxiter), int(inner), infos))
    return st, [_info_dict(inf) for inf in infos]


def dd_field_bytes(ctx, prec):
    return lib().dd_field_bytes(ctx, prec)


def dd_pack_spinor(ctx, dst, src, prec):
    return _check(ctx, lib().dd_pack_spinor(ctx, _dev(dst, what="dst"), _dev(src, what="src"), prec))


def dd_unpack_spinor(ctx, dst, src, prec):
    return _check(ctx, lib().dd_unpack_spinor(ctx, _dev(dst, what="dst"), _dev(src, what="src"), prec))


def dirac_apply_packed(ctx, out, inp, prec, op):
    return _check(ctx, lib().dirac_apply_packed(ctx, _dev(out, what="out"), _dev(inp, what="in"), prec, op))


def dirac_apply_packed_f16in(ctx, out, inp):
    return _check(ctx, lib().dirac_apply_packed_f16in(ctx, _dev(out, what="out"), _dev(inp, what="in")))


def dd_timing_enable(ctx, on):
    return _check(ctx, lib().dd_timing_enable(ctx, int(on)))


def dd_timing_query(ctx, cls):
    """(launches, ms, algorithmic bytes, flops) of one kernel class since enabling."""
    n = ctypes.c_longlong(0)
    ms, by, fl = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(ctx, lib().dd_timing_query(ctx, cls, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                      ctypes.byref(fl)))
    return n.value, ms.value, by.value, fl.value


# ------------------------------------------------------------------ convenience

class Solver:
    """A context with its gauge field: Dirac apply, SAP and BiCGStab on torch tensors."""

    def __init__(self, params, U=None, stream=None):
        self.params = params
        self.shape = params.shape
        self.gauge_version = 0  # counts dd_load_gauge calls (the autograd backward checks it)
        self.ctx = dd_create(params, stream)
        if U is not None:
            self.load_gauge(U)

    def close(self):
        if self.ctx:
            dd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_gauge(self, U):
        dd_load_gauge(self.ctx, U, self.shape)
        self.gauge_version += 1

    def new_spinor(self):
        return torch.zeros(self.shape + (3, 4), dtype=torch.complex128, device="cuda")

    def apply(self, x, op=DD_OP_D, prec=DD_F64, out=None):
        out = self.new_spinor() if out is None else out
        dirac_apply(self.ctx, out, x, prec, op, self.shape)
        return out

    def precondition(self, b, prec=DD_F32, out=None):
        out = self.new_spinor() if out is None else out
        sap_precondition(self.ctx, out, b, prec, self.shape)
        return out

    def solve(self, b, tol=1e-10, maxiter=10000, mode=DD_SOLVE_MIXED, x0=None):
        x = self.new_spinor() if x0 is None else x0.clone()
        st, info = bicgstab_solve(self.ctx, x, b, tol, maxiter, mode, self.shape)
        return x, info

    def history(self):
        """{"outer": true FP64 residual per defect-correction pass, "inner": recursive residual per
        inner iteration} of the last solve on this context."""
        return {"outer": dd_solve_history(self.ctx, 0), "inner": dd_solve_history(self.ctx, 1)}

    def solve_dagger(self, b, tol=1e-10, maxiter=10000, mode=DD_SOLVE_MIXED, x0=None):
        """x with D^dagger x = b (through D^dagger = gamma_5 D gamma_5)."""
        x = self.new_spinor() if x0 is None else x0.clone()
        st, info = bicgstab_solve_dagger(self.ctx, x, b, tol, maxiter, mode, self.shape)
        return x, info

    def norm2(self, x):
        return dd_spinor_norm2(self.ctx, x, self.shape)

    def set_csw(self, csw):
        """Change c_SW; load the gauge field again before the next operator call."""
        dd_set_csw(self.ctx, csw)
        self.params.csw = float(csw)

    def force(self, psi, chi, su3=False, out=None, want_dcsw=True):
        """(per-link gradient dL/dRe U + i dL/dIm U, or the su(3) force; dL/dc_SW) for
        L = |psi|^2 with psi = D^{-1} phi and chi = D^{-dagger} psi."""
        out = torch.empty((4,) + self.shape + (3, 3), dtype=torch.complex128, device="cuda") if out is None else out
        dcsw = dd_force(self.ctx, out, psi, chi, int(su3), self.shape, want_dcsw)
        return out, dcsw

    def apply_batch(self, xs, op=DD_OP_A, prec=DD_F32, out=None):
        """op applied to each of xs[r] (shape (nrhs,) + lattice + (3, 4)), one batched launch per 12."""
        out = torch.empty_like(xs) if out is None else out
        dirac_apply_batch(self.ctx, out, xs, xs.shape[0], prec, op, self.shape)
        return out

    def amsap(self, b, prec=DD_F32, out=None):
        """A M_SAP b (Alg. 3; fused into the SAP's last half-sweeps at FP32)."""
        out = self.new_spinor() if out is None else out
        sap_precondition_amsap(self.ctx, out, b, prec, self.shape)
        return out

    def precondition_batch(self, bs, out=None):
        """M_SAP b_r for each of bs[r] (FP16 storage; one launch per half-sweep for all of them)."""
        out = torch.empty_like(bs) if out is None else out
        sap_precondition_batch(self.ctx, out, bs, bs.shape[0], self.shape)
        return out

    def batch_variant(self, variant=-1):
        """Force the batched kernel variant, or -1 for the autotuner."""
        dd_batch_set_variant(self.ctx, variant)

    def batch_tuning(self, nrhs):
        v, ms = dd_batch_tuning(self.ctx, nrhs)
        n = sum(1 for m in ms if m > 0)
        return {"variant": v, "name": dd_batch_variant_name(v) if v >= 0 else None,
                "ms": {dd_batch_variant_name(k): ms[k] for k in range(len(ms)) if ms[k] > 0}, "timed": n}

    def solve_batch(self, bs, tol=1e-10, maxiter=50, inner=DD_BATCH_INNER_SAP, x0=None):
        """x_r with D x_r = b_r for every r (bs: (nrhs,) + lattice + (3, 4)); returns (x, infos)."""
        x = torch.zeros_like(bs) if x0 is None else x0.clone()
        st, infos = bicgstab_solve_batch(self.ctx, x, bs, bs.shape[0], tol, maxiter, inner, self.shape)
        return x, infos

    def field(self, prec):
        """An internal-layout field buffer for the packed entry points."""
        n = dd_field_bytes(self.ctx, prec)
        return torch.empty((n + 255) // 256 * 256, dtype=torch.uint8, device="cuda")

    def pack(self, x, prec, out=None):
        out = self.field(prec) if out is None else out
        dd_pack_spinor(self.ctx, out, x, prec)
        return out

    def unpack(self, f, prec, out=None):
        out = self.new_spinor() if out is None else out
        dd_unpack_spinor(self.ctx, out, f, prec)
        return out

    def apply_packed(self, out, inp, op=DD_OP_A, prec=DD_F32):
        dirac_apply_packed(self.ctx, out, inp, prec, op)
        return out

    def apply_packed_f16in(self, out, inp):
        """out (FP32 field) = A inp (FP16 field): the inner solver's operator application."""
        dirac_apply_packed_f16in(self.ctx, out, inp)
        return out

    def timing(self, on=True):
        dd_timing_enable(self.ctx, on)

    def timing_report(self):
        """{class: {launches, ms, bytes, flops}} since timing was enabled."""
        out = {}
        for name, cls in KERNEL_CLASSES.items():
            n, ms, by, fl = dd_timing_query(self.ctx, cls)
            out[name] = {"launches": n, "ms": ms, "bytes": by, "flops": fl}
        return out


class Multi:
    """Several independent lattices whose FP32 operator runs in one persistent launch
    (dd_multi_*): load a gauge field per lattice, apply A to all, or solve all in lockstep."""

    def __init__(self, params_list, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self.params = list(params_list)
        self.shapes = [p.shape for p in self.params]
        arr = (_Params * len(self.params))(*[p.c() for p in self.params])
        out = ctypes.c_void_p()
        st = lib().dd_multi_create(arr, len(self.params), h, ctypes.byref(out))
        if st < 0:
            raise DDError(st, "dd_multi_create failed")
        self.m = out

    def _check(self, st):
        if st < 0:
            raise DDError(st, lib().dd_multi_last_error(self.m).decode())
        return st

    def close(self):
        if self.m:
            lib().dd_multi_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def context(self, k):
        return ctypes.c_void_p(lib().dd_multi_context(self.m, k))

    def load_gauge(self, k, U):
        self._check(lib().dd_multi_load_gauge(self.m, k, _c128(U, (4,) + self.shapes[k] + (3, 3), "gauge field")))

    def _ptrs(self, ts, what):
        return (ctypes.c_void_p * len(ts))(*[_c128(t, sh + (3, 4), what) for t, sh in zip(ts, self.shapes)])

    def apply(self, xs):
        """[A_k x_k] for every lattice, FP32, one launch."""
        outs = [torch.empty_like(x) for x in xs]
        self._check(lib().dirac_apply_multi(self.m, self._ptrs(outs, "out"), self._ptrs(xs, "in")))
        return outs

    def solve(self, bs, tol=1e-10, maxiter=50, x0=None):
        xs = [torch.zeros_like(b) for b in bs] if x0 is None else [x.clone() for x in x0]
        infos = (_Info * len(bs))()
        st = self._check(lib().bicgstab_solve_multi(self.m, self._ptrs(xs, "x"), self._ptrs(bs, "b"), float(tol),
                                                    int(maxiter), infos))
        return xs, [_info_dict(inf) for inf in infos]

    def timing(self, on=True):
        dd_timing_enable(self.context(0), on)

    def timing_report(self):
        """{class: {launches, ms, bytes, flops}} of lattice 0's context (it times the multi-lattice launches)."""
        out = {}
        for name, cls in KERNEL_CLASSES.items():
            n, ms, by, fl = dd_timing_query(self.context(0), cls)
            out[name] = {"launches": n, "ms": ms, "bytes": by, "flops": fl}
        return out

