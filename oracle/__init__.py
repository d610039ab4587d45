"""FP64 CPU oracle for the Clover-Wilson quark solver (arXiv 2109.10687).

TEST INFRASTRUCTURE ONLY: the parity checker for the GPU path.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg import this package; the
product library never does, and nothing here imports the product package.

Arrays are numpy complex128 in the canonical layout:
  links   U[mu][t][z][y][x][a][b]        (mu = 0..3 is the paper's mu = 1..4)
  spinor  psi[t][z][y][x][colour][spin]  (colour outer, spin inner, Sec. 4)
  clover  C[t][z][y][x][12][12]          (row/column index colour*4 + spin)

Each function names the passage of the paper it follows; the C source holds the
arithmetic (oracle.c).
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_LIB = None


class _CParams(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int * 4),
        ("blk", ctypes.c_int * 4),
        ("kappa", ctypes.c_double),
        ("csw", ctypes.c_double),
        ("phase_re", ctypes.c_double * 4),
        ("phase_im", ctypes.c_double * 4),
        ("n_sap", ctypes.c_int),
        ("n_jac", ctypes.c_int),
    ]


def lib():
    """Load liboracle.so, compiling it with gcc first when it is not there."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER(_CParams)
        vp = ctypes.c_void_p
        i, d, lg = ctypes.c_int, ctypes.c_double, ctypes.c_long
        pi, pd = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        sig = {
            "orc_gamma": (None, [i, vp]),
            "orc_site_colour": (i, [P, lg]),
            "orc_clover_field": (None, [P, vp, vp]),
            "orc_clover_inverse": (i, [P, vp, vp]),
            "orc_hop": (None, [P, vp, vp, vp, i]),
            "orc_dirac_D": (None, [P, vp, vp, vp, vp]),
            "orc_dirac_A": (None, [P, vp, vp, vp, vp]),
            "orc_dirac_D_sites": (None, [P, vp, vp, vp, lg, vp]),
            "orc_block_apply": (None, [P, vp, vp, vp, vp, i, i]),
            "orc_jacobi": (None, [P, vp, vp, vp, vp, i]),
            "orc_sap": (None, [P, vp, vp, vp, vp]),
            "orc_amsap": (None, [P, vp, vp, vp, vp]),
            "orc_bicgstab": (i, [P, vp, vp, vp, i, vp, vp, d, i, pi, pd]),
            "orc_dci": (i, [P, vp, vp, vp, vp, vp, d, d, i, i, i, i, pi, pi, pd]),
            "orc_force": (None, [P, vp, vp, vp, vp]),
            "orc_dirac_A_sites": (i, [P, vp, vp, vp, lg, vp]),
            "orc_dcsw": (d, [P, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


@dataclass
class Params:
    """Operator and solver parameters (Sec. 3, appendix).  dims = (Lx, Ly, Lz, Lt)."""
    dims: tuple
    kappa: float
    csw: float
    block: tuple = (2, 2, 2, 2)
    phases: tuple = (1.0, 1.0, 1.0, -1.0)
    n_sap: int = 2
    n_jac: int = 4

    @property
    def volume(self):
        return int(np.prod(self.dims))

    @property
    def shape(self):
        Lx, Ly, Lz, Lt = self.dims
        return (Lt, Lz, Ly, Lx)

    def c(self):
        cp = _CParams()
        for mu in range(4):
            cp.L[mu] = int(self.dims[mu])
            cp.blk[mu] = int(self.block[mu])
            ph = complex(self.phases[mu])
            cp.phase_re[mu] = ph.real
            cp.phase_im[mu] = ph.imag
        cp.kappa = float(self.kappa)
        cp.csw = float(self.csw)
        cp.n_sap = int(self.n_sap)
        cp.n_jac = int(self.n_jac)
        return cp


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def gamma(mu):
    """gamma_1..gamma_4 for mu = 0..3 as printed in the appendix; mu = 4 gives gamma_1 gamma_2 gamma_3 gamma_4."""
    out = np.zeros(16, dtype=np.complex128)
    lib().orc_gamma(mu, _ptr(out))
    return out.reshape(4, 4)


def site_colour(p, n):
    """Colour (0 = E, 1 = O) of the Schwarz block holding site n (Sec. 3)."""
    cp = p.c()
    return lib().orc_site_colour(ctypes.byref(cp), int(n))


def colour_mask(p):
    """Per-site block colour as an array of shape (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = p.dims
    bx, by, bz, bt = p.block
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return ((x // bx + y // by + z // bz + t // bt) % 2).astype(np.int8)


def clover_field(p, U):
    """C(n) = (i/2) kappa c_SW sigma_{mu nu} F_{mu nu}(n) with the four-leaf F (appendix)."""
    U = _c128(U)
    C = np.zeros(p.shape + (12, 12), dtype=np.complex128)
    cp = p.c()
    lib().orc_clover_field(ctypes.byref(cp), _ptr(U), _ptr(C))
    return C


def clover_inverse(p, C):
    """C_inv = (1 + C)^{-1} per site (appendix)."""
    C = _c128(C)
    Ci = np.zeros_like(C)
    cp = p.c()
    bad = lib().orc_clover_inverse(ctypes.byref(cp), _ptr(C), _ptr(Ci))
    if bad:
        raise ValueError(f"1 + C singular at {bad} sites")
    return Ci


def hop(p, U, x, part=0):
    """H x (part 0), its in-block hops (1) or its cross-block hops (2)."""
    U, x = _c128(U), _c128(x)
    y = np.zeros_like(x)
    cp = p.c()
    lib().orc_hop(ctypes.byref(cp), _ptr(U), _ptr(x), _ptr(y), part)
    return y


def dirac_D(p, U, C, x):
    """D x = (1 + C) x - kappa H x (appendix)."""
    U, C, x = _c128(U), _c128(C), _c128(x)
    y = np.zeros_like(x)
    cp = p.c()
    lib().orc_dirac_D(ctypes.byref(cp), _ptr(U), _ptr(C), _ptr(x), _ptr(y))
    return y


def dirac_A(p, U, Cinv, x):
    """A x = x - kappa C_inv H x (Sec. 3)."""
    U, Cinv, x = _c128(U), _c128(Cinv), _c128(x)
    y = np.zeros_like(x)
    cp = p.c()
    lib().orc_dirac_A(ctypes.byref(cp), _ptr(U), _ptr(Cinv), _ptr(x), _ptr(y))
    return y


def dirac_D_sites(p, U, x, sites):
    """(D x)(n) at the listed lexicographic sites, clover built on the fly; shape (len(sites), 3, 4)."""
    U, x = _c128(U), _c128(x)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    y = np.zeros((len(sites), 3, 4), dtype=np.complex128)
    cp = p.c()
    lib().orc_dirac_D_sites(ctypes.byref(cp), _ptr(U), _ptr(x), _ptr(sites), len(sites), _ptr(y))
    return y


def dirac_A_sites(p, U, x, sites):
    """(A x)(n) = x(n) - kappa C_inv(n) (H x)(n) at the listed lexicographic sites (Sec. 3), with
    the clover and its inverse built on the fly; shape (len(sites), 3, 4)."""
    U, x = _c128(U), _c128(x)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    y = np.zeros((len(sites), 3, 4), dtype=np.complex128)
    cp = p.c()
    bad = lib().orc_dirac_A_sites(ctypes.byref(cp), _ptr(U), _ptr(x), _ptr(sites), len(sites), _ptr(y))
    if bad:
        raise ValueError(f"1 + C singular at {bad} listed sites")
    return y


def block_apply(p, U, Cinv, x, colour, part, y=None):
    """Rows of colour c of A_cc x (part 1) or A_{c,c'} x (part 2); other rows of y kept (Sec. 3)."""
    U, Cinv, x = _c128(U), _c128(Cinv), _c128(x)
    y = np.zeros_like(x) if y is None else _c128(y).copy()
    cp = p.c()
    lib().orc_block_apply(ctypes.byref(cp), _ptr(U), _ptr(Cinv), _ptr(x), _ptr(y), colour, part)
    return y


def jacobi(p, U, Cinv, b, colour):
    """x_c = B_cc b_c by Alg. 2 (rows of the other colour are zero)."""
    U, Cinv, b = _c128(U), _c128(Cinv), _c128(b)
    x = np.zeros_like(b)
    cp = p.c()
    lib().orc_jacobi(ctypes.byref(cp), _ptr(U), _ptr(Cinv), _ptr(b), _ptr(x), colour)
    return x


def sap(p, U, Cinv, b):
    """x = M_SAP b by Alg. 1."""
    U, Cinv, b = _c128(U), _c128(Cinv), _c128(b)
    x = np.zeros_like(b)
    cp = p.c()
    lib().orc_sap(ctypes.byref(cp), _ptr(U), _ptr(Cinv), _ptr(b), _ptr(x))
    return x


def amsap(p, U, Cinv, b):
    """x = A M_SAP b (Alg. 3, computed as A applied to Alg. 1's output)."""
    U, Cinv, b = _c128(U), _c128(Cinv), _c128(b)
    x = np.zeros_like(b)
    cp = p.c()
    lib().orc_amsap(ctypes.byref(cp), _ptr(U), _ptr(Cinv), _ptr(b), _ptr(x))
    return x


OP_D, OP_A, OP_AMSAP = 0, 1, 2


@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iters: int
    relres: float
    outer: int = 0
    extra: dict = field(default_factory=dict)


def bicgstab(p, U, C, Cinv, b, op=OP_D, tol=1e-10, maxiter=10000):
    """Alg. 5 on D (op 0), A (op 1) or A M_SAP (op 2, returns x = M_SAP y)."""
    U, b = _c128(U), _c128(b)
    C = _c128(C) if C is not None else np.zeros(1, np.complex128)
    Cinv = _c128(Cinv) if Cinv is not None else np.zeros(1, np.complex128)
    x = np.zeros_like(b)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0)
    cp = p.c()
    st = lib().orc_bicgstab(ctypes.byref(cp), _ptr(U), _ptr(C), _ptr(Cinv), op, _ptr(b), _ptr(x), tol, maxiter,
                            ctypes.byref(it), ctypes.byref(rr))
    return SolveResult(x, st, it.value, rr.value)


def dci(p, U, C, Cinv, b, tol=1e-10, inner_tol=1e-6, inner_maxiter=1000, inner_op=OP_AMSAP, round_sp=True,
        max_outer=50):
    """Alg. 4: defect correction for D x = b around an inner solver on A = C_inv D."""
    U, C, Cinv, b = _c128(U), _c128(C), _c128(Cinv), _c128(b)
    x = np.zeros_like(b)
    no, ni = ctypes.c_int(0), ctypes.c_int(0)
    rr = ctypes.c_double(0)
    cp = p.c()
    st = lib().orc_dci(ctypes.byref(cp), _ptr(U), _ptr(C), _ptr(Cinv), _ptr(b), _ptr(x), tol, inner_tol,
                       inner_maxiter, inner_op, int(round_sp), max_outer, ctypes.byref(no), ctypes.byref(ni),
                       ctypes.byref(rr))
    return SolveResult(x, st, ni.value, rr.value, outer=no.value)


def gamma5_apply(x):
    """gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 on a canonical spinor (spin is the last index)."""
    g5 = gamma(4)
    return np.ascontiguousarray(np.einsum("ab,...b->...a", g5, x))


def force(p, U, psi, chi):
    """Link derivative of a loss whose variation is -2 Re <chi| dD psi>: the matrices W_mu(n)
    with dL = Re sum_{mu,n} tr(dU_mu(n) W_mu(n)); hop term and four-leaf clover term
    (appendix operator; derivation in oracle.c).  Shape of U."""
    U, psi, chi = _c128(U), _c128(psi), _c128(chi)
    W = np.zeros_like(U)
    cp = p.c()
    lib().orc_force(ctypes.byref(cp), _ptr(U), _ptr(psi), _ptr(chi), _ptr(W))
    return W


def dcsw(p, U, psi, chi):
    """dL/dc_SW = -2 Re <chi| (C / c_SW) psi> for the clover field C of the appendix (C / c_SW
    is the clover built with c_SW = 1, so this holds at c_SW = 0 as well)."""
    U, psi, chi = _c128(U), _c128(psi), _c128(chi)
    cp = p.c()
    return lib().orc_dcsw(ctypes.byref(cp), _ptr(U), _ptr(psi), _ptr(chi))


def grad_from_force(W):
    """The gradient dL/dRe U + i dL/dIm U of each link entry, from W: the conjugate transpose.
    With dL = Re sum tr(dU W) = Re sum_ab dU_ab W_ba and, for a real function of complex entries,
    dL = Re sum_ab conj(G_ab) dU_ab, G_ab = conj(W_ba)."""
    return np.ascontiguousarray(np.conj(np.swapaxes(W, -1, -2)))


def source_grad(chi):
    """The gradient dL/dRe phi + i dL/dIm phi of L = |D^{-1} phi|^2 from chi = D^{-dagger} psi:
    dL = 2 Re <psi| D^{-1} dphi> = 2 Re <chi| dphi>, so the gradient is 2 chi."""
    return 2.0 * np.ascontiguousarray(chi)


def su3_force(U, W):
    """Traceless Hermitian F_mu(n) with dL = tr(omega F) for U -> exp(i omega) U, omega Hermitian:
    F = (i/2)(X - X^dagger) with X = U W, trace removed."""
    X = np.matmul(U, W)
    F = 0.5j * (X - np.conj(np.swapaxes(X, -1, -2)))
    tr = np.trace(F, axis1=-2, axis2=-1) / 3.0
    return F - tr[..., None, None] * np.eye(3)


@dataclass
class LossGrad:
    loss: float
    psi: np.ndarray
    chi: np.ndarray
    W: np.ndarray
    dcsw: float


def loss_and_force(p, U, phi, tol=1e-13, maxiter=20000):
    """L = |D^{-1} phi|^2 and its derivatives: psi = D^{-1} phi, chi = D^{-dagger} psi =
    gamma_5 D^{-1} gamma_5 psi (D^dagger = gamma_5 D gamma_5), then the force bilinear and dL/dc_SW.
    Both solves are the plain FP64 BiCGStab."""
    U = _c128(U)
    C = clover_field(p, U)
    r1 = bicgstab(p, U, C, None, phi, op=OP_D, tol=tol, maxiter=maxiter)
    if r1.status != 0:
        raise RuntimeError(f"oracle solve failed ({r1.status})")
    psi = r1.x
    r2 = bicgstab(p, U, C, None, gamma5_apply(psi), op=OP_D, tol=tol, maxiter=maxiter)
    if r2.status != 0:
        raise RuntimeError(f"oracle adjoint solve failed ({r2.status})")
    chi = gamma5_apply(r2.x)
    L = float(np.vdot(psi, psi).real)
    return LossGrad(L, psi, chi, force(p, U, psi, chi), dcsw(p, U, psi, chi))


class Oracle:
    """Convenience holder: parameters, links and the clover fields built from them."""

    def __init__(self, p, U):
        self.p = p
        self.U = _c128(U)
        self.C = clover_field(p, self.U)
        self.Cinv = clover_inverse(p, self.C)

    def D(self, x):
        return dirac_D(self.p, self.U, self.C, x)

    def A(self, x):
        return dirac_A(self.p, self.U, self.Cinv, x)

    def sap(self, b):
        return sap(self.p, self.U, self.Cinv, b)

    def amsap(self, b):
        return amsap(self.p, self.U, self.Cinv, b)

    def solve(self, b, op=OP_D, tol=1e-10, maxiter=10000):
        return bicgstab(self.p, self.U, self.C, self.Cinv, b, op=op, tol=tol, maxiter=maxiter)

    def dci(self, b, **kw):
        return dci(self.p, self.U, self.C, self.Cinv, b, **kw)
