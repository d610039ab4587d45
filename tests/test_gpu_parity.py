"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sizes: the 4^4 correctness lattice (2^4 blocks), an anisotropic lattice with
mixed block extents, 8^4 with the 32^4 / 64^3 x 128 operator parameters
(kappa 0.1365, c_SW 1.7, links exp(0.3 i H), 4^4 blocks), and 8^4 with 4^4
blocks and a complex boundary phase in every direction.  Every case spans
several Schwarz blocks and several workgroups.

Bars: FP64 Dirac apply within 1e-13 (relative, max norm); FP32 Dirac apply
within 1e-6 relative (L2), the bound the FP32 operator must meet; FP32 SAP
within 1e-5; FP16-storage results within about three times the largest error
measured over these cases (A 1e-3; SAP 3e-3 with packed FP16 arithmetic,
1.2e-3 with FP32 arithmetic); solves must reach the requested true FP64
residual, recomputed by the oracle on the GPU's solution.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2109_10687_amd as dd
import synth

pytestmark = pytest.mark.gpu

CASES = {
    # name: dims, block, kappa, csw, eps, phases
    "4^4": ((4, 4, 4, 4), (2, 2, 2, 2), 0.12, 1.0, 0.5, (1, 1, 1, -1)),
    "aniso": ((8, 4, 16, 8), (4, 2, 4, 2), 0.13, 1.3, 0.4, (1, np.exp(0.3j), 1, -1)),
    "8^4": ((8, 8, 8, 8), (4, 4, 4, 4), 0.1365, 1.7, 0.3, (1, 1, 1, -1)),
    # 4^4 blocks (the kernels specialised for that shape) with a complex phase in every direction
    "8^4-twist": ((8, 8, 8, 8), (4, 4, 4, 4), 0.125, 1.5, 0.3,
                  (np.exp(0.3j), np.exp(-0.5j), np.exp(1.1j), -np.exp(0.2j))),
}


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


class Case:
    def __init__(self, name, n_sap=2, n_jac=4, seed=101, fp16_arith=0, fused_tail=0):
        dims, block, kappa, csw, eps, phases = CASES[name]
        self.name = name
        self.U = synth.su3_links(dims, eps, seed)
        self.op = O.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases, n_sap=n_sap, n_jac=n_jac)
        self.gp = dd.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases, n_sap=n_sap, n_jac=n_jac,
                            sap_fp16_arith=fp16_arith, sap_fused_tail=fused_tail)
        self.orc = O.Oracle(self.op, self.U.numpy())
        self.solver = dd.Solver(self.gp, self.U.cuda())

    def spinor(self, seed):
        return synth.gaussian_spinor(self.op.dims, seed)


_cache = {}


def case(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _cache:
        _cache[key] = Case(name, **kw)
    return _cache[key]


def g5(x):
    G = O.gamma(4)
    return np.einsum("ij,...aj->...ai", G, x)


@pytest.mark.parametrize("name", list(CASES))
def test_dirac_D_fp64(name):
    c = case(name)
    x = c.spinor(1)
    got = c.solver.apply(x.cuda(), op=dd.DD_OP_D, prec=dd.DD_F64).cpu().numpy()
    want = c.orc.D(x.numpy())
    assert rel_max(got, want) < 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_dirac_Ddag_fp64(name):
    c = case(name)
    x = c.spinor(2)
    got = c.solver.apply(x.cuda(), op=dd.DD_OP_DDAG, prec=dd.DD_F64).cpu().numpy()
    want = g5(c.orc.D(g5(x.numpy())))
    assert rel_max(got, want) < 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_dirac_A_fp32(name):
    c = case(name)
    x = c.spinor(3)
    got = c.solver.apply(x.cuda(), op=dd.DD_OP_A, prec=dd.DD_F32).cpu().numpy()
    want = c.orc.A(x.numpy())
    assert rel_l2(got, want) < 1e-6
    assert rel_max(got, want) < 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_dirac_A_fp16_input(name):
    """The inner solver's apply: FP16-storage input, FP32 links, C_inv and output.  The oracle
    applies A to the values the FP16 field holds, so the FP32 bar applies."""
    c = case(name)
    x = c.spinor(5).cuda()
    f16 = c.solver.pack(x, dd.DD_F16)
    held = c.solver.unpack(f16, dd.DD_F16).cpu().numpy()
    f32 = c.solver.field(dd.DD_F32)
    c.solver.apply_packed_f16in(f32, f16)
    got = c.solver.unpack(f32, dd.DD_F32).cpu().numpy()
    want = c.orc.A(held)
    assert rel_l2(got, want) < 1e-6
    assert rel_max(got, want) < 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_dirac_A_fp16_storage(name):
    c = case(name)
    x = c.spinor(4)
    got = c.solver.apply(x.cuda(), op=dd.DD_OP_A, prec=dd.DD_F16).cpu().numpy()
    want = c.orc.A(x.numpy())
    err = rel_l2(got, want)
    print(f"FP16-storage A apply relative L2 error {err:.3e}")
    assert err < 1e-3


@pytest.mark.parametrize("name,n_sap", [("4^4", 0), ("4^4", 2), ("aniso", 1), ("8^4", 0), ("8^4", 1), ("8^4", 2)])
def test_sap_fp32(name, n_sap):
    c = case(name, n_sap=n_sap)
    b = c.spinor(5)
    got = c.solver.precondition(b.cuda(), prec=dd.DD_F32).cpu().numpy()
    want = c.orc.sap(b.numpy())
    assert rel_l2(got, want) < 1e-5


@pytest.mark.parametrize("name,n_sap", [("4^4", 0), ("4^4", 2), ("aniso", 1), ("8^4", 2), ("8^4-twist", 4)])
def test_amsap_fp32_fused_tail(name, n_sap):
    """Alg. 3 at FP32: A M_SAP b from the fused tail against the oracle's A(M_SAP b), within the FP32
    SAP bar, and against the GPU's own FP32 A applied to its M_SAP b (the separate product the
    fused tail replaces) within FP32 rounding."""
    c = case(name, n_sap=n_sap)
    b = c.spinor(11)
    got = c.solver.amsap(b.cuda(), prec=dd.DD_F32).cpu().numpy()
    want = c.orc.amsap(b.numpy())
    assert rel_l2(got, want) < 1e-5
    mb = c.solver.precondition(b.cuda(), prec=dd.DD_F32)
    sep = c.solver.apply(mb, op=dd.DD_OP_A, prec=dd.DD_F32).cpu().numpy()
    assert rel_l2(got, sep) < 2e-6


@pytest.mark.parametrize("name", ["4^4", "8^4"])
def test_amsap_fp16(name):
    """A M_SAP b with the FP16-storage SAP: the FP32 operator on its FP16-stored output."""
    c = case(name, fp16_arith=1)
    b = c.spinor(12)
    got = c.solver.amsap(b.cuda(), prec=dd.DD_F16).cpu().numpy()
    assert rel_l2(got, c.orc.amsap(b.numpy())) < 3e-3


@pytest.mark.parametrize("fp16_arith", [0, 1])
@pytest.mark.parametrize("name", ["4^4", "aniso", "8^4", "8^4-twist"])
def test_sap_fp16_storage(name, fp16_arith):
    """FP16 storage with FP32 arithmetic, or with packed FP16 block-local
    arithmetic (one rounding of ~5e-4 per operation on a block-normalised source)."""
    c = case(name, fp16_arith=fp16_arith)
    b = c.spinor(6)
    got = c.solver.precondition(b.cuda(), prec=dd.DD_F16).cpu().numpy()
    want = c.orc.sap(b.numpy())
    err = rel_l2(got, want)
    print(f"FP16-storage SAP (fp16 arithmetic {fp16_arith}) relative L2 error {err:.3e}")
    # about three times the largest error measured over these cases (1.26e-3 packed FP16, 4.0e-4 FP32)
    assert err < (3e-3 if fp16_arith else 1.2e-3)


def true_relres(c, x, b):
    return float(np.linalg.norm((b - c.orc.D(x)).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("name", ["4^4", "8^4"])
def test_solve_plain_fp64(name):
    c = case(name)
    b = c.spinor(7)
    x, info = c.solver.solve(b.cuda(), tol=1e-10, maxiter=5000, mode=dd.DD_SOLVE_F64_PLAIN)
    assert info["status"] == "DD_OK", info
    xn = x.cpu().numpy()
    res = true_relres(c, xn, b.numpy())
    assert res < 1e-10 and abs(res - info["relres_true"]) < 1e-11
    ref = c.orc.solve(b.numpy(), op=O.OP_D, tol=1e-12, maxiter=20000)
    assert rel_l2(xn, ref.x) < 1e-7


@pytest.mark.parametrize("fused_tail", [0, 1])
@pytest.mark.parametrize("name", ["4^4", "8^4", "8^4-twist"])
def test_solve_fp32_sap(name, fused_tail):
    """FP32 SAP-BiCGStab, A M_SAP applied separately to the SAP output or by the fused tail of Alg. 3."""
    c = case(name, fused_tail=fused_tail)
    b = c.spinor(8)
    x, info = c.solver.solve(b.cuda(), tol=1e-6, maxiter=500, mode=dd.DD_SOLVE_F32_SAP)
    assert info["status"] == "DD_OK", info
    assert info["relres_inner_last"] < 1e-6
    res = true_relres(c, x.cpu().numpy(), b.numpy())
    print(f"FP32 SAP-BiCGStab: {info['iters_inner_total']} iterations, true residual {res:.2e}")
    assert res < 1e-5


@pytest.mark.parametrize("fp16_arith", [0, 1])
@pytest.mark.parametrize("mode", [dd.DD_SOLVE_MIXED, dd.DD_SOLVE_MIXED_GCR, dd.DD_SOLVE_FGMRES])
@pytest.mark.parametrize("name", ["4^4", "aniso", "8^4", "8^4-twist"])
def test_solve_mixed(name, mode, fp16_arith):
    c = case(name, fp16_arith=fp16_arith)
    b = c.spinor(9)
    x, info = c.solver.solve(b.cuda(), tol=1e-10, maxiter=20, mode=mode)
    assert info["status"] == "DD_OK", info
    xn = x.cpu().numpy()
    res = true_relres(c, xn, b.numpy())
    print(f"mixed: {info['iters_outer']} outer, {info['iters_inner_total']} inner, true residual {res:.2e}")
    assert res < 1e-10
    h = c.solver.history()
    assert len(h["outer"]) == info["iters_outer"] + 1 and len(h["inner"]) == info["iters_inner_total"]
    assert h["outer"][-1] == pytest.approx(info["relres_true"], rel=1e-6)
    ref = c.orc.solve(b.numpy(), op=O.OP_D, tol=1e-12, maxiter=20000)
    assert rel_l2(xn, ref.x) < 1e-7


@pytest.mark.parametrize("name", ["4^4", "8^4"])
def test_sap_fp16_after_gauge_reload(name):
    """The packed-FP16 half-sweep reads per-gauge-field copies of the links and C_inv: after a
    second gauge field is loaded into the same context its SAP must follow the new field."""
    dims, block, kappa, csw, eps, phases = CASES[name]
    op = O.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases, n_sap=2, n_jac=4)
    gp = dd.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases, n_sap=2, n_jac=4, sap_fp16_arith=1)
    U1 = synth.su3_links(dims, eps, 301)
    U2 = synth.su3_links(dims, eps, 302)
    s = dd.Solver(gp, U1.cuda())
    b = synth.gaussian_spinor(dims, 7)
    first = s.precondition(b.cuda(), prec=dd.DD_F16).cpu().numpy()
    s.load_gauge(U2.cuda())
    got = s.precondition(b.cuda(), prec=dd.DD_F16).cpu().numpy()
    want = O.Oracle(op, U2.numpy()).sap(b.numpy())
    assert rel_l2(got, want) < 3e-3
    assert rel_l2(first, want) > 1e-1  # the two fields give different preconditioners
    s.close()
