"""Edge cases, error paths, invariants at sizes the oracle cannot reach quickly,
and determinism of the HIP path, all through the C ABI.

Invariants checked on the GPU path alone (no oracle needed at any size):
gamma_5-hermiticity <y, D^dagger x> = <D y, x>, the free-field plane-wave
closed form, and gauge covariance D[U^Om](Om x) = Om D[U] x.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_2109_10687_amd as dd
import synth

pytestmark = pytest.mark.gpu


def make(dims, block=(4, 4, 4, 4), kappa=0.1365, csw=1.7, eps=0.3, seed=3, **kw):
    p = dd.Params(dims=dims, kappa=kappa, csw=csw, block=block, **kw)
    U = synth.su3_links(dims, eps, seed, device="cuda")
    return dd.Solver(p, U), U


def vdot(a, b):
    return torch.sum(a.conj() * b).item()


# ------------------------------------------------------------------ invariants at size

def test_gamma5_hermiticity_16x16x16x32():
    s, _ = make((16, 16, 16, 32))
    x = synth.gaussian_spinor(s.params.dims, 1, device="cuda")
    y = synth.gaussian_spinor(s.params.dims, 2, device="cuda")
    lhs = vdot(y, s.apply(x, op=dd.DD_OP_DDAG))
    rhs = vdot(s.apply(y, op=dd.DD_OP_D), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_free_field_plane_wave_32x16x16x16():
    dims = (32, 16, 16, 16)
    kappa = 0.125
    p = dd.Params(dims=dims, kappa=kappa, csw=1.7)
    s = dd.Solver(p, synth.unit_links(dims, device="cuda"))
    k = (3, 1, 5, 2)
    mom = [2 * math.pi * k[0] / 32, 2 * math.pi * k[1] / 16, 2 * math.pi * k[2] / 16, (2 * k[3] + 1) * math.pi / 16]
    t, z, y, x = torch.meshgrid(*[torch.arange(L, dtype=torch.float64) for L in reversed(dims)], indexing="ij")
    ph = torch.exp(1j * (mom[0] * x + mom[1] * y + mom[2] * z + mom[3] * t))
    u = torch.arange(12, dtype=torch.float64).reshape(3, 4) * (0.3 - 0.2j) + 0.5
    psi = (ph[..., None, None] * u).cuda().contiguous()
    M = (1 - 2 * kappa * sum(math.cos(m) for m in mom)) * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 2j * kappa * math.sin(mom[mu]) * O.gamma(mu)
    want = ph[..., None, None] * torch.einsum("ij,aj->ai", torch.from_numpy(M), u)
    got = s.apply(psi, op=dd.DD_OP_D).cpu()
    assert (got - want).abs().max().item() < 1e-13
    # the FP32 A apply on the same wave: the clover vanishes, so A = D
    got32 = s.apply(psi, op=dd.DD_OP_A, prec=dd.DD_F32).cpu()
    assert ((got32 - want).norm() / want.norm()).item() < 1e-6


def test_gauge_covariance_16x8x8x16():
    dims = (16, 8, 8, 16)
    p = dd.Params(dims=dims, kappa=0.1365, csw=1.7)
    U = synth.su3_links(dims, 0.3, 11, device="cuda")
    Om = synth.gauge_transform(dims, 12, device="cuda")
    Ug = torch.empty_like(U)
    for mu in range(4):
        Om_fwd = torch.roll(Om, -1, dims=3 - mu)
        Ug[mu] = Om @ U[mu] @ Om_fwd.conj().transpose(-1, -2).contiguous()
    x = synth.gaussian_spinor(dims, 13, device="cuda")
    s1, s2 = dd.Solver(p, U), dd.Solver(p, Ug.contiguous())
    lhs = s2.apply((Om @ x).contiguous(), op=dd.DD_OP_D)
    rhs = Om @ s1.apply(x, op=dd.DD_OP_D)
    assert ((lhs - rhs).abs().max() / rhs.abs().max()).item() < 1e-13


# ------------------------------------------------------------------ degenerate inputs and errors

def test_zero_source_gives_zero_solution():
    s, _ = make((8, 8, 8, 8))
    b = s.new_spinor()
    for mode in (dd.DD_SOLVE_F64_PLAIN, dd.DD_SOLVE_F32_SAP, dd.DD_SOLVE_MIXED, dd.DD_SOLVE_MIXED_GCR,
                 dd.DD_SOLVE_FGMRES):
        x0 = synth.gaussian_spinor(s.params.dims, 5, device="cuda")
        x, info = s.solve(b, tol=1e-10, maxiter=10, mode=mode, x0=x0)
        assert info["status"] == "DD_OK"
        assert x.abs().max().item() == 0.0


def test_nonfinite_source_is_rejected_and_x_untouched():
    s, _ = make((8, 8, 8, 8))
    b = synth.gaussian_spinor(s.params.dims, 6, device="cuda")
    b[0, 0, 0, 0, 1, 2] = float("nan")
    x = torch.full_like(b, 7.0)
    with pytest.raises(dd.DDError) as e:
        dd.bicgstab_solve(s.ctx, x, b, 1e-10, 100, dd.DD_SOLVE_MIXED, s.shape)
    assert e.value.status == -5
    assert torch.all(x == 7.0)


def test_maxiter_reached_returns_not_converged():
    s, _ = make((8, 8, 8, 8))
    b = synth.gaussian_spinor(s.params.dims, 7, device="cuda")
    x, info = s.solve(b, tol=1e-10, maxiter=1, mode=dd.DD_SOLVE_F64_PLAIN)
    assert info["status"] == "DD_NOT_CONVERGED" and info["iters_inner_total"] == 1
    assert 1e-10 < info["relres_true"] < 1.0


@pytest.mark.parametrize("mode", [dd.DD_SOLVE_MIXED, dd.DD_SOLVE_FGMRES])
def test_resume_from_previous_solution(mode):
    s, _ = make((8, 8, 8, 8))
    b = synth.gaussian_spinor(s.params.dims, 8, device="cuda")
    x1, i1 = s.solve(b, tol=1e-6, mode=mode)
    x2, i2 = s.solve(b, tol=1e-10, mode=mode, x0=x1)
    assert i2["status"] == "DD_OK" and i2["relres_true"] < 1e-10
    assert i2["iters_outer"] < 3


def test_fgmres_cycle_of_one_restarts_and_maxiter_caps():
    """fgmres_nkv = 1 restarts after every outer iteration (each cycle then is one defect-correction
    pass with a least-squares step length); maxiter caps the outer iterations."""
    dims = (8, 8, 8, 8)
    p = dd.Params(dims=dims, kappa=0.13, csw=1.5, fgmres_nkv=1)
    s = dd.Solver(p, synth.su3_links(dims, 0.3, 91, device="cuda"))
    b = synth.gaussian_spinor(dims, 92, device="cuda")
    x, info = s.solve(b, tol=1e-10, maxiter=20, mode=dd.DD_SOLVE_FGMRES)
    assert info["status"] == "DD_OK" and info["relres_true"] < 1e-10 and info["iters_outer"] >= 2
    x, info = s.solve(b, tol=1e-10, maxiter=1, mode=dd.DD_SOLVE_FGMRES)
    assert info["status"] == "DD_NOT_CONVERGED" and info["iters_outer"] == 1 and info["relres_true"] < 1e-3


@pytest.mark.parametrize("flags,level", [(0, 0), (dd.DD_DEBUG_ZERO_OMEGA_F16, 1),
                                         (dd.DD_DEBUG_ZERO_OMEGA_F16 | dd.DD_DEBUG_ZERO_OMEGA_F32, 2)])
def test_precision_fallback_after_forced_breakdown(flags, level):
    """omega forced to zero from the host in every FP16-SAP inner iteration (and in every FP32-SAP
    one): every pass of such a level breaks down after its first half step (a pass that still gained
    10x is restarted once), the solve falls back to FP32 SAP-BiCGStab (then to plain FP64 BiCGStab)
    and still reaches 1e-10, checked by the oracle's residual."""
    dims, kappa, csw = (8, 8, 8, 8), 0.13, 1.5
    U = synth.su3_links(dims, 0.3, 41)
    s = dd.Solver(dd.Params(dims=dims, kappa=kappa, csw=csw, debug_flags=flags), U.cuda())
    b = synth.gaussian_spinor(dims, 42)
    x, info = s.solve(b.cuda(), tol=1e-10, maxiter=20, mode=dd.DD_SOLVE_MIXED)
    assert info["status"] == "DD_OK" and info["precision_level"] == level, info
    orc = O.Oracle(O.Params(dims=dims, kappa=kappa, csw=csw, block=(4, 4, 4, 4)), U.numpy())
    r = b.numpy() - orc.D(x.cpu().numpy())
    assert np.linalg.norm(r.ravel()) / np.linalg.norm(b.numpy().ravel()) < 1e-10
    h = s.history()["outer"]
    assert all(h[i + 1] < h[i] for i in range(len(h) - 1))


def test_forced_breakdown_without_fallback_is_reported():
    """With no_fallback the forced inner breakdowns stay at the FP16 SAP: the solve keeps its best
    iterate and reports DD_NOT_CONVERGED or DD_BREAKDOWN, never DD_OK, within maxiter passes."""
    dims = (8, 8, 8, 8)
    p = dd.Params(dims=dims, kappa=0.13, csw=1.5, no_fallback=1, debug_flags=dd.DD_DEBUG_ZERO_OMEGA_F16)
    s = dd.Solver(p, synth.su3_links(dims, 0.3, 41, device="cuda"))
    b = synth.gaussian_spinor(dims, 42, device="cuda")
    x, info = s.solve(b, tol=1e-10, maxiter=4, mode=dd.DD_SOLVE_MIXED)
    assert info["status"] in ("DD_NOT_CONVERGED", "DD_BREAKDOWN") and info["precision_level"] == 0, info
    assert info["iters_outer"] <= 4 and info["relres_true"] <= 1.0


def test_operator_precision_combinations_and_state():
    p = dd.Params(dims=(8, 8, 8, 8), kappa=0.13, csw=1.0)
    s = dd.Solver(p)
    x = s.new_spinor()
    with pytest.raises(dd.DDError) as e:
        s.apply(x, op=dd.DD_OP_D)
    assert e.value.status == -7  # no gauge field yet
    s.load_gauge(synth.su3_links(p.dims, 0.3, 1, device="cuda"))
    with pytest.raises(dd.DDError) as e:
        s.apply(x, op=dd.DD_OP_D, prec=dd.DD_F32)
    assert e.value.status == -1
    with pytest.raises(dd.DDError) as e:
        s.precondition(x, prec=dd.DD_F64)
    assert e.value.status == -1


def test_clover_not_positive_definite_is_reported():
    p = dd.Params(dims=(8, 8, 8, 8), kappa=0.5, csw=50.0)
    s = dd.Solver(p)
    with pytest.raises(dd.DDError) as e:
        s.load_gauge(synth.su3_links(p.dims, 0.8, 1, device="cuda"))
    assert e.value.status == -6


def test_nonfinite_gauge_field_is_rejected():
    p = dd.Params(dims=(8, 8, 8, 8), kappa=0.13, csw=1.0)
    U = synth.su3_links(p.dims, 0.3, 1, device="cuda")
    U[2, 1, 1, 1, 1, 0, 0] = float("inf")
    s = dd.Solver(p)
    with pytest.raises(dd.DDError) as e:
        s.load_gauge(U)
    assert e.value.status == -5


def test_lattice_beyond_device_memory_is_refused_and_released():
    """96^3 x 128 needs about 530 GB of fields against the 288 GB of one MI355X: dd_create fails
    part-way with DD_ERR_NOMEM, frees what it had allocated, and a context made afterwards works."""
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    with pytest.raises(dd.DDError) as e:
        dd.dd_create(dd.Params(dims=(96, 96, 96, 128), kappa=0.13, csw=1.7))
    assert e.value.status == -4
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 > free0 - (1 << 30)  # nothing of the failed context is left behind
    s, U = make((8, 8, 8, 8))
    x = synth.gaussian_spinor((8, 8, 8, 8), 9, device="cuda")
    assert torch.isfinite(s.apply(x, op=dd.DD_OP_D, prec=dd.DD_F64)).all()


def test_minimal_lattice_one_block_pair_per_direction():
    """The smallest legal geometry: two blocks per direction."""
    dims = (4, 4, 4, 4)
    p = dd.Params(dims=dims, kappa=0.12, csw=1.0, block=(2, 2, 2, 2))
    U = synth.su3_links(dims, 0.5, 9)
    s = dd.Solver(p, U.cuda())
    b = synth.gaussian_spinor(dims, 10)
    x, info = s.solve(b.cuda(), tol=1e-12, maxiter=20, mode=dd.DD_SOLVE_MIXED)
    orc = O.Oracle(O.Params(dims=dims, kappa=0.12, csw=1.0, block=(2, 2, 2, 2)), U.numpy())
    bn = b.numpy()
    res = np.linalg.norm(bn - orc.D(x.cpu().numpy())) / np.linalg.norm(bn)
    assert info["status"] == "DD_OK" and res < 1e-12


# ------------------------------------------------------------------ determinism

def test_solve_is_bitwise_deterministic():
    s, _ = make((16, 16, 16, 16))
    b = synth.gaussian_spinor(s.params.dims, 11, device="cuda")
    x1, i1 = s.solve(b, tol=1e-10, mode=dd.DD_SOLVE_MIXED)
    x2, i2 = s.solve(b, tol=1e-10, mode=dd.DD_SOLVE_MIXED)
    assert i1["iters_inner_total"] == i2["iters_inner_total"]
    assert torch.equal(x1, x2)
