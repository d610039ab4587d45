"""Pins of the oracle's derivative of L = |D^{-1} phi|^2 with respect to the
links and c_SW (the fermion-force bilinear).

The force is pinned against finite differences of quantities the other pins
already fix (the operator D of the appendix and the plain BiCGStab):
  * the bilinear itself, for arbitrary psi and chi, against central
    differences of D: -2 Re <chi| dD psi> (no solve involved);
  * the loss gradient against differences of L computed with the differenced
    solve  psi+ - psi- = -D+^{-1} (D+ - D-) psi-,  whose source is O(h), so the
    difference is free of solve noise;
  * dL/dc_SW the same way;
  * gauge covariance of the bilinear;
  * the link gradient in PyTorch's convention (grad_from_force) and the source
    gradient 2 chi (source_grad), against central differences of L.
"""
import numpy as np
import pytest

import oracle as O
import synth


def shift(f, mu, d):
    return np.roll(f, -d, axis=3 - mu)


def rand_direction(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def rand_hermitian_traceless(rng):
    Z = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    H = 0.5 * (Z + Z.conj().T)
    return H - np.trace(H) / 3 * np.eye(3)


def expm_herm(T, t):
    """exp(i t T) for Hermitian T"""
    w, v = np.linalg.eigh(T)
    return (v * np.exp(1j * t * w)) @ v.conj().T


def params(dims, kappa=0.12, csw=1.3, tphase=np.exp(0.3j)):
    return O.Params(dims=dims, kappa=kappa, csw=csw, block=(2, 2, 2, 2),
                    phases=(1.0, 1.0, 1.0, tphase))


def delta_loss(p, Up, Um, phi, tol=1e-14):
    """L(Up) - L(Um) through the differenced solve (both in FP64 BiCGStab)."""
    Cp, Cm = O.clover_field(p, Up), O.clover_field(p, Um)
    rm = O.bicgstab(p, Um, Cm, None, phi, op=O.OP_D, tol=tol, maxiter=20000)
    assert rm.status == 0
    psim = rm.x
    src = -(O.dirac_D(p, Up, Cp, psim) - O.dirac_D(p, Um, Cm, psim))
    rd = O.bicgstab(p, Up, Cp, None, src, op=O.OP_D, tol=1e-12, maxiter=20000)
    assert rd.status == 0
    d = rd.x
    return float(np.vdot(d, 2 * psim + d).real)


DIMS = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def setup():
    p = params(DIMS)
    U = synth.su3_links(DIMS, 0.5, 21).numpy()
    phi = synth.gaussian_spinor(DIMS, 22).numpy()
    g = O.loss_and_force(p, U, phi)
    return p, U, phi, g


@pytest.mark.parametrize("csw", [0.0, 1.3])
def test_force_bilinear_is_derivative_of_D(csw):
    """-2 Re <chi| D(U + hE) psi - D(U - hE) psi> / 2h  ==  Re sum tr(E W), any psi, chi."""
    dims = (4, 2, 4, 6)
    p = params(dims, kappa=0.13, csw=csw)
    U = synth.su3_links(dims, 0.4, 31).numpy()
    psi = synth.gaussian_spinor(dims, 32).numpy()
    chi = synth.gaussian_spinor(dims, 33).numpy()
    E = rand_direction(U.shape, 34)
    W = O.force(p, U, psi, chi)
    want = np.sum(np.einsum("...ab,...ba->...", E, W)).real
    h = 1e-5  # central-difference error ~ h^2 (5.7e-8 at h = 1e-4, 5.6e-10 at 1e-5)
    Up, Um = U + h * E, U - h * E
    Dp = O.dirac_D(p, Up, O.clover_field(p, Up), psi)
    Dm = O.dirac_D(p, Um, O.clover_field(p, Um), psi)
    got = -2.0 * np.vdot(chi, Dp - Dm).real / (2 * h)
    assert abs(got - want) <= 1e-8 * abs(want)


def test_force_gauge_covariance():
    """U_mu(n) -> Om(n) U Om(n+mu)^dagger, psi, chi -> Om psi, Om chi  give
    W_mu(n) -> Om(n+mu) W_mu(n) Om(n)^dagger."""
    dims = (4, 4, 2, 4)
    p = params(dims, kappa=0.125, csw=1.7)
    U = synth.su3_links(dims, 0.3, 41).numpy()
    Om = synth.gauge_transform(dims, 42).numpy()
    psi = synth.gaussian_spinor(dims, 43).numpy()
    chi = synth.gaussian_spinor(dims, 44).numpy()
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], shift(Om, mu, +1).conj())
    rot = lambda x: np.einsum("...ab,...bs->...as", Om, x)
    W = O.force(p, U, psi, chi)
    Wg = O.force(p, Ug, rot(psi), rot(chi))
    for mu in range(4):
        want = np.einsum("...ab,...bc,...dc->...ad", shift(Om, mu, +1), W[mu], Om.conj())
        np.testing.assert_allclose(Wg[mu], want, atol=1e-12 * np.abs(W).max())


def test_loss_gradient_global_direction(setup):
    """(L(U + hE) - L(U - hE)) / 2h against Re sum tr(E W) for a random complex E on every link."""
    p, U, phi, g = setup
    E = rand_direction(U.shape, 51)
    want = np.sum(np.einsum("...ab,...ba->...", E, g.W)).real
    h = 1e-6
    got = delta_loss(p, U + h * E, U - h * E, phi) / (2 * h)
    assert abs(got - want) <= 1e-7 * abs(want)


def test_loss_gradient_single_links_su3(setup):
    """U -> exp(i t T) U on single links (one per direction, two crossing the lattice edge where
    the boundary phase acts): dL/dt = tr(T F) with F the su(3) projection of the force."""
    p, U, phi, g = setup
    F = O.su3_force(U, g.W)
    # F is Hermitian and traceless
    np.testing.assert_allclose(F, np.conj(np.swapaxes(F, -1, -2)), atol=1e-12 * np.abs(F).max())
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-12 * np.abs(F).max()
    rng = np.random.default_rng(61)
    links = [(0, (1, 2, 3, 0)), (1, (0, 3, 1, 2)), (2, (2, 1, 0, 3)), (3, (3, 0, 2, 1)),
             (3, (1, 1, 1, 3)), (0, (3, 2, 2, 2))]  # (mu, (x, y, z, t)); the last two wrap
    h = 1e-6
    for mu, (x, y, z, t) in links:
        T = rand_hermitian_traceless(rng)
        Up, Um = U.copy(), U.copy()
        Up[mu, t, z, y, x] = expm_herm(T, h) @ U[mu, t, z, y, x]
        Um[mu, t, z, y, x] = expm_herm(T, -h) @ U[mu, t, z, y, x]
        got = delta_loss(p, Up, Um, phi) / (2 * h)
        want = np.trace(T @ F[mu, t, z, y, x]).real
        assert abs(got - want) <= 1e-6 * abs(want) + 1e-10 * np.abs(F).max(), (mu, x, y, z, t, got, want)


@pytest.mark.parametrize("csw", [0.0, 1.3])
def test_dcsw_finite_difference(csw):
    """dL/dc_SW against central differences in c_SW (also at c_SW = 0, where the clover vanishes
    but its derivative does not)."""
    p = params(DIMS, csw=csw)
    U = synth.su3_links(DIMS, 0.5, 21).numpy()
    phi = synth.gaussian_spinor(DIMS, 22).numpy()
    g = O.loss_and_force(p, U, phi)
    h = 1e-6
    pp, pm = params(DIMS, csw=csw + h), params(DIMS, csw=csw - h)
    # L(csw + h) - L(csw - h) with the differenced solve
    Cp, Cm = O.clover_field(pp, U), O.clover_field(pm, U)
    rm = O.bicgstab(pm, U, Cm, None, phi, op=O.OP_D, tol=1e-14, maxiter=20000)
    src = -(O.dirac_D(pp, U, Cp, rm.x) - O.dirac_D(pm, U, Cm, rm.x))
    rd = O.bicgstab(pp, U, Cp, None, src, op=O.OP_D, tol=1e-12, maxiter=20000)
    dL = float(np.vdot(rd.x, 2 * rm.x + rd.x).real)
    got = dL / (2 * h)
    assert abs(got - g.dcsw) <= 1e-7 * abs(g.dcsw)


def test_loss_and_adjoint_solution(setup):
    """psi solves D psi = phi, chi solves D^dagger chi = psi (D^dagger = gamma_5 D gamma_5, itself
    pinned by the gamma_5-hermiticity test), and L = |psi|^2."""
    p, U, phi, g = setup
    C = O.clover_field(p, U)
    r1 = O.dirac_D(p, U, C, g.psi) - phi
    assert np.linalg.norm(r1) < 1e-12 * np.linalg.norm(phi)
    Ddag_chi = O.gamma5_apply(O.dirac_D(p, U, C, O.gamma5_apply(g.chi)))
    assert np.linalg.norm(Ddag_chi - g.psi) < 1e-12 * np.linalg.norm(g.psi)
    assert abs(g.loss - np.vdot(g.psi, g.psi).real) < 1e-12 * g.loss


def test_link_gradient_in_torch_convention(setup):
    """grad_from_force gives PyTorch's gradient of a real function of complex entries,
    G = dL/dRe U + i dL/dIm U, for which dL = Re sum conj(G) dU: pinned by central differences of L
    along a random complex direction on every link, and along a purely real and a purely imaginary
    one (a transpose without the conjugate, or a conjugate without the transpose, fails them)."""
    p, U, phi, g = setup
    G = O.grad_from_force(g.W)
    rng = np.random.default_rng(71)
    h = 1e-6
    slips = {"transpose only": np.swapaxes(g.W, -1, -2), "conjugate only": np.conj(g.W), "W itself": g.W}
    missed = {k: False for k in slips}
    for kind in ("complex", "real", "imag"):
        E = rng.normal(size=U.shape) + (1j * rng.normal(size=U.shape) if kind == "complex" else 0)
        if kind == "imag":
            E = 1j * E
        want = float(np.sum(np.conj(G) * E).real)
        got = delta_loss(p, U + h * E, U - h * E, phi) / (2 * h)
        assert abs(got - want) <= 1e-7 * abs(want), (kind, got, want)
        for k, wrong in slips.items():
            missed[k] |= abs(got - float(np.sum(np.conj(wrong) * E).real)) > 1e-3 * abs(want)
    # each plausible slip in the convention fails along at least one of the directions
    assert all(missed.values()), missed


def test_source_gradient_finite_difference(setup):
    """source_grad(chi) = 2 chi is the gradient of L in phi in PyTorch's convention: the central
    difference of L along a random complex direction E (L is quadratic in phi, so the difference is
    exact up to the solves' rounding) equals Re sum conj(2 chi) E."""
    p, U, phi, g = setup
    C = O.clover_field(p, U)
    E = rand_direction(phi.shape, 72)
    h = 1e-3
    L = []
    for sgn in (+1, -1):
        r = O.bicgstab(p, U, C, None, phi + sgn * h * E, op=O.OP_D, tol=1e-14, maxiter=20000)
        assert r.status == 0
        L.append(float(np.vdot(r.x, r.x).real))
    got = (L[0] - L[1]) / (2 * h)
    want = float(np.sum(np.conj(O.source_grad(g.chi)) * E).real)
    assert abs(got - want) <= 1e-8 * abs(want), (got, want)
