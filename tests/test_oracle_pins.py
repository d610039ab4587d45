"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test pins one piece of the oracle to something other than the oracle
itself: the gamma matrices printed in the appendix, the Clifford algebra, the
free-field plane-wave closed form, gamma_5-hermiticity, gauge covariance, a
constant abelian field with a closed-form clover, the support of the clover of
a single excited link, dense LU on 4^4, the Neumann-series forms of Alg. 2 and
Alg. 1, and the block-triangular identity of A K for exact block inverses.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.lapack

import oracle as O
import synth


# ---------------------------------------------------------------- helpers

def read_gammas(golden_dir):
    mats, cur = {}, None
    with open(f"{golden_dir}/gamma_matrices.txt") as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("gamma"):
                cur = line
                mats[cur] = []
            else:
                mats[cur].append([complex(v) for v in line.split()])
    return [np.array(mats[f"gamma{k}"]) for k in (1, 2, 3, 4)]


def shift(f, mu, d):
    """f(n + d*mu_hat) at n for a field with leading site axes (t, z, y, x)."""
    return np.roll(f, -d, axis=3 - mu)


def spin_apply(M, psi):
    """apply a 4x4 spin matrix to psi[..., colour, spin]"""
    return np.einsum("ij,...aj->...ai", M, psi)


def colour_apply(W, psi):
    """apply per-site 3x3 colour matrices W[t,z,y,x,a,b] to psi[t,z,y,x,b,s]"""
    return np.einsum("...ab,...bs->...as", W, psi)


def dense(op, shape):
    """dense matrix of a linear map on spinor fields of the given shape"""
    N = int(np.prod(shape))
    M = np.zeros((N, N), dtype=np.complex128)
    e = np.zeros(N, dtype=np.complex128)
    for j in range(N):
        e[:] = 0
        e[j] = 1
        M[:, j] = op(e.reshape(shape)).reshape(N)
    return M


def eo_index(p):
    """flat spinor indices of the E rows and of the O rows"""
    col = O.colour_mask(p).reshape(-1)
    per = np.repeat(col, 12)
    return np.nonzero(per == 0)[0], np.nonzero(per == 1)[0]


P44 = dict(dims=(4, 4, 4, 4), kappa=0.12, csw=1.0, block=(2, 2, 2, 2), n_sap=2, n_jac=4)


@pytest.fixture(scope="module")
def cfg1():
    p = O.Params(**P44)
    U = synth.su3_links(p.dims, 0.5, 11).numpy()
    return O.Oracle(p, U)


@pytest.fixture(scope="module")
def dense_cfg1(cfg1):
    shp = cfg1.p.shape + (3, 4)
    return dense(cfg1.D, shp), dense(cfg1.A, shp)


# ---------------------------------------------------------------- gamma matrices (appendix)

def test_gamma_matrices_match_paper(golden_dir):
    paper = read_gammas(golden_dir)
    for mu in range(4):
        np.testing.assert_array_equal(O.gamma(mu), paper[mu])


def test_gamma_clifford_hermitian_gamma5(golden_dir):
    g = [O.gamma(mu) for mu in range(4)]
    for mu in range(4):
        np.testing.assert_allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            np.testing.assert_allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=0)
    g5 = O.gamma(4)
    want = np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]])
    np.testing.assert_allclose(g5, want, atol=0)
    for mu in range(4):
        np.testing.assert_allclose(g5 @ g[mu] + g[mu] @ g5, 0, atol=0)


# ---------------------------------------------------------------- synthetic links

def test_su3_links_unitary_det_one():
    U = synth.su3_links((4, 4, 4, 4), 0.3, 5).numpy().reshape(-1, 3, 3)
    UU = np.einsum("nab,ncb->nac", U, U.conj())
    assert np.abs(UU - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    # eps sets the distance from the identity: mean Re tr U / 3 shrinks as eps grows
    U5 = synth.su3_links((4, 4, 4, 4), 0.5, 5).numpy().reshape(-1, 3, 3)
    assert np.trace(U5, axis1=1, axis2=2).real.mean() < np.trace(U, axis1=1, axis2=2).real.mean() < 3.0


# ---------------------------------------------------------------- hopping term: free field closed form

@pytest.mark.parametrize("k", [(0, 0, 0, 0), (1, 2, 1, 3), (3, 5, 1, 6)])
def test_free_field_plane_wave(k):
    """With U = 1 the clover vanishes and D acts on exp(i p.n) u as
    1 - 2 kappa sum cos p + 2 i kappa sum gamma_mu sin p_mu, with
    p_mu = (2 pi k_mu + theta_mu) / L_mu for a boundary phase exp(i theta_mu)."""
    dims = (4, 6, 2, 8)
    theta = (0.0, 0.7, 0.0, np.pi)
    kappa = 0.137
    p = O.Params(dims=dims, kappa=kappa, csw=1.3, block=(2, 2, 2, 2),
                 phases=tuple(np.exp(1j * th) for th in theta))
    U = synth.unit_links(dims).numpy()
    orc = O.Oracle(p, U)
    assert np.abs(orc.C).max() == 0.0
    mom = [(2 * np.pi * k[mu] + theta[mu]) / dims[mu] for mu in range(4)]
    rng = np.random.default_rng(0)
    u = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    t, z, y, x = np.meshgrid(*[np.arange(L) for L in reversed(dims)], indexing="ij")
    ph = np.exp(1j * (mom[0] * x + mom[1] * y + mom[2] * z + mom[3] * t))
    psi = ph[..., None, None] * u
    M = (1 - 2 * kappa * sum(np.cos(m) for m in mom)) * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 2j * kappa * np.sin(mom[mu]) * O.gamma(mu)
    want = ph[..., None, None] * spin_apply(M, u)
    np.testing.assert_allclose(orc.D(psi), want, atol=1e-13)


def test_free_field_solve_closed_form():
    """D^{-1} of a plane wave is (a - i b.gamma)/(a^2 + |b|^2) times it,
    a = 1 - 2 kappa sum cos p, b_mu = 2 kappa sin p_mu."""
    dims = (4, 4, 4, 8)
    kappa = 0.12
    p = O.Params(dims=dims, kappa=kappa, csw=1.0, block=(2, 2, 2, 2))
    orc = O.Oracle(p, synth.unit_links(dims).numpy())
    k = (1, 0, 2, 1)
    mom = [2 * np.pi * k[0] / 4, 0.0, 2 * np.pi * k[2] / 4, (2 * k[3] + 1) * np.pi / 8]
    u = np.arange(12).reshape(3, 4) * (1 + 0.5j) + 1.0
    t, z, y, x = np.meshgrid(*[np.arange(L) for L in reversed(dims)], indexing="ij")
    ph = np.exp(1j * (mom[0] * x + mom[1] * y + mom[2] * z + mom[3] * t))
    src = ph[..., None, None] * u
    a = 1 - 2 * kappa * sum(np.cos(m) for m in mom)
    b = [2 * kappa * np.sin(m) for m in mom]
    Minv = (a * np.eye(4) - 1j * sum(b[mu] * O.gamma(mu) for mu in range(4))) / (a * a + sum(v * v for v in b))
    want = ph[..., None, None] * spin_apply(Minv, u)
    r = orc.solve(src, op=O.OP_D, tol=1e-12, maxiter=500)
    assert r.status == 0
    np.testing.assert_allclose(r.x, want, atol=1e-10 * np.abs(want).max())


# ---------------------------------------------------------------- adjoint structure and covariance

def test_gamma5_hermiticity(cfg1):
    g5 = O.gamma(4)
    x = synth.gaussian_spinor(cfg1.p.dims, 1).numpy()
    y = synth.gaussian_spinor(cfg1.p.dims, 2).numpy()
    lhs = np.vdot(y, spin_apply(g5, cfg1.D(spin_apply(g5, x))))
    rhs = np.vdot(cfg1.D(y), x)
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs) * 10


def test_gamma5_hermiticity_with_phase():
    dims = (4, 2, 4, 6)
    p = O.Params(dims=dims, kappa=0.13, csw=1.7, block=(2, 2, 2, 2), phases=(1, np.exp(0.4j), 1, -1))
    orc = O.Oracle(p, synth.su3_links(dims, 0.3, 3).numpy())
    g5 = O.gamma(4)
    x = synth.gaussian_spinor(dims, 1).numpy()
    y = synth.gaussian_spinor(dims, 2).numpy()
    lhs = np.vdot(y, spin_apply(g5, orc.D(spin_apply(g5, x))))
    rhs = np.vdot(orc.D(y), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_gauge_covariance():
    """U_mu(n) -> Om(n) U_mu(n) Om(n+mu)^dagger and x(n) -> Om(n) x(n) give
    D[U^Om](Om x) = Om D[U] x, clover included."""
    dims = (4, 4, 2, 6)
    p = O.Params(dims=dims, kappa=0.1365, csw=1.7, block=(2, 2, 2, 2))
    U = synth.su3_links(dims, 0.3, 7).numpy()
    Om = synth.gauge_transform(dims, 8).numpy()
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], shift(Om, mu, +1).conj())
    x = synth.gaussian_spinor(dims, 9).numpy()
    o1, o2 = O.Oracle(p, U), O.Oracle(p, Ug)
    lhs = o2.D(colour_apply(Om, x))
    rhs = colour_apply(Om, o1.D(x))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13 * np.abs(rhs).max())
    # the clover block itself rotates as Om(n) C(n) Om(n)^dagger
    Omk = np.einsum("...ab,ij->...aibj", Om, np.eye(4)).reshape(o1.C.shape)
    np.testing.assert_allclose(o2.C, Omk @ o1.C @ Omk.conj().swapaxes(-1, -2), atol=1e-13)


# ---------------------------------------------------------------- clover normalisation and geometry

def test_clover_constant_abelian_field(golden_dir):
    """U_x(n) = exp(i theta y), U_y(x, y=L-1) = exp(-i theta L x), theta = 2 pi / L^2:
    every xy plaquette equals exp(-i theta), so F_xy = -i sin(theta) and
    C = kappa c_SW sin(theta) sigma_12 with sigma_12 = (i/2)[gamma_1, gamma_2];
    1 + C has eigenvalues 1 +- kappa c_SW sin(theta)."""
    L = 4
    dims = (L, L, 2, 2)
    kappa, csw = 0.1365, 1.7
    theta = 2 * np.pi / L ** 2
    U = synth.unit_links(dims).numpy()
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in reversed(dims)], indexing="ij")
    U[0] = np.exp(1j * theta * y)[..., None, None] * np.eye(3)
    yl = (y == L - 1)
    U[1][yl] = np.exp(-1j * theta * L * x[yl])[..., None, None] * np.eye(3)
    p = O.Params(dims=dims, kappa=kappa, csw=csw, block=(2, 2, 2, 2))
    C = O.clover_field(p, U)
    g1, g2 = read_gammas(golden_dir)[:2]
    sigma12 = 0.5j * (g1 @ g2 - g2 @ g1)
    want = kappa * csw * np.sin(theta) * np.kron(np.eye(3), sigma12)
    np.testing.assert_allclose(C, np.broadcast_to(want, C.shape), atol=1e-15)
    ev = np.linalg.eigvalsh(np.eye(12) + C.reshape(-1, 12, 12)[0])
    d = kappa * csw * np.sin(theta)
    np.testing.assert_allclose(ev, [1 - d] * 6 + [1 + d] * 6, atol=1e-14)


def test_clover_support_of_single_link():
    """Exciting one link U_x(n0) of the free field excites the clover exactly at
    the far corners n0 +- nu, n0 + x +- nu (nu != x) of the six plaquettes that
    contain it.  At the link's own ends n0 and n0 + x the two leaves of each
    plane run through the link in opposite senses (U and U^dagger), so F
    cancels there."""
    dims = (4, 4, 4, 4)
    p = O.Params(dims=dims, kappa=0.12, csw=1.0, block=(2, 2, 2, 2))
    U = synth.unit_links(dims).numpy()
    n0 = np.array([1, 1, 1, 1])  # (x, y, z, t)
    U[0, n0[3], n0[2], n0[1], n0[0]] = synth.random_su3(1, 0.6, 3).numpy()[0]
    C = O.clover_field(p, U)
    nonzero = np.abs(C).reshape(p.shape + (-1,)).max(-1) > 1e-14
    want = np.zeros(p.shape, dtype=bool)
    ex = np.array([1, 0, 0, 0])
    for nu in (1, 2, 3):
        en = np.eye(4, dtype=int)[nu]
        for s in (+1, -1):
            for corner in (n0 + s * en, n0 + ex + s * en):
                c = corner % np.array(dims)
                want[c[3], c[2], c[1], c[0]] = True
    np.testing.assert_array_equal(nonzero, want)


def test_clover_hermitian_and_inverse(cfg1):
    C = cfg1.C.reshape(-1, 12, 12)
    np.testing.assert_allclose(C, C.conj().swapaxes(1, 2), atol=1e-15)
    M = np.eye(12) + C
    np.testing.assert_allclose(M @ cfg1.Cinv.reshape(-1, 12, 12), np.broadcast_to(np.eye(12), M.shape), atol=1e-13)
    # C commutes with gamma_5 (sigma_{mu nu} does), so 1 + C splits into two 6x6 blocks
    G5 = np.kron(np.eye(3), O.gamma(4))
    np.testing.assert_allclose(G5 @ C, C @ G5, atol=1e-15)


# ---------------------------------------------------------------- operator pieces

def test_A_is_cinv_D(cfg1, dense_cfg1):
    D, A = dense_cfg1
    V = cfg1.p.volume
    Ci = cfg1.Cinv.reshape(V, 12, 12)
    CiD = np.zeros_like(D)
    for n in range(V):
        CiD[n * 12:(n + 1) * 12] = Ci[n] @ D[n * 12:(n + 1) * 12]
    np.testing.assert_allclose(A, CiD, atol=1e-13)


def test_D_sites_matches_full(cfg1):
    x = synth.gaussian_spinor(cfg1.p.dims, 4).numpy()
    full = cfg1.D(x).reshape(-1, 3, 4)
    sites = np.array([0, 7, 63, 100, 255])
    got = O.dirac_D_sites(cfg1.p, cfg1.U, x, sites)
    np.testing.assert_allclose(got, full[sites], atol=1e-14)


def test_A_sites_matches_full(cfg1):
    x = synth.gaussian_spinor(cfg1.p.dims, 5).numpy()
    full = cfg1.A(x).reshape(-1, 3, 4)
    sites = np.array([0, 1, 17, 128, 200, 255])
    got = O.dirac_A_sites(cfg1.p, cfg1.U, x, sites)
    np.testing.assert_allclose(got, full[sites], atol=1e-13)


def test_block_pieces_are_blocks_of_A(cfg1, dense_cfg1):
    """A_EE, A_OO keep in-block hops, A_EO, A_OE cross-block hops: they are the
    four blocks of A in the E/O ordering (Sec. 3), and A_EE never couples
    different blocks."""
    _, A = dense_cfg1
    p = cfg1.p
    E, Oi = eo_index(p)
    shp = p.shape + (3, 4)
    N = A.shape[0]
    rng = np.random.default_rng(1)
    x = (rng.normal(size=N) + 1j * rng.normal(size=N))
    for c, rows, cols_in, cols_out in ((0, E, E, Oi), (1, Oi, Oi, E)):
        xin = np.zeros(N, complex)
        xin[cols_in] = x[cols_in]
        xout = np.zeros(N, complex)
        xout[cols_out] = x[cols_out]
        yin = O.block_apply(p, cfg1.U, cfg1.Cinv, xin.reshape(shp), c, 1).reshape(N)
        yout = O.block_apply(p, cfg1.U, cfg1.Cinv, xout.reshape(shp), c, 2).reshape(N)
        np.testing.assert_allclose(yin[rows], A[np.ix_(rows, cols_in)] @ x[cols_in], atol=1e-13)
        np.testing.assert_allclose(yout[rows], A[np.ix_(rows, cols_out)] @ x[cols_out], atol=1e-13)
    # no coupling between different blocks inside A_EE
    blk = np.zeros(p.shape, dtype=np.int64)
    t, z, y, xx = np.meshgrid(*[np.arange(n) for n in p.shape], indexing="ij")
    blk = (xx // 2) + 2 * ((y // 2) + 2 * ((z // 2) + 2 * (t // 2)))
    bi = np.repeat(blk.reshape(-1), 12)
    AEE = A[np.ix_(E, E)]
    coupled = np.abs(AEE) > 0
    rows, cols = np.nonzero(coupled)
    assert np.all(bi[E][rows] == bi[E][cols])


def test_jacobi_is_truncated_neumann(cfg1, dense_cfg1):
    """Alg. 2 computes B_EE b = sum_{j=0}^{N_JAC} (I - A_EE)^j b."""
    _, A = dense_cfg1
    p = cfg1.p
    E, Oi = eo_index(p)
    b = synth.gaussian_spinor(p.dims, 5).numpy()
    for c, rows in ((0, E), (1, Oi)):
        got = O.jacobi(p, cfg1.U, cfg1.Cinv, b, c).reshape(-1)
        Acc = A[np.ix_(rows, rows)]
        T = np.eye(len(rows)) - Acc
        want = np.zeros(len(rows), complex)
        v = b.reshape(-1)[rows]
        for _ in range(p.n_jac + 1):
            want += v
            v = T @ v
        np.testing.assert_allclose(got[rows], want, atol=1e-12)
        other = Oi if c == 0 else E
        assert np.all(got[other] == 0)


def _dense_K(A, E, Oi, BEE, BOO):
    N = A.shape[0]
    K = np.zeros((N, N), complex)
    K[np.ix_(E, E)] = BEE
    K[np.ix_(Oi, Oi)] = BOO
    K[np.ix_(Oi, E)] = -BOO @ A[np.ix_(Oi, E)] @ BEE
    return K


@pytest.mark.parametrize("n_sap", [0, 1, 2, 4])
def test_sap_is_neumann_series_in_AK(cfg1, dense_cfg1, n_sap):
    """Alg. 1 with loop count n_sap computes K sum_{j=0}^{n_sap} (1 - A K)^j b,
    K = [[B_EE, 0], [-B_OO A_OE B_EE, B_OO]] with the Jacobi B (Sec. 3)."""
    _, A = dense_cfg1
    p = O.Params(**{**P44, "n_sap": n_sap})
    E, Oi = eo_index(p)
    B = []
    for rows in (E, Oi):
        T = np.eye(len(rows)) - A[np.ix_(rows, rows)]
        S, Tj = np.zeros_like(T), np.eye(len(rows))
        for _ in range(p.n_jac + 1):
            S += Tj
            Tj = Tj @ T
        B.append(S)
    K = _dense_K(A, E, Oi, B[0], B[1])
    R = np.eye(A.shape[0]) - A @ K
    b = synth.gaussian_spinor(p.dims, 6).numpy().reshape(-1)
    acc, v = np.zeros_like(b), b.copy()
    for _ in range(n_sap + 1):
        acc += v
        v = R @ v
    want = K @ acc
    got = O.sap(p, cfg1.U, cfg1.Cinv, b.reshape(p.shape + (3, 4))).reshape(-1)
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())
    # and Alg. 3 is A times it
    got3 = O.amsap(p, cfg1.U, cfg1.Cinv, b.reshape(p.shape + (3, 4))).reshape(-1)
    np.testing.assert_allclose(got3, A @ want, atol=1e-12 * np.abs(want).max())


def test_exact_block_inverse_makes_AK_block_triangular(cfg1, dense_cfg1):
    """With B_EE = A_EE^{-1}, B_OO = A_OO^{-1}: the O-E block of A K vanishes and
    its O-O block is the identity (Sec. 3)."""
    _, A = dense_cfg1
    E, Oi = eo_index(cfg1.p)
    BEE = np.linalg.inv(A[np.ix_(E, E)])
    BOO = np.linalg.inv(A[np.ix_(Oi, Oi)])
    AK = A @ _dense_K(A, E, Oi, BEE, BOO)
    np.testing.assert_allclose(AK[np.ix_(Oi, E)], 0, atol=1e-12)
    np.testing.assert_allclose(AK[np.ix_(Oi, Oi)], np.eye(len(Oi)), atol=1e-12)
    np.testing.assert_allclose(AK[np.ix_(E, Oi)], A[np.ix_(E, Oi)] @ BOO, atol=1e-12)


def test_sap_approaches_inverse(cfg1):
    """A M_SAP tends to the identity as the SAP loop count grows."""
    b = synth.gaussian_spinor(cfg1.p.dims, 7).numpy()
    errs = []
    for n_sap in (0, 1, 2, 4):
        p = O.Params(**{**P44, "n_sap": n_sap})
        errs.append(np.linalg.norm(O.amsap(p, cfg1.U, cfg1.Cinv, b) - b) / np.linalg.norm(b))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-2


# ---------------------------------------------------------------- solvers against dense LU

def test_bicgstab_matches_dense_lu(cfg1, dense_cfg1):
    D, A = dense_cfg1
    b = synth.gaussian_spinor(cfg1.p.dims, 8).numpy()
    lu, piv = scipy.linalg.lu_factor(D)
    x_lu = scipy.linalg.lu_solve((lu, piv), b.reshape(-1))
    # LAPACK's 1-norm condition estimate from the LU factors
    rcond, info = scipy.linalg.lapack.zgecon(lu, np.linalg.norm(D, 1), norm="1")
    cond = 1.0 / rcond
    assert info == 0 and 3 < cond < 100
    for op, rhs, mat in ((O.OP_D, b, D), (O.OP_A, None, A), (O.OP_AMSAP, None, A)):
        if rhs is None:  # A x = C_inv b has the same solution
            rhs = (cfg1.Cinv.reshape(-1, 12, 12) @ b.reshape(-1, 12, 1)).reshape(b.shape)
        r = cfg1.solve(rhs, op=op, tol=1e-12, maxiter=1000)
        assert r.status == 0
        err = np.linalg.norm(r.x.reshape(-1) - x_lu) / np.linalg.norm(x_lu)
        assert err < cond * 1e-11, (op, err)
        res = np.linalg.norm(b.reshape(-1) - D @ r.x.reshape(-1)) / np.linalg.norm(b)
        assert res < 1e-10


def test_bicgstab_exit_and_iteration_counts(cfg1):
    """Strict '<' at both exit points; SAP preconditioning cuts the count."""
    b = synth.gaussian_spinor(cfg1.p.dims, 9).numpy()
    plain = cfg1.solve(b, op=O.OP_D, tol=1e-10)
    pre = cfg1.solve((cfg1.Cinv.reshape(-1, 12, 12) @ b.reshape(-1, 12, 1)).reshape(b.shape), op=O.OP_AMSAP,
                     tol=1e-10)
    assert plain.status == 0 and pre.status == 0
    assert plain.relres < 1e-10 and pre.relres < 1e-10
    assert pre.iters * 4 < plain.iters
    one = cfg1.solve(b, op=O.OP_D, tol=1e-10, maxiter=1)
    assert one.status == 1 and one.iters == 1
    zero = cfg1.solve(np.zeros_like(b), op=O.OP_D)
    assert zero.status == 0 and np.all(zero.x == 0)


def test_defect_correction_reaches_tolerance(cfg1, dense_cfg1):
    D, _ = dense_cfg1
    b = synth.gaussian_spinor(cfg1.p.dims, 10).numpy()
    r = cfg1.dci(b, tol=1e-10, inner_tol=1e-6, round_sp=True)
    assert r.status == 0 and 2 <= r.outer <= 4
    res = np.linalg.norm(b.reshape(-1) - D @ r.x.reshape(-1)) / np.linalg.norm(b)
    assert res < 1e-10
    x_lu = np.linalg.solve(D, b.reshape(-1))
    assert np.linalg.norm(r.x.reshape(-1) - x_lu) / np.linalg.norm(x_lu) < 1e-9
