"""Pins of the FP64 CPU oracle against results fixed by the mathematics, independent of
the oracle's own code: closed forms, textbook routines, invariants and a hand-computed
special case.  A plausible slip in the oracle (hopping sign, kappa normalisation,
boundary sign, gamma basis, clover orientation or sign, even-odd algebra, contraction
bookkeeping) fails at least one of these.
"""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs
from tests import closed_forms as cf


def rand_spinor(dims, seed, n=None):
    rng = np.random.default_rng(seed)
    X, Y, Z, T = dims
    shape = ((n,) if n else ()) + (T, Z, Y, X, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def inner(a, b):
    return np.vdot(a.ravel(), b.ravel())


def g5(psi):
    return np.einsum("ij,...jc->...ic", cf.GAMMA5, psi)


# ---------------------------------------------------------------------------------------
# gamma basis
# ---------------------------------------------------------------------------------------
def test_gamma_basis_matches_hand_written(orc):
    g = cf.gammas()
    for mu in range(4):
        assert np.allclose(orc.gamma(mu), g[mu], atol=0)
    assert np.allclose(orc.gamma(4), cf.GAMMA5, atol=0)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            acomm = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(acomm, 2 * np.eye(4) * (mu == nu))


# ---------------------------------------------------------------------------------------
# P1: free field closed form (hopping sign, kappa normalisation, boundary sign)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("dims,kappa,tbc", [((4, 4, 4, 8), 0.125, -1), ((4, 2, 6, 4), 0.12, 1),
                                            ((2, 4, 2, 6), 0.13, -1)])
def test_free_field_operator_closed_form(orc, dims, kappa, tbc):
    U = inputs.unit_gauge(dims)
    A = orc.clover(U, kappa, 1.7)  # F = 0 at unit links: c_sw must drop out
    assert np.allclose(A, np.broadcast_to(np.eye(12), A.shape), atol=1e-15)
    psi = rand_spinor(dims, 11)
    got = orc.apply_D(U, A, kappa, psi, tbc)
    want = cf.free_apply(dims, kappa, tbc, psi)
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("dims,kappa,tbc", [((4, 4, 4, 8), 0.125, -1), ((4, 4, 4, 4), 0.12, 1)])
def test_free_field_solve_closed_form(orc, dims, kappa, tbc):
    U = inputs.unit_gauge(dims)
    A = orc.clover(U, kappa, 1.0)
    eta = inputs.z2_noise(dims, 2, seed=7)
    X, info = orc.solve(U, A, kappa, eta, tbc, tol=1e-13)
    assert np.all(info[:, 2] == 1)
    for i in range(2):
        want = cf.free_solve(dims, kappa, tbc, eta[i])
        assert np.linalg.norm(X[i] - want) / np.linalg.norm(want) < 1e-12


def test_periodic_kappa_one_eighth_is_singular():
    """At kappa = 1/8 with periodic time, D(p = 0) vanishes (why free tests there use antiperiodic t)."""
    D = cf.dirac_p((4, 4, 4, 4), 0.125, 1)
    assert np.abs(np.linalg.det(D[0, 0, 0, 0])) < 1e-14


# ---------------------------------------------------------------------------------------
# P2: gamma5-hermiticity and clover structure
# ---------------------------------------------------------------------------------------
def test_gamma5_hermiticity_full_and_schur(orc):
    dims = (4, 2, 4, 6)
    U = inputs.gauge_field(dims, 0.6, seed=3)
    kappa, csw = 0.13, 1.4
    A = orc.clover(U, kappa, csw)
    Ainv = orc.invert_sites(A)
    for tbc in (1, -1):
        phi, psi = rand_spinor(dims, 1), rand_spinor(dims, 2)
        lhs = inner(phi, orc.apply_D(U, A, kappa, psi, tbc))
        rhs = inner(g5(orc.apply_D(U, A, kappa, g5(phi), tbc)), psi)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
        odd = (orc.parity_mask(dims) == 1)[..., None, None]
        phio, psio = np.where(odd, phi, 0), np.where(odd, psi, 0)
        lhs = inner(phio, orc.schur(U, A, Ainv, kappa, psio, tbc))
        rhs = inner(g5(orc.schur(U, A, Ainv, kappa, g5(phio), tbc)), psio)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_clover_hermitian_chiral_traceless(orc):
    dims = (2, 4, 2, 4)
    U = inputs.gauge_field(dims, 0.8, seed=5)
    A = orc.clover(U, 0.12, 1.3).reshape(-1, 12, 12)
    G5 = np.kron(cf.GAMMA5, np.eye(3))
    assert np.allclose(A, np.conj(np.swapaxes(A, 1, 2)), atol=1e-15)
    assert np.max(np.abs(A @ G5 - G5 @ A)) < 1e-15
    spin_tr = (A - np.eye(12)).reshape(-1, 4, 3, 4, 3)
    assert np.max(np.abs(np.einsum("nscsd->ncd", spin_tr))) < 1e-15
    assert np.max(np.abs(A - np.eye(12))) > 1e-2  # the field is not trivial


def test_field_strength_antihermitian(orc):
    """F = (Q - Q^dag)/8 is anti-Hermitian; its trace is kept (no su(3) projection)."""
    dims = (2, 2, 4, 4)
    U = inputs.gauge_field(dims, 0.5, seed=9)
    F = orc.field_strength(U)
    assert np.allclose(F, -np.conj(np.swapaxes(F, -1, -2)), atol=1e-15)


# ---------------------------------------------------------------------------------------
# P3: clover sign and normalisation, hand-computed single-link configuration
# ---------------------------------------------------------------------------------------
def test_clover_single_link_by_hand(orc):
    dims = (6, 6, 4, 4)
    X, Y, Z, T = dims
    U = inputs.unit_gauge(dims)
    theta = 0.7
    T3 = np.diag([0.5, -0.5, 0.0])
    W = np.diag(np.exp(1j * theta * np.diag(T3)))
    x0 = (2, 2, 1, 1)  # (x, y, z, t)
    U[x0[3], x0[2], x0[1], x0[0], 0] = W  # U_1(x0) in the x direction
    kappa, csw = 0.11, 1.3
    A = orc.clover(U, kappa, csw)
    sinT = np.diag(np.sin(theta * np.diag(T3)))
    # hand derivation: only the (1,2), (1,3), (1,4) planes see the modified link; at
    # x0 + 2hat the single leaf containing it gives F_12 = (W - W^dag)/8 = (i/4) sin(theta T3)
    # and sigma_12 = i gamma_1 gamma_2 = diag(-1, 1, -1, 1) in the chiral basis, so
    # A = 1 + i kappa c_sw sigma_12 (x) (i/4) sin(theta T3) = 1 - (kappa c_sw / 4) sigma_12 (x) sin(theta T3).
    sig12 = np.diag([-1.0, 1.0, -1.0, 1.0])

    def at(x, y, z, t):
        return A[t % T, z % Z, y % Y, x % X]

    want_plus = np.eye(12) - (kappa * csw / 4) * np.kron(sig12, sinT)
    want_minus = np.eye(12) + (kappa * csw / 4) * np.kron(sig12, sinT)
    x, y, z, t = x0
    assert np.max(np.abs(at(x, y + 1, z, t) - want_plus)) < 1e-15
    assert np.max(np.abs(at(x + 1, y + 1, z, t) - want_plus)) < 1e-15
    assert np.max(np.abs(at(x, y - 1, z, t) - want_minus)) < 1e-15
    assert np.max(np.abs(at(x + 1, y - 1, z, t) - want_minus)) < 1e-15
    # the two sites touching the link in every plane: leaves with W and W^dag cancel
    assert np.max(np.abs(at(x, y, z, t) - np.eye(12))) < 1e-15
    assert np.max(np.abs(at(x + 1, y, z, t) - np.eye(12))) < 1e-15
    # and a far-away site is untouched
    assert np.max(np.abs(at(x + 3, y + 3, z, t + 2) - np.eye(12))) < 1e-15


# ---------------------------------------------------------------------------------------
# P4: gauge covariance (link orientation, leaf paths)
# ---------------------------------------------------------------------------------------
def test_gauge_covariance(orc):
    dims = (4, 2, 2, 4)
    X, Y, Z, T = dims
    U = inputs.gauge_field(dims, 0.5, seed=21)
    g = inputs.random_su3(X * Y * Z * T, seed=22).reshape(T, Z, Y, X, 3, 3)
    Ug = np.empty_like(U)
    for mu, ax in enumerate((3, 2, 1, 0)):
        gfwd = np.roll(g, -1, axis=ax)  # g(x + mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gfwd, -1, -2))
    kappa, csw, tbc = 0.12, 1.5, -1
    # F -> g F g^dag
    F, Fg = orc.field_strength(U), orc.field_strength(Ug)
    gd = np.conj(np.swapaxes(g, -1, -2))
    assert np.max(np.abs(Fg - g[..., None, :, :] @ F @ gd[..., None, :, :])) < 1e-14
    A, Ag = orc.clover(U, kappa, csw), orc.clover(Ug, kappa, csw)
    eta = inputs.z2_noise(dims, 4, seed=23)
    geta = np.einsum("tzyxab,ntzyxsb->ntzyxsa", g, eta)
    # D[U^g] (g psi) = g D[U] psi
    lhs = orc.apply_D(Ug, Ag, kappa, geta[0], tbc)
    rhs = np.einsum("tzyxab,tzyxsb->tzyxsa", g, orc.apply_D(U, A, kappa, eta[0], tbc))
    assert np.max(np.abs(lhs - rhs)) < 1e-13
    X0, _ = orc.solve(U, A, kappa, eta, tbc, tol=1e-13)
    Xg, _ = orc.solve(Ug, Ag, kappa, geta, tbc, tol=1e-13)
    gX0 = np.einsum("tzyxab,ntzyxsb->ntzyxsa", g, X0)
    assert np.linalg.norm(Xg - gX0) / np.linalg.norm(gX0) < 1e-11
    C0, O0 = orc.contract_pion(eta, X0)
    Cg, Og = orc.contract_pion(geta, Xg)
    assert np.max(np.abs(Og - O0)) < 1e-10 * np.max(np.abs(O0))
    assert np.max(np.abs(Cg - C0)) < 1e-10 * np.max(np.abs(C0))


# ---------------------------------------------------------------------------------------
# P5: solver and even-odd algebra against dense LU (LAPACK)
# ---------------------------------------------------------------------------------------
def dense_operator(apply, dims):
    X, Y, Z, T = dims
    n = 12 * X * Y * Z * T
    M = np.empty((n, n), complex)
    e = np.zeros(n, complex)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = apply(e.reshape(T, Z, Y, X, 4, 3)).ravel()
    return M


@pytest.mark.parametrize("dims,tbc", [((2, 2, 2, 2), -1), ((2, 2, 2, 4), 1)])
def test_solve_matches_dense_lu(orc, dims, tbc):
    U = inputs.gauge_field(dims, 0.4, seed=31)
    kappa, csw = 0.125, 1.2
    A = orc.clover(U, kappa, csw)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    eta = inputs.z2_noise(dims, 3, seed=32)
    X, info = orc.solve(U, A, kappa, eta, tbc, tol=1e-13)
    Xlu = np.linalg.solve(D, eta.reshape(3, -1).T).T.reshape(eta.shape)
    assert np.all(info[:, 3] <= 1e-13)
    assert np.linalg.norm(X - Xlu) / np.linalg.norm(Xlu) < 1e-12


@pytest.mark.parametrize("dims,tbc", [((2, 2, 2, 2), -1), ((2, 2, 2, 4), 1)])
def test_cgnr_matches_dense_lu(orc, dims, tbc):
    U = inputs.gauge_field(dims, 0.4, seed=33)
    kappa, csw = 0.125, 1.2
    A = orc.clover(U, kappa, csw)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    eta = inputs.z2_noise(dims, 3, seed=34)
    X, info = orc.solve_cgnr(U, A, kappa, eta, tbc, tol=1e-13)
    Xlu = np.linalg.solve(D, eta.reshape(3, -1).T).T.reshape(eta.shape)
    assert np.all(info[:, 3] <= 1e-13) and np.all(info[:, 2] == 1)
    assert np.linalg.norm(X - Xlu) / np.linalg.norm(Xlu) < 1e-12


def test_cgnr_iterate_minimises_residual_over_krylov_space(orc):
    """After k steps from zero, CG on the normal equations gives the x of the Krylov space
    K_k(D^dag D, D^dag b) with the smallest ||b - D x|| (its defining property): compared with
    a dense least-squares fit over an orthonormal basis of that space, k = 1..6; the residual
    history is non-increasing."""
    dims, tbc = (2, 2, 2, 2), -1
    U = inputs.gauge_field(dims, 0.5, seed=35)
    kappa = 0.13
    A = orc.clover(U, kappa, 1.5)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    b = inputs.z2_noise(dims, 1, seed=36)[0]
    bf = b.ravel()
    N = D.conj().T @ D
    Q = np.zeros((bf.size, 0), complex)
    v = D.conj().T @ bf
    for k in range(1, 7):
        for _ in range(2):  # Gram-Schmidt, twice
            v = v - Q @ (Q.conj().T @ v)
        Q = np.hstack([Q, (v / np.linalg.norm(v))[:, None]])
        y, *_ = np.linalg.lstsq(D @ Q, bf, rcond=None)
        xk = Q @ y
        x, hist = orc.cgnr_fixed(U, A, kappa, b, tbc, k)
        assert np.linalg.norm(x.ravel() - xk) / np.linalg.norm(xk) < 1e-10, k
        assert abs(hist[-1] - np.linalg.norm(bf - D @ xk) / np.linalg.norm(bf)) < 1e-12
        assert np.all(np.diff(hist) <= 1e-15)
        v = N @ Q[:, -1]


def test_cgnr_and_bicgstab_agree(orc):
    dims, tbc = (4, 4, 4, 8), -1
    U = inputs.gauge_field(dims, 0.35, seed=37)
    kappa = 0.125
    A = orc.clover(U, kappa, 1.5)
    eta = inputs.z2_noise(dims, 2, seed=38)
    Xb, ib = orc.solve(U, A, kappa, eta, tbc, tol=1e-12)
    Xc, ic = orc.solve_cgnr(U, A, kappa, eta, tbc, tol=1e-12)
    assert np.all(ic[:, 3] <= 1e-12) and np.all(ib[:, 3] <= 1e-12)
    assert np.linalg.norm(Xc - Xb) / np.linalg.norm(Xb) < 1e-10
    assert np.all(ic[:, 0] > ib[:, 0])  # the squared condition number costs iterations


def test_schur_identity_against_dense_lu(orc):
    """x_o from the dense Schur system, x_e from reconstruction, equal the full LU solution;
    and the full residual of that assembled solution vanishes on both parities."""
    dims = (2, 2, 2, 4)
    tbc = -1
    U = inputs.gauge_field(dims, 0.5, seed=41)
    kappa, csw = 0.13, 1.5
    A = orc.clover(U, kappa, csw)
    Ainv = orc.invert_sites(A)
    eta = inputs.z2_noise(dims, 1, seed=42)[0]
    odd = (orc.parity_mask(dims) == 1)[..., None, None]
    oddflat = np.broadcast_to(odd, eta.shape).ravel()
    M = dense_operator(lambda v: orc.schur(U, A, Ainv, kappa, v, tbc), dims)
    Moo = M[np.ix_(oddflat, oddflat)]
    b = orc.schur_rhs(U, A, Ainv, kappa, eta, tbc).ravel()[oddflat]
    xo = np.zeros(eta.size, complex)
    xo[oddflat] = np.linalg.solve(Moo, b)
    X = orc.reconstruct_even(U, Ainv, kappa, eta, xo.reshape(eta.shape), tbc)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    Xlu = np.linalg.solve(D, eta.ravel())
    assert np.linalg.norm(X.ravel() - Xlu) / np.linalg.norm(Xlu) < 1e-13
    assert np.linalg.norm(D @ X.ravel() - eta.ravel()) < 1e-13 * np.linalg.norm(eta)


def test_site_inverse(orc):
    dims = (2, 2, 2, 2)
    U = inputs.gauge_field(dims, 0.9, seed=51)
    A = orc.clover(U, 0.13, 2.0).reshape(-1, 12, 12)
    Ainv = orc.invert_sites(A)
    assert np.max(np.abs(Ainv @ A - np.eye(12))) < 1e-14
    assert np.max(np.abs(Ainv - np.linalg.inv(A))) < 1e-14


def test_solvers_match_dense_lu_on_the_small_workload(orc):
    """The small workload's lattice (4^3x8, N = 6144): BiCGStab and CGNR solutions of the
    workload's field and sources against a dense LAPACK solve of the assembled operator."""
    w = inputs.WORKLOADS["tiny_4c8"]
    dims, tbc, kappa, csw = w["dims"], w["tbc"], w["kappa"], w["csw"]
    U = inputs.gauge_field(dims, w["eps"], w["gauge_seed"])
    A = orc.clover(U, kappa, csw)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    eta = inputs.z2_noise(dims, w["nsrc"], w["noise_seed"])
    n = eta.shape[0]
    Xlu = np.linalg.solve(D, eta.reshape(n, -1).T).T.reshape(eta.shape)
    del D
    Xb, ib = orc.solve(U, A, kappa, eta, tbc, tol=1e-13)
    Xc, ic = orc.solve_cgnr(U, A, kappa, eta, tbc, tol=1e-13)
    assert np.all(ib[:, 2] == 1) and np.all(ic[:, 2] == 1)
    for i in range(n):
        nrm = np.linalg.norm(Xlu[i])
        assert np.linalg.norm(Xb[i] - Xlu[i]) / nrm < 1e-12, i
        assert np.linalg.norm(Xc[i] - Xlu[i]) / nrm < 1e-12, i


def test_bicgstab_fixed_matches_library_bicgstab(orc):
    """The fixed-iteration BiCGStab (the loop the CPU baseline times) after k = 1..6
    iterations from zero equals scipy's BiCGStab (van der Vorst 1992, shadow vector r0,
    no restarts) on the dense operator of 2^4 after the same number of iterations, and its
    residual history is the true residual ||b - D x_k|| / ||b|| of those iterates."""
    import scipy.sparse.linalg as spla

    dims, tbc = (2, 2, 2, 2), -1
    U = inputs.gauge_field(dims, 0.5, seed=61)
    kappa = 0.13
    A = orc.clover(U, kappa, 1.5)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    b = inputs.z2_noise(dims, 1, seed=62)[0]
    bf = b.ravel()
    for k in range(1, 7):
        xs, info = spla.bicgstab(D, bf, rtol=0.0, atol=0.0, maxiter=k)
        assert info == k  # ran all k iterations (no early exit)
        x, hist = orc.bicgstab_fixed(U, A, kappa, b, tbc, k)
        assert np.linalg.norm(x.ravel() - xs) / np.linalg.norm(xs) < 1e-12, k
        assert abs(hist[-1] - np.linalg.norm(bf - D @ xs) / np.linalg.norm(bf)) < 1e-12, k
