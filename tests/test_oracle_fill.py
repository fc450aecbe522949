"""Pins of the oracle's outer-product fill (Sec. 7, eq. Sfill) and of its contraction.

  full dilution  with one unit source per (x, spin, colour) on the source timeslice, N S is
                 the dense inverse's block D^-1(t, z; t_src, x) for every t (LAPACK LU), and
                 N^2 C(t) its squared Frobenius norm;
  dagger         one source: the dagger block (z, x) equals eta(x) X(z)^dag, built by hand;
  contraction    sum_{z,x} tr[S1 S2^dag] equals the Gram-matrix form
                 (1/N^2) sum_ij <eta1_i, eta2_j>_{t_src} <X2_j, X1_i>_t, written as loops.
"""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs
from tests.test_oracle_pins import dense_operator


@pytest.mark.parametrize("t_src", [0, 3])
def test_fill_full_dilution_is_the_inverse(orc, t_src):
    dims, tbc, kappa = (2, 2, 2, 4), -1, 0.125
    X_, Y, Z, T = dims
    V3 = X_ * Y * Z
    U = inputs.gauge_field(dims, 0.4, seed=71)
    A = orc.clover(U, kappa, 1.3)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    Dinv = np.linalg.inv(D)
    n = 12 * V3
    eta = np.zeros((n, T, Z, Y, X_, 4, 3), np.complex128)
    for k in range(n):
        eta[k, t_src].reshape(-1)[k] = 1.0
    X = (Dinv @ eta.reshape(n, -1).T).T.reshape(eta.shape)
    C = orc.contract_fill(eta, X, eta, X, t_src)
    for t in range(T):
        S = orc.fill_propagator(eta, X, t_src, t)
        block = Dinv[t * n:(t + 1) * n, t_src * n:(t_src + 1) * n]
        assert np.max(np.abs(n * S - block)) < 1e-13
        assert abs(n * n * C[t] - np.sum(np.abs(block) ** 2)) < 1e-12 * np.sum(np.abs(block) ** 2)


def test_fill_dagger_blocks_by_hand(orc):
    dims = (2, 2, 2, 2)
    rng = np.random.default_rng(3)
    shape = (1, 2, 2, 2, 2, 4, 3)
    eta = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    X = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    Sd = orc.fill_propagator(eta, X, 1, 0, dagger=True)
    S = orc.fill_propagator(eta, X, 1, 0)
    Xz = X[0, 0].reshape(8, 12)
    ex = eta[0, 1].reshape(8, 12)
    for z in range(8):
        for x in range(8):
            assert np.allclose(Sd[12 * z:12 * z + 12, 12 * x:12 * x + 12], np.outer(ex[x], np.conj(Xz[z])), atol=1e-15)
            assert np.allclose(S[12 * z:12 * z + 12, 12 * x:12 * x + 12], np.outer(Xz[z], np.conj(ex[x])), atol=1e-15)
    assert np.allclose(orc.fill_propagator(eta, X, 1, 0, dagger=True).reshape(8, 12, 8, 12).transpose(0, 3, 2, 1).conj(),
                       S.reshape(8, 12, 8, 12), atol=0)


def test_fill_contraction_equals_gram_form(orc):
    rng = np.random.default_rng(4)
    N, shape = 5, (5, 4, 2, 2, 2, 4, 3)
    f = [rng.normal(size=shape) + 1j * rng.normal(size=shape) for _ in range(4)]
    eta1, X1, eta2, X2 = f
    t_src = 2
    C = orc.contract_fill(eta1, X1, eta2, X2, t_src)
    for t in range(4):
        ref = 0j
        for i in range(N):
            for j in range(N):
                E = np.vdot(eta1[i, t_src], eta2[j, t_src])
                F = np.vdot(X2[j, t], X1[i, t])
                ref += E * F
        ref /= N * N
        assert abs(C[t] - ref) < 1e-12 * abs(ref), t
