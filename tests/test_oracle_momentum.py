"""Pins of the oracle's dilution and momentum-projected stochastic operators.

  zero momentum  stochastic_operators_mom / pion_mom at p = 0 equal the C oracle's
                 stochastic operators and unbiased pion (an independent implementation);
  full dilution  with unit sources the raw all-pairs sum at momentum p equals
                 sum_t0 tr[Phi_t1(p) B(t1, t0) Phi_t0(-p) B(t0, t1)] from the dense inverse
                 (B = gamma_5 D^-1 blocks, Phi diagonal phases), for complex phases (X = 4);
  dilution       the pieces of a noise vector partition it (disjoint supports, sum = eta);
  estimator      the diluted momentum-projected estimator equals the double sum over pairs of
                 distinct noise vectors of tr[Phi g5 S_j Phi^* g5 S_i] with each S_i = sum_d
                 X_i^(d) eta_i^(d)^dag assembled as a dense matrix;
  statistics     the time-spin-colour diluted unbiased estimator agrees with the exact
                 correlator within 4 jackknife standard deviations (over noise vectors), with
                 a smaller error than the undiluted estimator from the same noise vectors.
"""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs
from tests import closed_forms as cf
from tests.test_oracle_contraction import exact_pieces, unit_sources
from tests.test_oracle_pins import dense_operator


def test_zero_momentum_matches_c_oracle(orc):
    dims = (2, 2, 2, 4)
    rng = np.random.default_rng(5)
    shape = (6, 4, 2, 2, 2, 4, 3)
    eta = inputs.z2_noise(dims, 6, seed=8)
    X = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    O = orc.stochastic_operators(eta, X)
    assert np.max(np.abs(orc.stochastic_operators_mom(eta, X, (0, 0, 0)) - O)) < 1e-13 * np.max(np.abs(O))
    C = orc.pion_from_O(O, orc.MODE_UNBIASED)
    assert np.max(np.abs(orc.pion_mom(eta, X, (0, 0, 0)) - C)) < 1e-13 * np.max(np.abs(C))


@pytest.fixture(scope="module")
def field4(orc):
    dims, kappa, tbc = (4, 2, 2, 4), 0.12, -1
    U = inputs.gauge_field(dims, 0.5, seed=62)
    A = orc.clover(U, kappa, 1.3)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    return dict(dims=dims, U=U, A=A, kappa=kappa, tbc=tbc, S=np.linalg.inv(D))


@pytest.mark.parametrize("p", [(1, 0, 0), (1, 1, 0), (3, 0, 1)])
def test_full_dilution_momentum_exact(orc, field4, p):
    f = field4
    dims = f["dims"]
    X_, Y, Z, T = dims
    V3 = X_ * Y * Z
    n = 12 * V3
    eta = unit_sources(dims)
    Xs = (f["S"] @ eta.reshape(eta.shape[0], -1).T).T.reshape(eta.shape)
    raw = orc.pion_mom(eta, Xs, p, mode=orc.MODE_RAW_ALL)
    g5 = np.tile(np.repeat(np.diag(cf.GAMMA5).real, 3), V3 * T)
    GS = g5[:, None] * f["S"]
    # exp(-i p.y) per row of a timeslice (rows: z, y, x, then 12 spin-colour components)
    ph = np.array([np.exp(-2j * np.pi * (p[0] * x / X_ + p[1] * y / Y + p[2] * z / Z))
                   for z in range(Z) for y in range(Y) for x in range(X_) for _ in range(12)])

    def B(t1, t2):
        return GS[t1 * n:(t1 + 1) * n, t2 * n:(t2 + 1) * n]

    want = np.array([sum(np.trace((ph[:, None] * B((t0 + dt) % T, t0)) @ (np.conj(ph)[:, None] * B(t0, (t0 + dt) % T)))
                         for t0 in range(T)) for dt in range(T)])
    assert np.max(np.abs(raw - want)) < 1e-11 * np.max(np.abs(want))
    # C(-p) = conj C(p) here, so a sign error in the phase shows only through Im C, which must
    # be far above the tolerance for the comparison to pin the sign
    assert np.max(np.abs(want.imag)) > 1e-7 * np.max(np.abs(want))


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_dilution_partitions_the_noise(orc, scheme):
    dims = (2, 2, 2, 4)
    eta = inputs.z2_noise(dims, 3, seed=9)
    out = orc.dilute(eta, scheme)
    D = orc.dilution_size(scheme, 4)
    assert out.shape[0] == 3 * D
    pieces = out.reshape((3, D) + eta.shape[1:])
    assert np.array_equal(pieces.sum(axis=1), eta)
    mask = np.abs(pieces) > 0
    assert np.all(mask.sum(axis=1) == 1)  # every component in exactly one piece


def jackknife(est, nv):
    full = est(list(range(nv)))
    loo = np.array([est([k for k in range(nv) if k != j]) for j in range(nv)])
    err = np.sqrt((nv - 1) / nv * np.sum(np.abs(loo - loo.mean(axis=0)) ** 2, axis=0))
    return full, err


def test_diluted_estimator_unbiased_and_less_noisy(orc):
    dims, kappa, tbc = (2, 2, 2, 4), 0.12, -1
    U = inputs.gauge_field(dims, 0.5, seed=61)
    A = orc.clover(U, kappa, 1.3)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    S = np.linalg.inv(D)
    pion, _, _ = exact_pieces(S, dims)
    exact = pion / (dims[3])  # the estimators average over t0
    nv = 8
    eta = inputs.z2_noise(dims, nv, seed=21)
    solve = lambda src: (S @ src.reshape(src.shape[0], -1).T).T.reshape(src.shape)
    G = orc.dilution_size(orc.DILUTE_TSC, 4)
    eta_d = orc.dilute(eta, orc.DILUTE_TSC)
    X_d, X_u = solve(eta_d), solve(eta)

    def est_dil(keep):
        idx = np.concatenate([np.arange(k * G, (k + 1) * G) for k in keep])
        return orc.pion_mom(eta_d[idx], X_d[idx], (0, 0, 0), group=G)

    def est_und(keep):
        return orc.pion_mom(eta[keep], X_u[keep], (0, 0, 0))

    cd, ed = jackknife(est_dil, nv)
    cu, eu = jackknife(est_und, nv)
    for dt in range(1, 4):
        assert abs(cd[dt].real - exact[dt].real) < 4 * ed[dt] + 1e-12, (dt, cd[dt], exact[dt], ed[dt])
        assert ed[dt] < eu[dt], (dt, ed[dt], eu[dt])


@pytest.mark.parametrize("scheme,p", [(3, (0, 0, 0)), (1, (1, 0, 1)), (2, (0, 1, 0))])
def test_diluted_estimator_equals_dense_double_sum(orc, scheme, p):
    dims = (2, 2, 2, 4)
    X_, Y, Z, T = dims
    V3 = X_ * Y * Z
    n = 12 * V3
    rng = np.random.default_rng(31)
    nv = 3
    eta = inputs.z2_noise(dims, nv, seed=33)
    G = orc.dilution_size(scheme, T)
    eta_d = orc.dilute(eta, scheme)
    shape = eta_d.shape
    X_d = rng.normal(size=shape) + 1j * rng.normal(size=shape)  # any fields: an algebraic identity
    C = orc.pion_mom(eta_d, X_d, p, group=G)
    Si = [sum(np.outer(X_d[i * G + d].ravel(), np.conj(eta_d[i * G + d].ravel())) for d in range(G))
          for i in range(nv)]
    g5 = np.tile(np.repeat([1, 1, -1, -1], 3), V3 * T)
    ph = np.array([np.exp(-2j * np.pi * (p[0] * x / X_ + p[1] * y / Y + p[2] * z / Z))
                   for z in range(Z) for y in range(Y) for x in range(X_) for _ in range(12)])
    want = np.zeros(T, complex)
    for dt in range(T):
        for t0 in range(T):
            t1 = (t0 + dt) % T
            r1, r0 = slice(t1 * n, (t1 + 1) * n), slice(t0 * n, (t0 + 1) * n)
            for i in range(nv):
                for j in range(nv):
                    if i == j:
                        continue
                    # sum_{x in t1, y in t0} e^{-ip(x - y)} tr[g5 S_j(y, x) g5 S_i(x, y)]
                    A = (g5[r0, None] * Si[j][r0, r1]) * ph[None, :]
                    B = (g5[r1, None] * Si[i][r1, r0]) * np.conj(ph)[None, :]
                    want[dt] += np.trace(A @ B)
    want /= T * nv * (nv - 1)
    assert np.max(np.abs(C - want)) < 1e-12 * np.max(np.abs(want))
