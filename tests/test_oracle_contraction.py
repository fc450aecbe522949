"""Pins of the oracle's stochastic-operator contraction (Sec. 7, eq. stoop) and of the
zero-momentum pi-pi diagram pieces (Sec. 5 / Sec. 8, diagrams 0-3).

* Full dilution: with the 12V unit vectors as "sources" the estimator is exact, so the raw
  sums equal the exact correlators, computed here from a dense LAPACK inverse of D by a
  different route (spin-colour matrix traces of S = D^{-1}), and for unit links from the
  momentum-space closed form.
* Invariants: C(dt) = C(T - dt) exactly (relabel a <-> b and shift t0).
* Statistics: the unbiased estimators (noise sets a != b, independent groups) agree with the
  exact values within 4 jackknife standard deviations.
"""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs
from tests import closed_forms as cf
from tests.test_oracle_pins import dense_operator


def unit_sources(dims):
    X, Y, Z, T = dims
    n = 12 * X * Y * Z * T
    return np.eye(n, dtype=complex).reshape(n, T, Z, Y, X, 4, 3)


def exact_pieces(S, dims):
    """Exact zero-momentum correlators from the dense propagator S = D^{-1} (12V x 12V).

    Gt = P_t G5 S restricted to rows at timeslice t; every quantity is a trace of products
    of blocks  B(t1, t2) = [G5 S]_{rows in t1, cols in t2}.
    """
    X, Y, Z, T = dims
    V3 = X * Y * Z
    n = 12 * V3
    g5 = np.tile(np.repeat(np.diag(cf.GAMMA5).real, 3), X * Y * Z * T)
    GS = g5[:, None] * S

    def B(t1, t2):
        return GS[t1 * n:(t1 + 1) * n, t2 * n:(t2 + 1) * n]

    def L(t1, t2):  # sum_{x in t1, y in t2} tr[g5 S(x;y) g5 S(y;x)]
        return np.trace(B(t1, t2) @ B(t2, t1))

    pion = np.array([sum(L((t0 + dt) % T, t0) for t0 in range(T)) for dt in range(T)])
    d0 = np.array([sum(L((t0 + dt) % T, t0) ** 2 for t0 in range(T)) for dt in range(T)])
    vac = np.array([L(t, t) for t in range(T)])
    d1 = np.array([sum(vac[(t0 + dt) % T] * vac[t0] for t0 in range(T)) for dt in range(T)])
    d2 = np.array([sum(np.trace(B(t0, t0) @ B(t0, (t0 + dt) % T) @ B((t0 + dt) % T, (t0 + dt) % T)
                                @ B((t0 + dt) % T, t0)) for t0 in range(T)) for dt in range(T)])
    d3 = np.array([sum(np.trace(B((t0 + dt) % T, (t0 + dt) % T) @ B((t0 + dt) % T, t0) @ B(t0, t0)
                                @ B(t0, (t0 + dt) % T)) for t0 in range(T)) for dt in range(T)])
    return pion, np.stack([d0, d1, d2, d3]), vac


@pytest.fixture(scope="module")
def tiny_field(orc):
    dims = (2, 2, 2, 4)
    U = inputs.gauge_field(dims, 0.5, seed=61)
    kappa, csw, tbc = 0.12, 1.3, -1
    A = orc.clover(U, kappa, csw)
    D = dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims)
    S = np.linalg.inv(D)
    return dict(dims=dims, U=U, A=A, kappa=kappa, tbc=tbc, S=S)


def test_unit_sources_free_field_closed_form(orc):
    dims = (2, 2, 2, 4)
    kappa, tbc = 0.12, -1
    U = inputs.unit_gauge(dims)
    A = orc.clover(U, kappa, 1.0)
    eta = unit_sources(dims)
    X, info = orc.solve(U, A, kappa, eta, tbc, tol=1e-13)
    assert np.all(info[:, 2] == 1)
    O = orc.stochastic_operators(eta, X)
    raw = orc.pion_from_O(O, orc.MODE_RAW_ALL)
    want = cf.free_pion_raw(dims, kappa, tbc)
    assert np.max(np.abs(raw - want)) < 1e-11 * np.max(np.abs(want))
    assert np.max(np.abs(want.imag)) < 1e-12 * np.max(np.abs(want))
    # a != b raw sum differs only at dt = 0 (the a = b terms need both points on one slice)
    raw_ne = orc.pion_from_O(O, orc.MODE_RAW_UNBIASED)
    assert np.max(np.abs(raw_ne[1:] - raw[1:])) < 1e-11 * np.max(np.abs(want))


def test_unit_sources_exact_pion_and_pipi(orc, tiny_field):
    f = tiny_field
    dims = f["dims"]
    eta = unit_sources(dims)
    X, info = orc.solve(f["U"], f["A"], f["kappa"], eta, f["tbc"], tol=1e-13)
    assert np.all(info[:, 2] == 1)
    O = orc.stochastic_operators(eta, X)
    pion, diag, vac = exact_pieces(f["S"], dims)
    raw = orc.pion_from_O(O, orc.MODE_RAW_ALL)
    scale = np.max(np.abs(pion))
    assert np.max(np.abs(raw - pion)) < 1e-11 * scale
    # four identical full-dilution groups give the exact diagram sums (raw normalisation)
    n = O.shape[1]
    O4 = np.tile(O, (1, 4, 4))
    assert O4.shape[1] == 4 * n
    d, v = orc.pipi_from_O(O4, normalise=False)
    for k in range(4):
        s = np.max(np.abs(diag[k]))
        assert np.max(np.abs(d[k] - diag[k])) < 1e-10 * s, k
    assert np.max(np.abs(v - vac)) < 1e-11 * np.max(np.abs(vac))
    # diagram 3 is the complex conjugate of diagram 2 for the exact propagator
    assert np.max(np.abs(diag[3] - np.conj(diag[2]))) < 1e-11 * np.max(np.abs(diag[2]))


def test_correlator_reflection_symmetry(orc, tiny_field):
    f = tiny_field
    dims = f["dims"]
    T = dims[3]
    eta = inputs.z2_noise(dims, 6, seed=71)
    X, _ = orc.solve(f["U"], f["A"], f["kappa"], eta, f["tbc"], tol=1e-12)
    for mode in (orc.MODE_UNBIASED, orc.MODE_ALL_PAIRS):
        C, _ = orc.contract_pion(eta, X, mode)
        for dt in range(1, T):
            assert abs(C[dt] - C[T - dt]) < 1e-13 * abs(C[0])


def _jackknife(values_fn, nblocks):
    full = values_fn(None)
    jk = np.array([values_fn(k) for k in range(nblocks)])
    err = np.sqrt((nblocks - 1) / nblocks * np.sum(np.abs(jk - jk.mean(axis=0)) ** 2, axis=0))
    return full, err


@pytest.mark.slow
def test_estimators_unbiased(orc, tiny_field):
    """Sec. 7: stochastic and exact all-to-all agree; independent noise per propagator."""
    f = tiny_field
    dims = f["dims"]
    T = dims[3]
    N = 64
    eta = inputs.z2_noise(dims, N, seed=81)
    X, info = orc.solve(f["U"], f["A"], f["kappa"], eta, f["tbc"], tol=1e-12)
    assert np.all(info[:, 2] == 1)
    O = orc.stochastic_operators(eta, X)
    pion, diag, vac = exact_pieces(f["S"], dims)

    def pion_est(drop):
        keep = [a for a in range(N) if a != drop]
        return orc.pion_from_O(O[:, keep][:, :, keep], orc.MODE_UNBIASED) * T

    est, err = _jackknife(pion_est, N)
    # C = R / (T N (N-1)); the raw exact sum over t0 is pion, so compare T*C with pion
    assert np.all(np.abs(est - pion) < 4 * err + 1e-12), (est, pion, err)
    assert err[0] / abs(pion[0]) < 0.05 and err[1] / abs(pion[1]) < 0.5  # the test has power

    n = N // 4

    def pipi_est(drop):
        if drop is None:
            sub = O
        else:
            keep = [g * n + i for g in range(4) for i in range(n) if i != drop]
            sub = O[:, keep][:, :, keep]
        d, _ = orc.pipi_from_O(sub, normalise=True)
        return d * T

    dest, derr = _jackknife(pipi_est, n)
    for k in (0, 2, 3):
        assert np.all(np.abs(dest[k] - diag[k]) < 4 * derr[k] + 1e-12 * np.max(np.abs(diag[k]))), k
