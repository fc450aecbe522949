"""Closed forms used to pin the oracle (free field, momentum space) and hand-written
gamma matrices.  Written from the mathematics, independent of ``oracle/``.

Free field (all links = 1): a plane wave psi(x) = exp(i p.x) u is an eigenvector of the
hopping term, and the Wilson operator in the hopping-parameter form becomes the 4x4
spin matrix
    D(p) = 1 - 2 kappa sum_mu cos p_mu + 2 i kappa sum_mu gamma_mu sin p_mu
(times the colour identity).  Antiperiodic time is handled by the substitution
psi(x) = exp(i pi t / T) phi(x) with phi periodic, which shifts p_4 by pi/T.
"""
import numpy as np

S1 = np.array([[0, 1], [1, 0]], complex)
S2 = np.array([[0, -1j], [1j, 0]], complex)
S3 = np.array([[1, 0], [0, -1]], complex)
Z2 = np.zeros((2, 2), complex)
E2 = np.eye(2)


def gammas():
    """Chiral basis: gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, 1], [1, 0]]."""
    g = [np.block([[Z2, -1j * s], [1j * s, Z2]]) for s in (S1, S2, S3)]
    g.append(np.block([[Z2, E2], [E2, Z2]]))
    return g


GAMMA5 = np.diag([1, 1, -1, -1]).astype(complex)


def momenta(dims, tbc):
    X, Y, Z, T = dims
    px = 2 * np.pi * np.arange(X) / X
    py = 2 * np.pi * np.arange(Y) / Y
    pz = 2 * np.pi * np.arange(Z) / Z
    pt = 2 * np.pi * np.arange(T) / T + (np.pi / T if tbc == -1 else 0.0)
    return px, py, pz, pt


def dirac_p(dims, kappa, tbc):
    """D(p) on the momentum grid, shape (T, Z, Y, X, 4, 4), axes ordered like the lattice."""
    px, py, pz, pt = momenta(dims, tbc)
    P = np.meshgrid(pt, pz, py, px, indexing="ij")  # t, z, y, x
    pmu = [P[3], P[2], P[1], P[0]]  # mu = x, y, z, t
    g = gammas()
    a = 1 - 2 * kappa * sum(np.cos(p) for p in pmu)
    D = a[..., None, None] * np.eye(4)
    for mu in range(4):
        D = D + 2j * kappa * np.sin(pmu[mu])[..., None, None] * g[mu]
    return D


def _twist(dims, tbc, sign):
    X, Y, Z, T = dims
    if tbc != -1:
        return np.ones((T, 1, 1, 1, 1, 1))
    t = np.arange(T)
    return np.exp(sign * 1j * np.pi * t / T).reshape(T, 1, 1, 1, 1, 1)


def free_apply(dims, kappa, tbc, psi):
    """D psi for unit links, via FFT.  psi: (T, Z, Y, X, 4, 3)."""
    D = dirac_p(dims, kappa, tbc)
    phi = psi * _twist(dims, tbc, -1)
    f = np.fft.fftn(phi, axes=(0, 1, 2, 3))
    g = np.einsum("...ij,...jc->...ic", D, f)
    return np.fft.ifftn(g, axes=(0, 1, 2, 3)) * _twist(dims, tbc, +1)


def free_solve(dims, kappa, tbc, eta):
    """D^{-1} eta for unit links, via FFT."""
    D = dirac_p(dims, kappa, tbc)
    Dinv = np.linalg.inv(D)
    phi = eta * _twist(dims, tbc, -1)
    f = np.fft.fftn(phi, axes=(0, 1, 2, 3))
    g = np.einsum("...ij,...jc->...ic", Dinv, f)
    return np.fft.ifftn(g, axes=(0, 1, 2, 3)) * _twist(dims, tbc, +1)


def free_pion_raw(dims, kappa, tbc):
    """sum_t0 sum_{x in t0+dt, y in t0} tr[g5 S(x;y) g5 S(y;x)] for unit links.

    Using gamma5-hermiticity and the spatial Fourier sums this equals
    T * 3 * sum_{p-vec} tr_spin[ St(p, dt) St(p, dt)^dag ],
    St(p, dt) = (1/T) sum_{p4} exp(i p4 dt) D(p-vec, p4)^{-1}.
    """
    X, Y, Z, T = dims
    Dinv = np.linalg.inv(dirac_p(dims, kappa, tbc))  # (T, Z, Y, X, 4, 4)
    _, _, _, pt = momenta(dims, tbc)
    out = np.zeros(T, complex)
    for dt in range(T):
        ph = np.exp(1j * pt * dt).reshape(T, 1, 1, 1, 1, 1)
        St = (ph * Dinv).sum(axis=0) / T  # (Z, Y, X, 4, 4)
        out[dt] = T * 3 * np.sum(St * np.conj(St))
    return out
