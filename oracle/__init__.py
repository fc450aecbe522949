"""Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product library never links or calls it; the two share no code.

The arithmetic lives in ``a2a_oracle.c`` (C99 complex doubles + OpenMP, canonical layout,
plain definitions).  This module compiles it with gcc and wraps it with ctypes, taking
and returning numpy complex128 arrays in the canonical layouts:

    links   (T, Z, Y, X, 4, 3, 3)      spinors (nsrc, T, Z, Y, X, 4, 3)

Parity status of every function: pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (free-field closed form, gamma5-hermiticity, gauge covariance,
a hand-computed clover, dense LU solves, the exact correlator from unit sources, the
free-field correlator closed form, estimator statistics; the outer-product fill by the dense
inverse under full dilution, a hand-built dagger block and the Gram-matrix form of its
contraction; dilution by its partition of the noise, momentum-projected operators by the C
oracle at zero momentum and by dense-inverse traces with phases under full dilution; the
point-source pi-pi diagrams by closed gamma_5 loops of the dense inverse and by their
factorised Gram form).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "a2a_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liba2a_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2 -fopenmp, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        Lg = ctypes.c_long
        sig = {
            "orc_gamma": [I, P],
            "orc_hop": [P, I, P, P, P],
            "orc_field_strength": [P, P, P],
            "orc_clover": [P, P, D, D, P],
            "orc_invert_sites": [Lg, P, P],
            "orc_site_matvec": [Lg, P, P, P],
            "orc_apply_D": [P, I, P, P, D, P, P],
            "orc_schur": [P, I, P, P, P, D, P, P],
            "orc_solve": [P, I, P, P, D, I, P, P, D, I, P],
            "orc_bicgstab_fixed": [P, I, P, P, D, P, P, I, P],
            "orc_solve_cgnr": [P, I, P, P, D, I, P, P, D, I, P],
            "orc_cgnr_fixed": [P, I, P, P, D, P, P, I, P],
            "orc_stochastic_operators": [P, I, P, P, P],
            "orc_pion_from_O": [I, I, P, I, P],
            "orc_contract_pion": [P, I, P, P, I, P, P],
            "orc_pipi_from_O": [I, I, P, I, P, P],
            "orc_contract_pipi": [P, I, P, P, P, P],
            "orc_num_threads": [],
            "orc_set_num_threads": [I],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = I
        _lib = L
    return _lib


def _c(a, dtype=np.complex128):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(links_or_dims):
    if isinstance(links_or_dims, np.ndarray) and links_or_dims.ndim == 7:
        T, Z, Y, X = links_or_dims.shape[:4]
        return np.array([X, Y, Z, T], dtype=np.int32)
    return np.array([int(d) for d in links_or_dims], dtype=np.int32)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on (for single-core timings)."""
    _check(lib().orc_set_num_threads(int(n)), "set_num_threads")


def gamma(mu):
    """gamma_mu (mu = 0..3 for x, y, z, t) or gamma_5 (mu = 4) as a 4x4 complex matrix."""
    out = np.zeros((4, 4), np.complex128)
    _check(lib().orc_gamma(int(mu), _p(out)), "gamma")
    return out


def hop(U, psi, tbc):
    """Full-lattice hopping term H psi (Wilson, r = 1, time boundary sign tbc)."""
    U = _c(U)
    psi = _c(psi)
    out = np.empty_like(psi)
    _check(lib().orc_hop(_p(_dims(U)), int(tbc), _p(U), _p(psi), _p(out)), "hop")
    return out


def field_strength(U):
    """F_munu per site, planes (xy, xz, xt, yz, yt, zt): shape (T,Z,Y,X,6,3,3)."""
    U = _c(U)
    out = np.empty(U.shape[:4] + (6, 3, 3), np.complex128)
    _check(lib().orc_field_strength(_p(_dims(U)), _p(U), _p(out)), "field_strength")
    return out


def clover(U, kappa, csw):
    """Dense 12x12 clover matrix A(x) = 1 + i kappa c_sw sum sigma F per site: (T,Z,Y,X,12,12)."""
    U = _c(U)
    out = np.empty(U.shape[:4] + (12, 12), np.complex128)
    _check(lib().orc_clover(_p(_dims(U)), _p(U), float(kappa), float(csw), _p(out)), "clover")
    return out


def invert_sites(A):
    A = _c(A)
    out = np.empty_like(A)
    n = A.size // 144
    _check(lib().orc_invert_sites(n, _p(A), _p(out)), "invert_sites")
    return out


def site_matvec(A, psi):
    A = _c(A)
    psi = _c(psi)
    out = np.empty_like(psi)
    _check(lib().orc_site_matvec(A.size // 144, _p(A), _p(psi), _p(out)), "site_matvec")
    return out


def apply_D(U, A, kappa, psi, tbc):
    """D psi = A psi - kappa H psi on the full lattice (one spinor field)."""
    U = _c(U)
    A = _c(A)
    psi = _c(psi)
    if psi.shape != U.shape[:4] + (4, 3) or A.shape != U.shape[:4] + (12, 12):
        raise ValueError(f"apply_D: spinor {psi.shape} / clover {A.shape} do not match links {U.shape}")
    out = np.empty_like(psi)
    _check(lib().orc_apply_D(_p(_dims(U)), int(tbc), _p(U), _p(A), float(kappa), _p(psi), _p(out)), "apply_D")
    return out


def schur(U, A, Ainv, kappa, psi, tbc):
    """Odd-site Schur complement A_oo x - kappa^2 H_oe A_ee^{-1} H_eo x (even part zero)."""
    U, A, Ainv, psi = _c(U), _c(A), _c(Ainv), _c(psi)
    out = np.empty_like(psi)
    _check(lib().orc_schur(_p(_dims(U)), int(tbc), _p(U), _p(A), _p(Ainv), float(kappa), _p(psi), _p(out)),
           "schur")
    return out


def solve(U, A, kappa, eta, tbc, tol=1e-13, maxit=100000):
    """X_i = D^{-1} eta_i (BiCGStab on the full system, restarted on the true residual).

    Returns (X, info) with info[i] = (iterations, restarts, converged, true rel. residual).
    """
    U, A, eta = _c(U), _c(A), _c(eta)
    single = eta.ndim == 6
    if single:
        eta = eta[None]
    X = np.empty_like(eta)
    info = np.zeros((eta.shape[0], 4))
    rc = lib().orc_solve(_p(_dims(U)), int(tbc), _p(U), _p(A), float(kappa), eta.shape[0], _p(eta), _p(X),
                         float(tol), int(maxit), _p(info))
    _check(rc, "solve")
    return (X[0] if single else X), info


def bicgstab_fixed(U, A, kappa, eta, tbc, iters):
    """Exactly `iters` BiCGStab iterations from zero on one source; returns (x, residual history)."""
    U, A, eta = _c(U), _c(A), _c(eta)
    X = np.empty_like(eta)
    hist = np.zeros(int(iters))
    _check(lib().orc_bicgstab_fixed(_p(_dims(U)), int(tbc), _p(U), _p(A), float(kappa), _p(eta), _p(X), int(iters),
                                    _p(hist)), "bicgstab_fixed")
    return X, hist


def solve_cgnr(U, A, kappa, eta, tbc, tol=1e-13, maxit=100000):
    """X_i = D^{-1} eta_i by CG on the normal equations D^dag D x = D^dag eta (CGNR, carrying
    the residual of the original system), restarted on the true residual.  Same returns as
    :func:`solve`."""
    U, A, eta = _c(U), _c(A), _c(eta)
    single = eta.ndim == 6
    if single:
        eta = eta[None]
    X = np.empty_like(eta)
    info = np.zeros((eta.shape[0], 4))
    rc = lib().orc_solve_cgnr(_p(_dims(U)), int(tbc), _p(U), _p(A), float(kappa), eta.shape[0], _p(eta), _p(X),
                              float(tol), int(maxit), _p(info))
    _check(rc, "solve_cgnr")
    return (X[0] if single else X), info


def cgnr_fixed(U, A, kappa, eta, tbc, iters):
    """Exactly `iters` CGNR steps from zero on one source; returns (x, residual history)."""
    U, A, eta = _c(U), _c(A), _c(eta)
    X = np.empty_like(eta)
    hist = np.zeros(int(iters))
    _check(lib().orc_cgnr_fixed(_p(_dims(U)), int(tbc), _p(U), _p(A), float(kappa), _p(eta), _p(X), int(iters),
                                _p(hist)), "cgnr_fixed")
    return X, hist


def stochastic_operators(eta, X):
    """O[t, a, b] = sum_{y in t} eta_a(y)^dag gamma_5 X_b(y)."""
    eta, X = _c(eta), _c(X)
    N = eta.shape[0]
    T = eta.shape[1]
    dims = np.array([eta.shape[4], eta.shape[3], eta.shape[2], T], np.int32)
    O = np.empty((T, N, N), np.complex128)
    _check(lib().orc_stochastic_operators(_p(dims), N, _p(eta), _p(X), _p(O)), "stochastic_operators")
    return O


MODE_UNBIASED, MODE_ALL_PAIRS, MODE_RAW_UNBIASED, MODE_RAW_ALL = 0, 1, 2, 3


def pion_from_O(O, mode=MODE_UNBIASED):
    O = _c(O)
    T, N, _ = O.shape
    corr = np.empty(T, np.complex128)
    _check(lib().orc_pion_from_O(T, N, _p(O), int(mode), _p(corr)), "pion_from_O")
    return corr


def contract_pion(eta, X, mode=MODE_UNBIASED):
    """Pion correlator C(dt) and the stochastic operators O."""
    O = stochastic_operators(eta, X)
    return pion_from_O(O, mode), O


def pipi_from_O(O, normalise=True):
    """(diagrams[4, T] = D0..D3, vac[T]) from the four-group block structure of O."""
    O = _c(O)
    T, N, _ = O.shape
    d = np.empty((4, T), np.complex128)
    v = np.empty(T, np.complex128)
    _check(lib().orc_pipi_from_O(T, N, _p(O), 1 if normalise else 0, _p(d), _p(v)), "pipi_from_O")
    return d, v


def contract_pipi(eta, X):
    return pipi_from_O(stochastic_operators(eta, X), True)


# ------------------------------------------------------------------------------------------
# even-odd helpers (plain definitions on full-lattice arrays)
# ------------------------------------------------------------------------------------------
def parity_mask(dims):
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return ((x + y + z + t) & 1).astype(np.int8)


def schur_rhs(U, A, Ainv, kappa, eta, tbc):
    """b_o = eta_o + kappa H_oe A_ee^{-1} eta_e, returned as a full-lattice field (zero on even)."""
    dims = _dims(U)
    odd = parity_mask(dims)[..., None, None] == 1
    e = np.where(odd, 0, eta)
    t = site_matvec(Ainv, e)
    t = np.where(odd, 0, t)
    h = hop(U, t, tbc)
    return np.where(odd, eta + kappa * h, 0)


def reconstruct_even(U, Ainv, kappa, eta, x_odd, tbc):
    """x_e = A_ee^{-1}(eta_e + kappa H_eo x_o); returns the full solution."""
    dims = _dims(U)
    odd = parity_mask(dims)[..., None, None] == 1
    xo = np.where(odd, x_odd, 0)
    h = hop(U, xo, tbc)
    xe = site_matvec(Ainv, np.where(odd, 0, eta + kappa * h))
    return np.where(odd, xo, xe)


# ---------------------------------------------------------------------------------------
# outer-product fill of the all-to-all propagator (Sec. 7, eq. Sfill) and its contraction
# ---------------------------------------------------------------------------------------
def fill_propagator(eta, X, t_src, t, dagger=False):
    """S(t, z; t_src, x)_{ab} = (1/N) sum_i X_i(t, z)_a conj(eta_i(t_src, x)_b) (Sec. 7, eq. Sfill),
    as a (12 L^3) x (12 L^3) matrix with row (z, a) and column (x, b): spatial sites in the
    canonical order (x fastest), a = 3 spin + colour.  dagger=True gives the spin-colour dagger
    of every 12 x 12 block, S(t, z; t_src, x)^dag (Sec. 7: the dagger acts on spin and colour
    only; the site indices are already exchanged)."""
    eta, X = _c(eta), _c(X)
    N = eta.shape[0]
    n = X[0, t].size
    S = np.zeros((n, n), np.complex128)
    for i in range(N):  # one outer product per source, summed in source order
        S += np.outer(X[i, t].ravel(), np.conj(eta[i, t_src].ravel()))
    S /= N
    if dagger:
        m = n // 12
        S = np.conj(S.reshape(m, 12, m, 12).transpose(0, 3, 2, 1)).reshape(n, n)
    return S


def contract_fill(eta1, X1, eta2, X2, t_src):
    """C(t) = sum_{z, x} tr[S1(t, z; t_src, x) S2(t, z; t_src, x)^dag] for every sink timeslice t,
    with S1 filled from (eta1, X1) and S2 from an independent set (eta2, X2) (the paper's
    "sum_x sum_z tr S_s S_s^dag" with independent noise for the two propagators, Sec. 7)."""
    T = _c(X1).shape[1]
    C = np.empty(T, np.complex128)
    for t in range(T):
        S1 = fill_propagator(eta1, X1, t_src, t)
        S2 = fill_propagator(eta2, X2, t_src, t)
        C[t] = np.sum(S1 * np.conj(S2))  # tr[S1 S2^dag] summed over both sites
    return C


# ---------------------------------------------------------------------------------------
# dilution and momentum projection (Sec. 7: time-spin-colour dilution; Sec. 5 momentum
# projection of the pion operators)
# ---------------------------------------------------------------------------------------
DILUTE_NONE, DILUTE_T, DILUTE_SC, DILUTE_TSC = 0, 1, 2, 3


def dilution_size(scheme, T):
    return {DILUTE_NONE: 1, DILUTE_T: T, DILUTE_SC: 12, DILUTE_TSC: 12 * T}[scheme]


def dilute(eta, scheme):
    """Diluted sources: every noise vector eta_i is split into pieces with disjoint supports
    (one timeslice, one spin-colour component, or both), in the order noise vector, then
    piece d = t, d = 3 spin + colour, or d = 12 t + 3 spin + colour.  The pieces of one noise
    vector sum to it."""
    eta = _c(eta)
    N, T = eta.shape[0], eta.shape[1]
    D = dilution_size(scheme, T)
    out = np.zeros((N * D,) + eta.shape[1:], np.complex128)
    for i in range(N):
        for d in range(D):
            v = out[i * D + d]
            if scheme == DILUTE_NONE:
                v[...] = eta[i]
            elif scheme == DILUTE_T:
                v[d] = eta[i, d]
            elif scheme == DILUTE_SC:
                v[..., d // 3, d % 3] = eta[i, ..., d // 3, d % 3]
            else:
                t, sc = d // 12, d % 12
                v[t, ..., sc // 3, sc % 3] = eta[i, t, ..., sc // 3, sc % 3]
    return out


def momentum_phase(dims, p):
    """exp(-i p.y) on the spatial sites (z, y, x), p = 2 pi (n_x / X, n_y / Y, n_z / Z)."""
    X, Y, Z = dims[0], dims[1], dims[2]
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return np.exp(-2j * np.pi * (p[0] * x / X + p[1] * y / Y + p[2] * z / Z))


def stochastic_operators_mom(eta, X, p):
    """O[t, a, b] = sum_{y in t} exp(-i p.y) eta_a(y)^dag gamma_5 X_b(y) (eq. stoop with the
    momentum projection of the operator at the source)."""
    eta, X = _c(eta), _c(X)
    T = eta.shape[1]
    dims = (eta.shape[4], eta.shape[3], eta.shape[2], T)
    ph = momentum_phase(dims, p)
    g5 = np.real(np.diag(gamma(4)))
    O = np.empty((T, eta.shape[0], X.shape[0]), np.complex128)
    for t in range(T):
        O[t] = np.einsum("azyxsc,zyx,s,bzyxsc->ab", np.conj(eta[:, t]), ph, g5, X[:, t])
    return O


def pion_mom(eta, X, p, group=1, mode=MODE_UNBIASED):
    """C(dt, p) = sum_{t0} sum_{a, b} O_ab(t0 + dt, p) O_ba(t0, -p) over pairs of sources from
    different noise vectors (sources a and b belong to noise vectors a // group, b // group;
    group = pieces per noise vector after dilution), normalised by 1 / (T n (n - 1)) with n
    noise vectors; MODE_RAW_ALL sums every pair without normalisation."""
    Op = stochastic_operators_mom(eta, X, p)
    Om = stochastic_operators_mom(eta, X, [-q for q in p])
    T, N, _ = Op.shape
    noise = np.arange(N) // group
    keep = np.ones((N, N)) if mode == MODE_RAW_ALL else (noise[:, None] != noise[None, :]).astype(float)
    C = np.empty(T, np.complex128)
    for dt in range(T):
        acc = 0j
        for t0 in range(T):
            acc += np.sum(keep * Op[(t0 + dt) % T] * Om[t0].T)
        C[dt] = acc
    if mode != MODE_RAW_ALL:
        n = N // group
        C /= T * n * (n - 1)
    return C


# ---------------------------------------------------------------------------------------
# point-source propagators and the pi-pi diagrams that combine them with stochastic ones
# (Sec. 8: diagram 2 from point propagators at the origin and stochastic propagators sourced
# at (t, z); diagram 1 from a stochastic timeslice loop and a point loop at the source)
# ---------------------------------------------------------------------------------------
def point_sources(dims, t0, x0):
    """The 12 unit sources at the site (t0, x0), x0 = (x, y, z): source k is 1 in spin-colour
    component k = 3 spin + colour there and 0 everywhere else."""
    X, Y, Z, T = dims
    e = np.zeros((12, T, Z, Y, X, 4, 3), np.complex128)
    for k in range(12):
        e[k, t0, x0[2], x0[1], x0[0], k // 3, k % 3] = 1.0
    return e


def _point_blocks(Sp, t):
    """S_p(t, y) for every spatial site y of timeslice t as [y][a][k]: a = sink spin-colour,
    k = source spin-colour (the solution of point source k)."""
    return np.moveaxis(Sp[:, t].reshape(12, -1, 12), 0, 2)


def pipi_mixed(Sp, t0, eta1, X1, eta2, X2):
    """The pi-pi diagrams with point propagators S_p(w) = S(w; t0, x0) (Sp = the solutions of
    the 12 point sources at (t0, x0)) and stochastic all-to-all propagators S1, S2 filled from
    two noise sets (eq. Sfill, normalised by 1/N1 and 1/N2), on one configuration, for every
    separation dt with t = t0 + dt (mod T):

      Cp(dt) = sum_y tr[S_p(t, y) S_p(t, y)^dag]                       point pion
      Cs(dt) = sum_{z, x} tr[S1(t, z; t0, x) S2(t, z; t0, x)^dag]      all-to-all pion
      L(dt)  = sum_{z, y} tr[S1(t, z; t, y) S2(t, z; t, y)^dag]        timeslice loop at t
      D0 = Cp Cs,  D1 = L Cp(0)                                        (Sec. 7 and Sec. 8)
      D2(dt) = sum_{x, y, z} tr[S_p(t0, x)^dag S1(t0, x; t, z) S2(t, y; t, z)^dag S_p(t, y)]
      D3 = conj(D2)

    (daggers on spin and colour only).  D0 and D1 are unsubtracted; their vacuum parts need
    ensemble averages of the pieces.  Returns (diagrams[4, T], pieces[3, T] = Cp, Cs, L)."""
    Sp = _c(Sp)
    T = Sp.shape[1]
    m = Sp[0, 0].size // 12  # spatial sites per timeslice
    P0 = _point_blocks(Sp, t0)
    cp0 = np.sum(np.abs(P0) ** 2)
    diagrams = np.zeros((4, T), np.complex128)
    pieces = np.zeros((3, T), np.complex128)
    for dt in range(T):
        t = (t0 + dt) % T
        Pt = _point_blocks(Sp, t)
        cp = np.sum(np.abs(Pt) ** 2)
        # tr[A B^dag] summed over both site indices is sum A conj(B) over all entries
        cs = np.sum(fill_propagator(eta1, X1, t0, t) * np.conj(fill_propagator(eta2, X2, t0, t)))
        S1tt = fill_propagator(eta1, X1, t, t)
        S2tt = fill_propagator(eta2, X2, t, t)
        loop = np.sum(S1tt * np.conj(S2tt))
        S1 = fill_propagator(eta1, X1, t, t0).reshape(m, 12, m, 12)  # S1(t0, x; t, z): [x][a][z][b]
        S2 = S2tt.reshape(m, 12, m, 12)                                # S2(t, y; t, z): [y][c][z][d]
        # tr[S_p(t0,x)^dag S1(t0,x;t,z) S2(t,y;t,z)^dag S_p(t,y)]: the (b, c) entry of the block
        # S2(t,y;t,z)^dag is conj(S2[y][c][z][b])
        d2 = np.einsum("xak,xazb,yczb,yck->", np.conj(P0), S1, np.conj(S2), Pt, optimize=True)
        diagrams[:, dt] = (cp * cs, loop * cp0, d2, np.conj(d2))
        pieces[:, dt] = (cp, cs, loop)
    return diagrams, pieces
