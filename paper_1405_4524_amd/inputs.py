"""Seeded synthetic inputs: near-identity SU(3) gauge fields and complex-Z2 noise sources.

This module only *draws inputs*; it holds none of the solver's or the contraction's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

Gauge field (stand-in for the paper's quenched ensemble, Sec. 8, which is not available):
    for every link draw a 3x3 complex matrix A with independent N(0,1) real and imaginary
    parts, form the traceless Hermitian H = (A + A^dag)/2 - tr(.)/3, and set
    U = exp(i eps H) through the eigen-decomposition of H.  The draws come from
    numpy's PCG64 stream in C order over the shape (T, Z, Y, X, 4, 3, 3, 2).

Noise (Sec. 7, eq. for the stochastic estimator: "Z2 noise"): every (source, site,
spin, colour) component is (+-1 +- i)/sqrt(2).  The two signs come from a counter
hash, so any slice can be regenerated independently and any other implementation of
the same published generator reproduces it bit for bit:
    k = ((src * V + site) * 4 + spin) * 3 + colour     (site lexicographic, x fastest)
    h = splitmix64_first_output(state = seed * 2**48 + k)
    Re sign = bit 0 of h, Im sign = bit 1 of h (bit set means minus).
splitmix64 is the generator of Steele, Lea and Flood (OOPSLA 2014): the state is
advanced by the golden-ratio increment 0x9E3779B97F4A7C15 and the result is passed
through the variant-13 mixing function (shifts 30, 27, 31).

Layouts (canonical, host side):
    links   [t][z][y][x][mu][row][col] complex128, mu = 0..3 for the x, y, z, t directions
    spinors [src][t][z][y][x][spin][colour] complex128
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def volume(dims):
    X, Y, Z, T = (int(d) for d in dims)
    return X * Y * Z * T


def check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {dims}")
    return dims


# ---------------------------------------------------------------------------------------
# gauge links
# ---------------------------------------------------------------------------------------
def _su3_from_normals(g, eps):
    """g: (..., 3, 3, 2) standard normals -> exp(i eps H) with H the traceless Hermitian part."""
    a = g[..., 0] + 1j * g[..., 1]
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return (v * ph[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def gauge_field(dims, eps, seed, out=None):
    """Near-identity SU(3) links U = exp(i eps H), H Gaussian traceless Hermitian.

    Returns complex128 array of shape (T, Z, Y, X, 4, 3, 3).  Generated one timeslice at
    a time (the PCG64 normal stream fills C order sequentially, so this equals one draw
    of the whole shape) to keep the peak host memory near the size of the result.
    """
    X, Y, Z, T = check_dims(dims)
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    if out is None:
        out = np.empty((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    for t in range(T):
        g = rng.standard_normal((Z, Y, X, 4, 3, 3, 2))
        out[t] = _su3_from_normals(g, float(eps))
    return out


def unit_gauge(dims):
    X, Y, Z, T = check_dims(dims)
    u = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3(n, seed, eps=1.0):
    """n random SU(3) matrices (used for gauge transformations in tests)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    g = rng.standard_normal((n, 3, 3, 2))
    return _su3_from_normals(g, eps)


# ---------------------------------------------------------------------------------------
# noise
# ---------------------------------------------------------------------------------------
def splitmix64(state):
    """First output of splitmix64 seeded with `state` (uint64 array, wraps mod 2**64)."""
    with np.errstate(over="ignore"):
        z = state.astype(np.uint64) + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def z2_noise(dims, nsrc, seed, src_offset=0, out=None):
    """Complex-Z2 sources (+-1 +- i)/sqrt(2), shape (nsrc, T, Z, Y, X, 4, 3) complex128.

    Source s of the result is global source index src_offset + s.
    """
    X, Y, Z, T = check_dims(dims)
    V = X * Y * Z * T
    per = 12 * V
    if out is None:
        out = np.empty((nsrc, T, Z, Y, X, 4, 3), dtype=np.complex128)
    flat = out.reshape(nsrc, per)
    base = np.uint64(int(seed) << 48)
    idx = np.arange(per, dtype=np.uint64)
    inv = np.sqrt(0.5)  # 1/sqrt(2) correctly rounded
    for s in range(nsrc):
        with np.errstate(over="ignore"):
            k = np.uint64((int(src_offset) + s) * per) + idx
            h = splitmix64(base + k)
        re = np.where((h & np.uint64(1)) != 0, -inv, inv)
        im = np.where((h & np.uint64(2)) != 0, -inv, inv)
        flat[s].real = re
        flat[s].imag = im
    return out


def z2_noise_timeslices(dims, nsrc, seed, ts, src_offset=0):
    """The components of :func:`z2_noise` on the timeslices `ts` only (same counter, so equal
    bit for bit to those timeslices of the whole-lattice draw), shape
    (nsrc, len(ts), Z, Y, X, 4, 3) complex128: large lattices without the whole field."""
    X, Y, Z, T = check_dims(dims)
    V = X * Y * Z * T
    V3 = X * Y * Z
    per = 12 * V
    ts = [int(t) for t in ts]
    out = np.empty((nsrc, len(ts), Z, Y, X, 4, 3), dtype=np.complex128)
    base = np.uint64(int(seed) << 48)
    idx = np.arange(12 * V3, dtype=np.uint64)
    inv = np.sqrt(0.5)
    for s in range(nsrc):
        for j, t in enumerate(ts):
            with np.errstate(over="ignore"):
                k = np.uint64((int(src_offset) + s) * per + t * 12 * V3) + idx
                h = splitmix64(base + k)
            flat = out[s, j].reshape(-1)
            flat.real = np.where((h & np.uint64(1)) != 0, -inv, inv)
            flat.imag = np.where((h & np.uint64(2)) != 0, -inv, inv)
    return out


# ---------------------------------------------------------------------------------------
# named workloads (lattice, field, operator and source parameters)
# ---------------------------------------------------------------------------------------
WORKLOADS = {
    # plain FP64 method on a tiny lattice
    "tiny_4c8": dict(dims=(4, 4, 4, 8), eps=0.20, gauge_seed=1, kappa=0.120, csw=1.0,
                     tbc=-1, nsrc=4, noise_seed=2, tol=1e-10),
    # FP64 / FP32 solver plus pion and pi-pi contractions
    "l16t32": dict(dims=(16, 16, 16, 32), eps=0.30, gauge_seed=1, kappa=0.1250, csw=1.2,
                   tbc=-1, nsrc=16, noise_seed=3, tol=1e-10),
    # FP16 / BF16 storage inner solves with FP64 reliable updates
    "l24t48": dict(dims=(24, 24, 24, 48), eps=0.35, gauge_seed=1, kappa=0.1300, csw=1.5,
                   tbc=-1, nsrc=32, noise_seed=4, tol=1e-10),
    # batched multi-RHS
    "l32t64": dict(dims=(32, 32, 32, 64), eps=0.35, gauge_seed=1, kappa=0.1300, csw=1.5,
                   tbc=-1, nsrc=48, noise_seed=5, tol=1e-10),
}
