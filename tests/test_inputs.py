"""Seeded input generators: SU(3) links and counter-hash complex-Z2 noise."""
import numpy as np

from paper_1405_4524_amd import inputs


def test_splitmix64_published_vectors():
    """splitmix64 (Steele, Lea, Flood 2014) seeded with 1234567: the first five outputs as
    published with the reference implementation; output k is mix(seed + (k+1) * golden)."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    seed = np.uint64(1234567)
    with np.errstate(over="ignore"):
        states = np.array([seed + np.uint64(k) * inputs.GOLDEN for k in range(5)], dtype=np.uint64)
    got = [int(v) for v in inputs.splitmix64(states)]
    assert got == want


def test_noise_is_complex_z2_and_counter_addressed():
    dims = (2, 4, 2, 4)
    eta = inputs.z2_noise(dims, 5, seed=9)
    assert np.all(np.abs(np.abs(eta) - 1.0) < 1e-15)
    assert set(np.unique(np.round(eta.real * np.sqrt(2)))) == {-1.0, 1.0}
    # slices regenerate independently from the global source index
    part = inputs.z2_noise(dims, 2, seed=9, src_offset=3)
    assert np.array_equal(part, eta[3:5])
    # statistics: mean ~ 0, E|eta|^2 = 1, components nearly uncorrelated
    big = inputs.z2_noise((4, 4, 4, 8), 8, seed=2).ravel()
    assert abs(big.mean()) < 4 / np.sqrt(big.size)
    assert abs(np.mean(big[:-1] * np.conj(big[1:]))) < 4 / np.sqrt(big.size)


def test_noise_bit_layout():
    """Component k of the flattened source uses bits 0 / 1 of splitmix64(seed * 2^48 + k)."""
    dims = (2, 2, 2, 2)
    seed = 5
    eta = inputs.z2_noise(dims, 2, seed=seed).reshape(-1)
    ks = np.array([0, 1, 17, 191, 192, 383], dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = inputs.splitmix64(np.uint64(seed << 48) + ks)
    for k, hv in zip(ks, h):
        re = -1 if int(hv) & 1 else 1
        im = -1 if int(hv) & 2 else 1
        assert eta[int(k)] == (re + 1j * im) * np.sqrt(0.5)
    # the modulus factor is 1/sqrt(2) correctly rounded (the same double every generator uses)
    assert np.sqrt(0.5) == float.fromhex("0x1.6a09e667f3bcdp-1")


def test_gauge_links_are_su3_and_chunking_is_exact():
    dims = (2, 4, 2, 4)
    U = inputs.gauge_field(dims, 0.35, seed=1)
    Ud = np.conj(np.swapaxes(U, -1, -2))
    assert np.max(np.abs(U @ Ud - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14
    # generated per timeslice == one draw of the whole shape
    rng = np.random.Generator(np.random.PCG64(1))
    g = rng.standard_normal((dims[3], dims[2], dims[1], dims[0], 4, 3, 3, 2))
    whole = inputs._su3_from_normals(g, 0.35)
    assert np.max(np.abs(whole - U)) < 1e-15


def test_gauge_near_identity_scale():
    """Mean link trace shrinks with eps as expected for exp(i eps H), E tr H^2 = 8."""
    U = inputs.gauge_field((4, 4, 4, 4), 0.35, seed=1)
    u0 = np.mean(np.trace(U, axis1=-2, axis2=-1).real) / 3
    # second-order estimate: 1 - eps^2 E tr H^2 / 6 = 1 - 0.35^2 * 8 / 6 = 0.837
    assert 0.80 < u0 < 0.87


def test_noise_timeslices_equal_whole_draw():
    dims = (4, 2, 6, 8)
    whole = inputs.z2_noise(dims, 3, 9, src_offset=2)
    part = inputs.z2_noise_timeslices(dims, 3, 9, [0, 5, 7], src_offset=2)
    assert np.array_equal(whole[:, [0, 5, 7]], part)
