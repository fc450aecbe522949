"""GPU parity of dilution and of the momentum-projected pion correlator (a2a_dilute_dev,
a2a_contract_pion_mom_dev) against the oracle: the diluted sources bit-exact; correlators of
the same sources and solutions to 1e-12 relative (FP64, different summation order); at p = 0
without dilution the existing unbiased pion; end to end, diluted sources solved on the GPU
against the oracle's solutions of the same sources (solves to 1e-12: correlators within 1e-9)."""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs

pytestmark = pytest.mark.gpu

MOMS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (3, 0, 1)]


@pytest.fixture(scope="module")
def ctx():
    from paper_1405_4524_amd import a2a

    c = a2a.Context(0)
    yield c
    c.finalize()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64)).cuda()


def host(t, n):
    return t.cpu().numpy().view(np.complex128)[..., 0][:n]


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_dilution_bit_exact(ctx, orc, scheme):
    import torch

    dims = (4, 2, 2, 4)
    eta = inputs.z2_noise(dims, 3, seed=41)
    D = orc.dilution_size(scheme, dims[3])
    out = torch.empty((3 * D,) + eta.shape[1:] + (2,), dtype=torch.float64, device="cuda")
    ctx.dilute_dev(dev(eta), 3, dims, scheme, out)
    assert np.array_equal(host(out, 3 * D), orc.dilute(eta, scheme))


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_pion_mom_matches_oracle(ctx, orc, scheme):
    print(f"[gpu] momentum pion scheme={scheme}", flush=True)
    dims = (4, 2, 2, 4)
    eta = orc.dilute(inputs.z2_noise(dims, 3, seed=42), scheme)
    G = orc.dilution_size(scheme, dims[3])
    rng = np.random.default_rng(7)
    X = rng.normal(size=eta.shape) + 1j * rng.normal(size=eta.shape)
    n = eta.shape[0]
    for mode in (0, 3):
        got = ctx.contract_pion_mom_dev(dev(eta), dev(X), n, dims, MOMS, scheme=scheme, mode=mode)
        for m, p in enumerate(MOMS):
            want = orc.pion_mom(eta, X, p, group=G, mode=mode)
            err = np.max(np.abs(got[m] - want)) / np.max(np.abs(want))
            assert err < 1e-12, (mode, p, err)


def test_zero_momentum_is_the_pion(ctx):
    dims = (4, 4, 2, 6)
    eta = inputs.z2_noise(dims, 5, seed=43)
    rng = np.random.default_rng(8)
    X = rng.normal(size=eta.shape) + 1j * rng.normal(size=eta.shape)
    got = ctx.contract_pion_mom_dev(dev(eta), dev(X), 5, dims, [(0, 0, 0)])[0]
    want, _ = ctx.contract_pion_2pt(eta, X)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_diluted_solve_and_momentum_correlator_end_to_end(ctx, orc):
    """Time-diluted sources of three noise vectors on 4^3x8, solved on the GPU (FP16 inner,
    FP64 reliable updates) and by the oracle; correlators at four momenta."""
    import torch

    from paper_1405_4524_amd import a2a

    print("[gpu] diluted solve + momentum correlator", flush=True)
    dims, tbc, kappa, csw = (4, 4, 4, 8), -1, 0.12, 1.0
    U = inputs.gauge_field(dims, 0.2, 1)
    A = orc.clover(U, kappa, csw)
    noise = inputs.z2_noise(dims, 3, seed=44)
    G = dims[3]
    src = torch.empty((3 * G,) + noise.shape[1:] + (2,), dtype=torch.float64, device="cuda")
    ctx.dilute_dev(dev(noise), 3, dims, a2a.DILUTE_T, src)
    sol = torch.zeros_like(src)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    info, rc = ctx.solve_propagators_dev(c, src, sol, 3 * G, kappa, csw, tol=1e-12, prec=a2a.F16_F32)
    assert rc == 0
    got = ctx.contract_pion_mom_dev(src, sol, 3 * G, dims, MOMS, scheme=a2a.DILUTE_T)
    eta_d = orc.dilute(noise, orc.DILUTE_T)
    Xo, io = orc.solve(U, A, kappa, eta_d, tbc, tol=1e-12)
    assert np.all(io[:, 2] == 1)
    for m, p in enumerate(MOMS):
        want = orc.pion_mom(eta_d, Xo, p, group=G)
        err = np.max(np.abs(got[m] - want)) / np.max(np.abs(want))
        assert err < 1e-9, (p, err)
    ctx.unload(g)
