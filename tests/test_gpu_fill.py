"""GPU parity of the outer-product fill (Sec. 7, eq. Sfill) and of the two routes to
sum_{z,x} tr[S1 S2^dag], against the oracle's plain definitions on host-generated complex
fields.  FP64 throughout; the products differ from the oracle only in summation order, so
the tolerance is 1e-13 relative for S and 1e-12 for the correlator.  Lattices give a timeslice
of 768 (whole 64-row tiles) and 288 (a ragged tile) spin-colour components; source counts that
are not multiples of the K step of 4 exercise the zero padding."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1405_4524_amd import a2a

    c = a2a.Context(0)
    yield c
    c.finalize()


def fields(dims, n, seed):
    X, Y, Z, T = dims
    rng = np.random.default_rng(seed)
    shape = (n, T, Z, Y, X, 4, 3)
    return [rng.normal(size=shape) + 1j * rng.normal(size=shape) for _ in range(4)]


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64)).cuda()


CASES = [((4, 4, 4, 8), 10, 1), ((2, 6, 2, 4), 7, 3), ((2, 6, 2, 4), 1, 0)]


@pytest.mark.parametrize("dims,n,t_src", CASES)
def test_fill_matches_oracle(ctx, orc, dims, n, t_src):
    import torch

    print(f"[gpu] fill {dims} n={n} t_src={t_src}", flush=True)
    eta, X, _, _ = fields(dims, n, 11)
    M = 12 * dims[0] * dims[1] * dims[2]
    de, dx = dev(eta), dev(X)
    S = torch.empty((M, M, 2), dtype=torch.float64, device="cuda")
    for t in (0, dims[3] - 1):
        for dagger in (False, True):
            ctx.fill_propagator_dev(dx, de, n, dims, t_src, t, S, dagger=dagger)
            got = S.cpu().numpy().view(np.complex128)[..., 0]
            want = orc.fill_propagator(eta, X, t_src, t, dagger=dagger)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert err < 1e-13, (t, dagger, err)


@pytest.mark.parametrize("dims,n,t_src", CASES)
def test_fill_and_gram_contractions_match_oracle(ctx, orc, dims, n, t_src):
    print(f"[gpu] fill contraction {dims} n={n} t_src={t_src}", flush=True)
    eta1, X1, eta2, X2 = fields(dims, n, 12)
    want = orc.contract_fill(eta1, X1, eta2, X2, t_src)
    d = [dev(a) for a in (X1, eta1, X2, eta2)]
    for method in ("fill", "gram"):
        got = ctx.contract_fill_2pt_dev(*d, n, dims, t_src, method=method)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert err < 1e-12, (method, err)


def test_fill_errors(ctx):
    from paper_1405_4524_amd import a2a

    dims = (2, 2, 2, 4)
    eta, X, _, _ = fields(dims, 2, 13)
    import torch

    S = torch.empty((96, 96, 2), dtype=torch.float64, device="cuda")
    for bad in (dict(t_src=4, t=0), dict(t_src=0, t=-1)):
        with pytest.raises(a2a.A2AError) as e:
            ctx.fill_propagator_dev(dev(X), dev(eta), 2, dims, bad["t_src"], bad["t"], S)
        assert e.value.code == a2a.EINVAL
    with pytest.raises(a2a.A2AError) as e:
        ctx.fill_propagator_dev(dev(X), dev(eta), 0, dims, 0, 0, S)
    assert e.value.code == a2a.EINVAL


def test_full_dilution_fill_is_exact(ctx, orc):
    """Unit sources on the source timeslice, solved on the GPU: M^2 sum tr[S S^dag] through both
    routes equals the squared Frobenius norm of the dense inverse's block (LAPACK), per t."""
    import torch

    from paper_1405_4524_amd import a2a, inputs
    from tests.test_oracle_pins import dense_operator

    print("[gpu] full dilution fill", flush=True)
    dims, tbc, kappa, csw = (2, 2, 2, 4), -1, 0.125, 1.3
    X_, Y, Z, T = dims
    M = 12 * X_ * Y * Z
    U = inputs.gauge_field(dims, 0.4, seed=71)
    A = orc.clover(U, kappa, csw)
    Dinv = np.linalg.inv(dense_operator(lambda v: orc.apply_D(U, A, kappa, v, tbc), dims))
    want = np.array([np.sum(np.abs(Dinv[t * M:(t + 1) * M, 0:M]) ** 2) for t in range(T)])
    unit = torch.zeros((M, T, Z, Y, X_, 4, 3, 2), dtype=torch.float64, device="cuda")
    unit.view(M, T, M, 2)[torch.arange(M), 0, torch.arange(M), 0] = 1.0
    sol = torch.zeros_like(unit)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    info, rc = ctx.solve_propagators_dev(c, unit, sol, M, kappa, csw, tol=1e-12, prec=a2a.F64)
    assert rc == 0
    for method in ("fill", "gram"):
        got = M * M * ctx.contract_fill_2pt_dev(sol, unit, sol, unit, M, dims, 0, method=method)
        assert np.max(np.abs(got - want)) < 1e-9 * np.max(want), method
    ctx.unload(g)
