"""GPU test of the allocation-free pion contraction (a2a_contract_pion_2pt_noalloc) against the
allocating entry point (a2a_contract_pion_2pt_dev) on the same device inputs, two calls in a
row with the second smaller, and against the oracle's stochastic operators.

Tolerance: 1e-12 relative (FP64 in both; the allocation-free call may split the site sum into
fewer chunks, so only the summation order differs).  The device memory in use by the library
must not change across the calls.
"""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.fixture(scope="module")
def ctx():
    from paper_1405_4524_amd import a2a

    print("\n[gpu] creating a2a context (allocation-free contraction)", flush=True)
    c = a2a.Context(0)
    yield c
    c.finalize()


CASES = [((6, 4, 4, 10), 20, 11), ((4, 4, 4, 8), 6, 12)]  # second call smaller


@pytest.mark.parametrize("want_O", [True, False])
def test_noalloc_pion_matches_allocating_call(ctx, orc, want_O):
    import torch

    dev = torch.device("cuda:0")
    for dims, n, seed in CASES:
        print(f"[gpu] no-alloc pion contraction dims={dims} n={n} want_O={want_O}", flush=True)
        X, Y, Z, T = dims
        eta = torch.empty((n, T, Z, Y, X, 4, 3, 2), dtype=torch.float64, device=dev)
        xs = torch.empty_like(eta)
        ctx.z2_noise_dev(dims, seed, 0, n, eta)
        rng = np.random.default_rng(seed)
        xs.copy_(torch.from_numpy(rng.standard_normal(tuple(xs.shape))))
        corr_ref, O_ref = ctx.contract_pion_2pt_dev(eta, xs, n, dims, -1, want_O=True)
        corr_t = torch.full((T,), float("nan"), dtype=torch.complex128, device=dev)
        O_t = torch.full((T, n, n), float("nan"), dtype=torch.complex128, device=dev) if want_O else None
        used = ctx.mem_in_use()
        ctx.contract_pion_2pt_noalloc(eta, xs, n, dims, corr_t, O_t, -1)
        torch.cuda.synchronize()
        assert ctx.mem_in_use() == used
        corr = corr_t.cpu().numpy()
        assert np.all(np.isfinite(corr))
        assert rel(corr, corr_ref) <= 1e-12, rel(corr, corr_ref)
        if want_O:
            O = O_t.cpu().numpy()
            assert rel(O, O_ref) <= 1e-12, rel(O, O_ref)
        # against the oracle on the host copies of the same inputs
        he = eta.cpu().numpy().view(np.complex128).reshape(n, T, Z, Y, X, 4, 3)
        hx = xs.cpu().numpy().view(np.complex128).reshape(n, T, Z, Y, X, 4, 3)
        want = orc.pion_from_O(orc.stochastic_operators(he, hx))
        assert rel(corr, want) <= 1e-12, rel(corr, want)


def test_noalloc_pion_rejects_oversize(ctx):
    import torch

    from paper_1405_4524_amd import a2a

    dims, n = (2, 2, 2, 64), 400  # 16 T n^2 = 164 MB > 32 MiB: refused before any launch
    dev = torch.device("cuda:0")
    eta = torch.zeros((n, 64, 2, 2, 2, 4, 3, 2), dtype=torch.float64, device=dev)
    corr_t = torch.zeros((64,), dtype=torch.complex128, device=dev)
    with pytest.raises(a2a.A2AError) as e:
        ctx.contract_pion_2pt_noalloc(eta, eta, n, dims, corr_t, None, -1)
    assert e.value.code == a2a.EINVAL
