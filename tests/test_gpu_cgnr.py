"""GPU tests of CG on the normal equations (option "solver" = CGNR) and of the CGNR fallback
after BiCGStab breakdowns: every source meets the binding criterion with the oracle's D, the
solutions agree with the oracle's CGNR solutions (both solved to 1e-10 or tighter; cond(D)
~ 10-100 bounds the difference by ~1e-8), and the info records name the method that finished
each source."""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.fixture(scope="module")
def ctx():
    from paper_1405_4524_amd import a2a

    c = a2a.Context(0)
    yield c
    c.finalize()


class options:
    def __init__(self, ctx, **kw):
        self.ctx, self.kw = ctx, kw

    def __enter__(self):
        for k, v in self.kw.items():
            self.ctx.set_option(k, v)

    def __exit__(self, *exc):
        defaults = dict(solver=0, cgnr_fallback=1, force_breakdown=0, interleave=1, mfma=1)
        for k in self.kw:
            self.ctx.set_option(k, defaults[k])


@pytest.fixture(scope="module")
def lattice(ctx, orc):
    dims, tbc, kappa, csw = (4, 4, 4, 8), -1, 0.125, 1.5
    U = inputs.gauge_field(dims, 0.35, 61)
    A = orc.clover(U, kappa, csw)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    eta = inputs.z2_noise(dims, 20, seed=62)  # FP16 / BF16: one 16-lane group + 4 per slot
    Xo, io = orc.solve_cgnr(U, A, kappa, eta[:4], tbc, tol=1e-12)
    assert np.all(io[:, 2] == 1)
    yield dict(dims=dims, tbc=tbc, kappa=kappa, csw=csw, U=U, A=A, c=c, eta=eta, Xo=Xo)
    ctx.unload(g)


def check_solutions(orc, L, X, n):
    for i in range(n):
        r = L["eta"][i] - orc.apply_D(L["U"], L["A"], L["kappa"], X[i], L["tbc"])
        assert np.linalg.norm(r) / np.linalg.norm(L["eta"][i]) <= 1e-10, i
    for i in range(4):
        assert rel(X[i], L["Xo"][i]) < 1e-8, i


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_cgnr_solve(ctx, orc, lattice, prec):
    from paper_1405_4524_amd import a2a

    print(f"[gpu] cgnr solve prec={prec}", flush=True)
    L = lattice
    with options(ctx, solver=a2a.SOLVER_CGNR):
        X, info, rc = ctx.solve_propagators(L["c"], L["eta"], L["kappa"], L["csw"], tol=1e-10, prec=prec,
                                            max_iter=20000)
    assert rc == 0, [x for x in info if not x["converged"]][:3]
    assert all(x["solver"] == a2a.SOLVER_CGNR and x["converged"] == 1 for x in info)
    check_solutions(orc, L, X, 20)
    # the normal equations square the condition number: more iterations than BiCGStab
    Xb, infb, rc = ctx.solve_propagators(L["c"], L["eta"][:4], L["kappa"], L["csw"], tol=1e-10, prec=prec)
    assert rc == 0 and all(x["solver"] == a2a.SOLVER_BICGSTAB for x in infb)
    assert np.mean([x["iters"] for x in info[:4]]) > np.mean([x["iters"] for x in infb])


@pytest.mark.parametrize("mfma", [1, 0])
def test_cgnr_interleaved_per_thread_and_matrix_cores(ctx, orc, lattice, mfma):
    """FP16 storage, 20 sources (one interleaved group and 4 per-slot arenas), with the matrix-
    core stencil and with the per-thread stencil on the same layout."""
    from paper_1405_4524_amd import a2a

    print(f"[gpu] cgnr interleaved mfma={mfma}", flush=True)
    L = lattice
    with options(ctx, solver=a2a.SOLVER_CGNR, mfma=mfma):
        X, info, rc = ctx.solve_propagators(L["c"], L["eta"], L["kappa"], L["csw"], tol=1e-10, prec=2,
                                            max_iter=20000)
    assert rc == 0
    check_solutions(orc, L, X, 20)


def test_cgnr_fallback_after_breakdown(ctx, orc, lattice):
    """With the breakdown hook every BiCGStab source stops at its first reliable update; the
    fallback finishes each one with CGNR from that iterate.  Without the fallback the call
    reports the breakdown."""
    from paper_1405_4524_amd import a2a

    print("[gpu] cgnr fallback", flush=True)
    L = lattice
    with options(ctx, force_breakdown=1):
        X, info, rc = ctx.solve_propagators(L["c"], L["eta"], L["kappa"], L["csw"], tol=1e-10, prec=2,
                                            max_iter=20000)
    assert rc == 0
    assert all(x["solver"] == a2a.SOLVER_CGNR and x["converged"] == 1 for x in info)
    check_solutions(orc, L, X, 20)
    with options(ctx, force_breakdown=1, cgnr_fallback=0):
        X, info, rc = ctx.solve_propagators(L["c"], L["eta"][:3], L["kappa"], L["csw"], tol=1e-10, prec=1,
                                            max_iter=20000, allow=(a2a.EBREAKDOWN,))
    assert rc == a2a.EBREAKDOWN
    assert all(x["solver"] == a2a.SOLVER_BICGSTAB and x["converged"] == 0 for x in info)
    # the breakdown left the iterate of the first update in place: finite and partly converged
    for i in range(3):
        assert 0 < info[i]["true_rel_residual"] < 1


def test_engine_cgnr_and_bicgstab_requests(ctx, orc, lattice):
    """Requests submitted under each solver option run side by side in one engine."""
    import torch

    from paper_1405_4524_amd import a2a

    print("[gpu] engine cgnr + bicgstab", flush=True)
    L = lattice
    eng = ctx.engine_create('{"max_slots": 64, "check_every": 4}')
    reqs = []
    for k, (method, n, prec) in enumerate([(a2a.SOLVER_CGNR, 20, 2), (a2a.SOLVER_BICGSTAB, 5, 2),
                                           (a2a.SOLVER_CGNR, 3, 1)]):
        src = torch.from_numpy(L["eta"][:n]).cuda()
        sol = torch.zeros_like(src)
        with options(ctx, solver=method):
            t = eng.submit(L["c"], L["kappa"], src, n, 1e-10, prec, 20000, sol)
        reqs.append((t, n, method, src, sol))
    for _ in range(3000):
        eng.step(8)
        if all(eng.poll(t, n)[0] != 0 for t, n, *_ in reqs):
            break
    for t, n, method, src, sol in reqs:
        done, info, rc = eng.poll(t, n)
        assert done == 1 and rc == 0, (done, rc)
        assert all(x["solver"] == method and x["converged"] == 1 for x in info)
        X = sol.cpu().numpy()
        if n >= 4:
            check_solutions(orc, L, X, n)
        else:
            for i in range(n):
                r = L["eta"][i] - orc.apply_D(L["U"], L["A"], L["kappa"], X[i], L["tbc"])
                assert np.linalg.norm(r) / np.linalg.norm(L["eta"][i]) <= 1e-10
    eng.destroy()
