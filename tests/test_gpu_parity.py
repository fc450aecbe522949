"""GPU parity: every stage of the HIP path, called through the C ABI, against the FP64 oracle
on the same seeded inputs.

Tolerances (relative 2-norm over the whole output unless stated):
  operators  FP64 1e-13 (rounding order only); FP32 2e-6 and FP16 4e-3, BF16 3e-2: the inputs,
             links and clover are rounded to the storage format (unit roundoff u = 6e-8, 4.9e-4,
             3.9e-3) and a site output sums ~60 such terms, so the error stays a few u.
  solves     the binding criterion: ||eta - D X|| / ||eta|| <= tol, recomputed here with the
             oracle's own D on the GPU's X; and ||X - X_oracle|| / ||X_oracle|| <= 1e-9 for
             solves at tol 1e-12 (error <= cond(D) * tol, cond(D) ~ 10-100 here).
  contractions 1e-12 (FP64, different summation order); the noise generator bit-exact.
"""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs

pytestmark = pytest.mark.gpu

OP_TOL = {0: 1e-13, 1: 2e-6, 2: 4e-3, 3: 3e-2}


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.fixture(scope="module")
def ctx():
    from paper_1405_4524_amd import a2a

    print("\n[gpu] creating a2a context", flush=True)
    c = a2a.Context(0)
    yield c
    c.finalize()


def field(orc, dims, eps, seed, kappa, csw):
    U = inputs.gauge_field(dims, eps, seed)
    A = orc.clover(U, kappa, csw)
    return U, A


# ---------------------------------------------------------------------------------------
# operators: FULL_D, SCHUR, HOP_EO, HOP_OE (and daggers) in every precision
# ---------------------------------------------------------------------------------------
SHAPES = [(2, 2, 2, 2), (4, 2, 6, 4), (6, 4, 4, 10), (8, 8, 8, 8)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("tbc", [-1, 1])
def test_operators_fp64(ctx, orc, dims, tbc):
    from paper_1405_4524_amd import a2a

    print(f"[gpu] operators f64 dims={dims} tbc={tbc}", flush=True)
    kappa, csw = 0.13, 1.4
    U, A = field(orc, dims, 0.5, 3, kappa, csw)
    Ai = orc.invert_sites(A)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    rng = np.random.default_rng(5)
    X, Y, Z, T = dims
    psi = rng.standard_normal((3, T, Z, Y, X, 4, 3)) + 1j * rng.standard_normal((3, T, Z, Y, X, 4, 3))
    odd = (orc.parity_mask(dims) == 1)[..., None, None]
    for op in (a2a.OP_FULL_D, a2a.OP_SCHUR, a2a.OP_HOP_EO, a2a.OP_HOP_OE):
        for dag in (False, True):
            got = ctx.dslash_clover(c, kappa, psi, op=op, dagger=dag, prec=a2a.F64)
            for i in range(3):
                x = psi[i]
                g5 = np.array([1, 1, -1, -1])[:, None]
                xin = g5 * x if dag else x
                if op == a2a.OP_FULL_D:
                    want = orc.apply_D(U, A, kappa, xin, tbc)
                elif op == a2a.OP_SCHUR:
                    want = orc.schur(U, A, Ai, kappa, np.where(odd, xin, 0), tbc)
                elif op == a2a.OP_HOP_EO:
                    want = np.where(odd, 0, orc.hop(U, np.where(odd, xin, 0), tbc))
                else:
                    want = np.where(odd, orc.hop(U, np.where(odd, 0, xin), tbc), 0)
                if dag:
                    want = g5 * want
                assert rel(got[i], want) < OP_TOL[0], (op, dag, i, rel(got[i], want))
    ctx.unload(g)


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_operators_low_precision(ctx, orc, prec):
    from paper_1405_4524_amd import a2a

    dims, tbc = (6, 4, 4, 10), -1
    print(f"[gpu] operators prec={prec} dims={dims}", flush=True)
    kappa, csw = 0.125, 1.2
    U, A = field(orc, dims, 0.35, 7, kappa, csw)
    Ai = orc.invert_sites(A)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    psi = inputs.z2_noise(dims, 2, seed=3)
    odd = (orc.parity_mask(dims) == 1)[..., None, None]
    for op in (a2a.OP_FULL_D, a2a.OP_SCHUR, a2a.OP_HOP_EO):
        got = ctx.dslash_clover(c, kappa, psi, op=op, prec=prec)
        for i in range(2):
            if op == a2a.OP_FULL_D:
                want = orc.apply_D(U, A, kappa, psi[i], tbc)
            elif op == a2a.OP_SCHUR:
                want = orc.schur(U, A, Ai, kappa, np.where(odd, psi[i], 0), tbc)
            else:
                want = np.where(odd, 0, orc.hop(U, np.where(odd, psi[i], 0), tbc))
            assert rel(got[i], want) < OP_TOL[prec], (op, i, rel(got[i], want))
    ctx.unload(g)


@pytest.mark.parametrize("R", [1, 2, 4])
def test_operator_rhs_blocking_is_exact(ctx, orc, R):
    """The multi-RHS stencil gives bitwise the same result per RHS for every block width."""
    from paper_1405_4524_amd import a2a

    dims, tbc = (4, 4, 6, 8), -1
    print(f"[gpu] rhs blocking R={R}", flush=True)
    U, _ = field(orc, dims, 0.4, 11, 0.12, 1.0)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, 1.0)
    psi = inputs.z2_noise(dims, 5, seed=4)
    ctx.set_option("rhs_block", 1)
    ref = ctx.dslash_clover(c, 0.12, psi, op=a2a.OP_SCHUR, prec=a2a.F32)
    ctx.set_option("rhs_block", R)
    got = ctx.dslash_clover(c, 0.12, psi, op=a2a.OP_SCHUR, prec=a2a.F32)
    ctx.set_option("rhs_block", 4)
    assert np.array_equal(got, ref)
    ctx.unload(g)


# ---------------------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------------------
def tiny_workload(orc):
    w = inputs.WORKLOADS["tiny_4c8"]
    U = inputs.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
    A = orc.clover(U, w["kappa"], w["csw"])
    eta = inputs.z2_noise(w["dims"], w["nsrc"], w["noise_seed"])
    return w, U, A, eta


@pytest.fixture(scope="module")
def tiny_ref(orc):
    w, U, A, eta = tiny_workload(orc)
    X, info = orc.solve(U, A, w["kappa"], eta, w["tbc"], tol=1e-13)
    assert np.all(info[:, 2] == 1)
    return w, U, A, eta, X


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_solve_tiny_residual_and_error(ctx, orc, tiny_ref, prec):
    w, U, A, eta, Xo = tiny_ref
    print(f"[gpu] solve tiny prec={prec}", flush=True)
    g = ctx.load_gauge(U, w["tbc"])
    c = ctx.load_clover(g, w["csw"])
    for tol in (1e-10, 1e-12):
        X, info, rc = ctx.solve_propagators(c, eta, w["kappa"], w["csw"], tol=tol, prec=prec, max_iter=20000)
        assert rc == 0, info
        for i in range(w["nsrc"]):
            assert info[i]["converged"] == 1
            r = eta[i] - orc.apply_D(U, A, w["kappa"], X[i], w["tbc"])
            true_rel = np.linalg.norm(r) / np.linalg.norm(eta[i])
            assert true_rel <= tol, (i, true_rel)
            assert abs(true_rel - info[i]["true_rel_residual"]) <= 1e-3 * tol + 1e-15
            if tol == 1e-12:
                assert rel(X[i], Xo[i]) <= 1e-9
    ctx.unload(g)


@pytest.mark.parametrize("R", [1, 2, 4])
@pytest.mark.parametrize("prec", [1, 2])
def test_solve_rhs_block_widths(ctx, orc, R, prec):
    """Every stencil RHS-block width solves to the tolerance (the binding criterion, checked
    with the oracle's D) on a lattice of several site blocks per parity."""
    dims, tbc, kappa, csw = (8, 8, 8, 16), -1, 0.13, 1.5
    print(f"[gpu] solve rhs_block={R} prec={prec}", flush=True)
    U = inputs.gauge_field(dims, 0.35, 1)
    A = orc.clover(U, kappa, csw)
    eta = inputs.z2_noise(dims, 5, seed=6)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    ctx.set_option("rhs_block", R)
    try:
        X, info, rc = ctx.solve_propagators(c, eta, kappa, csw, tol=1e-10, prec=prec, max_iter=5000)
    finally:
        ctx.set_option("rhs_block", 4)
    assert rc == 0, info
    for i in range(5):
        r = eta[i] - orc.apply_D(U, A, kappa, X[i], tbc)
        assert np.linalg.norm(r) / np.linalg.norm(eta[i]) <= 1e-10
    ctx.unload(g)


def test_solve_zero_source_and_initial_guess(ctx, orc, tiny_ref):
    w, U, A, eta, Xo = tiny_ref
    print("[gpu] zero source / x0", flush=True)
    g = ctx.load_gauge(U, w["tbc"])
    c = ctx.load_clover(g, w["csw"])
    src = eta[:2].copy()
    src[1] = 0
    X, info, rc = ctx.solve_propagators(c, src, w["kappa"], w["csw"], tol=1e-10, prec=2)
    assert rc == 0
    assert np.all(X[1] == 0) and info[1]["converged"] == 1 and info[1]["true_rel_residual"] == 0.0
    # resume from the oracle solution: converges without iterating
    X2, info2, rc = ctx.solve_propagators(c, eta[:1], w["kappa"], w["csw"], tol=1e-10, prec=0, x0=Xo[:1])
    assert rc == 0 and info2[0]["iters"] == 0 and info2[0]["converged"] == 1
    ctx.unload(g)


def test_solve_errors(ctx, orc, tiny_ref):
    from paper_1405_4524_amd import a2a

    w, U, A, eta, Xo = tiny_ref
    print("[gpu] error paths", flush=True)
    g = ctx.load_gauge(U, w["tbc"])
    c = ctx.load_clover(g, w["csw"])
    with pytest.raises(a2a.A2AError) as e:
        ctx.solve_propagators(c, eta[:1], w["kappa"], w["csw"] + 0.1)
    assert e.value.code == a2a.EINVAL
    with pytest.raises(a2a.A2AError) as e:
        ctx.solve_propagators(c, eta[:1], -0.1, w["csw"])
    assert e.value.code == a2a.EINVAL
    with pytest.raises(a2a.A2AError) as e:
        ctx.solve_propagators(c + 100, eta[:1], w["kappa"], w["csw"])
    assert e.value.code == a2a.EHANDLE
    bad = eta[:1].copy()
    bad[0, 0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(a2a.A2AError) as e:
        ctx.solve_propagators(c, bad, w["kappa"], w["csw"])
    assert e.value.code == a2a.ENAN
    X, info, rc = ctx.solve_propagators(c, eta[:1], w["kappa"], w["csw"], tol=1e-10, prec=0, max_iter=3)
    assert rc == a2a.ENOTCONV and info[0]["converged"] == 0
    ctx.unload(g)


def test_single_hip_runtime_and_native_library_loaded(ctx):
    """The HIP library is what runs (no fallback), and torch and liba2a share one HIP runtime."""
    from paper_1405_4524_amd import a2a

    maps = open("/proc/self/maps").read()
    hip = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hip) == 1, hip
    assert a2a.LIB_PATH in maps


# ---------------------------------------------------------------------------------------
# contractions and noise
# ---------------------------------------------------------------------------------------
def test_noise_generator_bit_exact(ctx):
    import torch

    dims = (4, 2, 6, 4)
    want = inputs.z2_noise(dims, 3, seed=9, src_offset=5)
    out = torch.empty(want.shape + (2,), dtype=torch.float64, device="cuda")
    ctx.z2_noise_dev(dims, 9, 5, 3, out)
    got = out.cpu().numpy()
    assert np.array_equal(got[..., 0], want.real) and np.array_equal(got[..., 1], want.imag)


@pytest.mark.parametrize("dims,n", [((4, 4, 4, 8), 4), ((2, 4, 6, 4), 7), ((4, 4, 2, 6), 70)])
def test_contraction_pion(ctx, orc, dims, n):
    from paper_1405_4524_amd import a2a

    print(f"[gpu] pion contraction dims={dims} n={n}", flush=True)
    rng = np.random.default_rng(3)
    X, Y, Z, T = dims
    eta = inputs.z2_noise(dims, n, seed=12)
    sol = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
    Oo = orc.stochastic_operators(eta, sol)
    for mode in (a2a.PION_UNBIASED, a2a.PION_ALL_PAIRS):
        corr, O = ctx.contract_pion_2pt(eta, sol, mode=mode)
        assert rel(O, Oo) < 1e-12
        want = orc.pion_from_O(Oo, mode)
        assert rel(corr, want) < 1e-12


def test_contraction_pipi(ctx, orc):
    dims, n = (4, 2, 2, 6), 16
    print("[gpu] pipi contraction", flush=True)
    rng = np.random.default_rng(4)
    eta = inputs.z2_noise(dims, n, seed=13)
    sol = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
    d, v, pc = ctx.contract_pipi_2pt(eta, sol, want_pion=True)
    dw, vw = orc.contract_pipi(eta, sol)
    for k in range(4):
        assert rel(d[k], dw[k]) < 1e-11, k
    assert rel(v, vw) < 1e-12
    pw, _ = orc.contract_pion(eta, sol)
    assert rel(pc, pw) < 1e-12


def test_tiny_end_to_end_correlator(ctx, orc, tiny_ref):
    """tiny workload: GPU solve (FP64, tol 1e-12) + GPU contraction vs oracle solve + oracle
    contraction; correlator relative error <= 1e-9."""
    w, U, A, eta, Xo = tiny_ref
    g = ctx.load_gauge(U, w["tbc"])
    c = ctx.load_clover(g, w["csw"])
    X, info, rc = ctx.solve_propagators(c, eta, w["kappa"], w["csw"], tol=1e-12, prec=0)
    corr, _ = ctx.contract_pion_2pt(eta, X)
    want, _ = orc.contract_pion(eta, Xo)
    assert rel(corr, want) < 1e-9
    T = w["dims"][3]
    for dt in range(1, T):
        assert abs(corr[dt] - corr[T - dt]) < 1e-9 * abs(corr[0])
    ctx.unload(g)


def test_solve_more_sources_than_one_batch(ctx, orc):
    """2100 sources (more than the 2048 of one lock-step batch) on a 2^3x4 lattice: every source
    converges, every info record is filled, and sampled solutions from both batches meet the
    binding criterion with the oracle's D."""
    import torch

    from paper_1405_4524_amd import a2a

    print("[gpu] solve 2100 sources in two batches", flush=True)
    dims, tbc, kappa, csw, n = (2, 2, 2, 4), -1, 0.125, 1.2, 2100
    U, A = field(orc, dims, 0.4, 17, kappa, csw)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    src = torch.empty((n,) + tuple(reversed(dims)) + (4, 3, 2), dtype=torch.float64, device="cuda")
    ctx.z2_noise_dev(dims, 23, 0, n, src)
    sol = torch.zeros_like(src)
    info, rc = ctx.solve_propagators_dev(c, src, sol, n, kappa, csw, tol=1e-10, prec=a2a.F32)
    assert rc == 0 and len(info) == n
    assert all(x["converged"] == 1 and 0 < x["iters"] and x["true_rel_residual"] <= 1e-10 for x in info)
    for i in (0, 2047, 2048, n - 1):
        eta = inputs.z2_noise(dims, 1, 23, src_offset=i)[0]
        X = sol[i].cpu().numpy().view(np.complex128)[..., 0]
        r = np.linalg.norm(eta - orc.apply_D(U, A, kappa, X, tbc)) / np.linalg.norm(eta)
        assert r <= 1e-10, (i, r)
    ctx.unload(g)
