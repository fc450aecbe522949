"""GPU tests of the lane-interleaved inner layout (FP16 / BF16 storage): slots of one call form
groups of up to 48 lanes (tiles of 16; a remainder below 12 sources stays per slot) sharing one
arena, and the stencil runs on the matrix cores.  The operators must match the oracle to the low-precision operator tolerances (with the
matrix-core stencil and with the per-thread stencil on the same layout), a RHS must give the
same operator output whatever group it sits in, and solves must meet the binding criterion with
the oracle's D and agree with the per-slot layout's solutions (both solved to 1e-10;
cond(D) ~ 10-100 bounds the difference by ~1e-8)."""
import numpy as np
import pytest

from paper_1405_4524_amd import inputs

pytestmark = pytest.mark.gpu

OP_TOL = {2: 4e-3, 3: 3e-2}


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.fixture(scope="module")
def ctx():
    from paper_1405_4524_amd import a2a

    c = a2a.Context(0)
    yield c
    c.finalize()


class interleaved:
    def __init__(self, ctx, on=1):
        self.ctx, self.on = ctx, on

    def __enter__(self):
        self.ctx.set_option("interleave", self.on)

    def __exit__(self, *exc):
        self.ctx.set_option("interleave", 1)


@pytest.mark.parametrize("mfma", [1, 0])
@pytest.mark.parametrize("prec", [2, 3])
def test_interleaved_operators(ctx, orc, prec, mfma):
    from paper_1405_4524_amd import a2a

    dims, tbc, kappa, csw = (6, 4, 4, 10), -1, 0.125, 1.2
    print(f"[gpu] interleaved operators prec={prec} mfma={mfma}", flush=True)
    ctx.set_option("mfma", mfma)
    U = inputs.gauge_field(dims, 0.35, 7)
    A = orc.clover(U, kappa, csw)
    Ai = orc.invert_sites(A)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    n = 28  # two lane tiles, the second with 12 lanes
    psi = inputs.z2_noise(dims, n, seed=13)
    odd = (orc.parity_mask(dims) == 1)[..., None, None]
    g5 = np.array([1, 1, -1, -1])[:, None]
    with interleaved(ctx):
        for op in (a2a.OP_FULL_D, a2a.OP_SCHUR, a2a.OP_HOP_EO, a2a.OP_HOP_OE):
            for dag in (False, True):
                got = ctx.dslash_clover(c, kappa, psi, op=op, dagger=dag, prec=prec)
                for i in (0, 5, 15, 16, 27):
                    x = g5 * psi[i] if dag else psi[i]
                    if op == a2a.OP_FULL_D:
                        want = orc.apply_D(U, A, kappa, x, tbc)
                    elif op == a2a.OP_SCHUR:
                        want = orc.schur(U, A, Ai, kappa, np.where(odd, x, 0), tbc)
                    elif op == a2a.OP_HOP_EO:
                        want = np.where(odd, 0, orc.hop(U, np.where(odd, x, 0), tbc))
                    else:
                        want = np.where(odd, orc.hop(U, np.where(odd, 0, x), tbc), 0)
                    if dag:
                        want = g5 * want
                    assert rel(got[i], want) < OP_TOL[prec], (op, dag, i, rel(got[i], want))
            # a RHS gives the same output in any lane of any group: lane 27 (tile 1 of a
            # 28-lane group) against lane 0 of a 16-lane group
            other = np.concatenate([psi[27:28], psi[:15]])
            assert np.array_equal(ctx.dslash_clover(c, kappa, other, op=op, prec=prec)[0],
                                  ctx.dslash_clover(c, kappa, psi, op=op, prec=prec)[27])
    ctx.set_option("mfma", 1)
    ctx.unload(g)


@pytest.mark.parametrize("prec", [2, 3])
def test_interleaved_solve(ctx, orc, prec):
    """70 sources: one full 48-lane group, one 16-lane group, and 6 sources in per-slot arenas
    (a remainder below 12 lanes stays per slot) in the same solve."""
    dims, tbc, kappa, csw = (4, 4, 4, 8), -1, 0.125, 1.5
    print(f"[gpu] interleaved solve prec={prec}", flush=True)
    U = inputs.gauge_field(dims, 0.35, 3)
    A = orc.clover(U, kappa, csw)
    eta = inputs.z2_noise(dims, 70, seed=17)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    with interleaved(ctx):
        X, info, rc = ctx.solve_propagators(c, eta, kappa, csw, tol=1e-10, prec=prec, max_iter=5000)
    assert rc == 0, [x for x in info if not x["converged"]][:3]
    with interleaved(ctx, 0):
        Xp, _, rc = ctx.solve_propagators(c, eta, kappa, csw, tol=1e-10, prec=prec, max_iter=5000)
    assert rc == 0
    for i in range(70):
        r = eta[i] - orc.apply_D(U, A, kappa, X[i], tbc)
        assert np.linalg.norm(r) / np.linalg.norm(eta[i]) <= 1e-10, i
        assert rel(X[i], Xp[i]) < 1e-8, i
    ctx.unload(g)


def test_interleaved_solve_larger_lattice(ctx, orc):
    """Several site blocks per parity (8^3x16: 16 blocks of 256), a 32-lane group and 8
    sources per slot."""
    dims, tbc, kappa, csw = (8, 8, 8, 16), -1, 0.13, 1.5
    print("[gpu] interleaved solve 8^3x16", flush=True)
    U = inputs.gauge_field(dims, 0.35, 1)
    A = orc.clover(U, kappa, csw)
    eta = inputs.z2_noise(dims, 40, seed=6)
    g = ctx.load_gauge(U, tbc)
    c = ctx.load_clover(g, csw)
    with interleaved(ctx):
        X, info, rc = ctx.solve_propagators(c, eta, kappa, csw, tol=1e-10, prec=2, max_iter=5000)
    assert rc == 0
    for i in range(0, 40, 3):
        r = eta[i] - orc.apply_D(U, A, kappa, X[i], tbc)
        assert np.linalg.norm(r) / np.linalg.norm(eta[i]) <= 1e-10, i
    ctx.unload(g)
