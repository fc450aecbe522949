"""GPU tests of batching and of the continuous-batching engine: results of each source are the
same alone, in a batch and in a mixed-lattice / mixed-kappa / mixed-precision stream, within
the solve tolerance (every one is also checked against the oracle's D)."""
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


LATS = [((4, 4, 4, 8), 0.35, 11), ((6, 4, 4, 10), 0.35, 12)]


@pytest.fixture(scope="module")
def fields(ctx, orc):
    out = []
    for dims, eps, seed in LATS:
        U = inputs.gauge_field(dims, eps, seed)
        g = ctx.load_gauge(U, -1)
        c = ctx.load_clover(g, 1.5)
        out.append(dict(dims=dims, U=U, g=g, c=c))
    return out


def test_batch_equals_alone(ctx, orc, fields):
    f = fields[0]
    print("[gpu] batch vs alone", flush=True)
    eta = inputs.z2_noise(f["dims"], 6, seed=21)
    Xb, infb, rc = ctx.solve_propagators(f["c"], eta, 0.125, 1.5, tol=1e-10, prec=2)
    assert rc == 0
    for i in (0, 3, 5):
        Xa, infa, rc = ctx.solve_propagators(f["c"], eta[i:i + 1], 0.125, 1.5, tol=1e-10, prec=2)
        assert rc == 0
        assert rel(Xa[0], Xb[i]) < 1e-8
    A = orc.clover(f["U"], 0.125, 1.5)
    for i in range(6):
        r = eta[i] - orc.apply_D(f["U"], A, 0.125, Xb[i], -1)
        assert np.linalg.norm(r) / np.linalg.norm(eta[i]) <= 1e-10


@pytest.mark.parametrize("prec,nsrc", [(2, 6), (2, 20), (3, 32), (1, 6)])
def test_autotune_config_solves(ctx, orc, fields, prec, nsrc):
    """The tuner picks a configuration of the path the solve runs (group width on the matrix
    cores for FP16 / BF16 with >= 12 sources, else the per-thread width; a brick tiling the
    lattice; the FP64 width), caches it, and a solve in that configuration meets 1e-10 with
    the oracle's D for every source."""
    f = fields[1]
    X_, Y_, Z_, T_ = f["dims"]
    print(f"[gpu] autotune prec={prec} nsrc={nsrc}", flush=True)
    r = ctx.autotune(f["c"], 0.125, prec, nsrc)
    assert r["candidates"] >= 3 and r["ms_schur"] > 0 and r["ms_schur64"] > 0
    by, bz, bt = r["brick"]
    assert Y_ % by == 0 and Z_ % bz == 0 and T_ % bt == 0
    assert r["rhs_block64"] in (1, 2)
    if prec in (2, 3) and nsrc >= 12:
        assert r["il_width"] in (16, 32, 48) and r["xcd_slab"] in (0, 1)
    else:
        assert r["il_width"] == 0 and r["rhs_block"] in (1, 2, 4) and r["xcd_slab"] == -1
    again = ctx.autotune(f["c"], 0.125, prec, nsrc)
    assert again["candidates"] == 0 and again["brick"] == r["brick"] and again["il_width"] == r["il_width"]
    ctx.set_option("autotune", 1)
    try:
        eta = inputs.z2_noise(f["dims"], nsrc, seed=31)
        X, info, rc = ctx.solve_propagators(f["c"], eta, 0.125, 1.5, tol=1e-10, prec=prec)
    finally:
        ctx.set_option("autotune", 0)
    assert rc == 0
    A = orc.clover(f["U"], 0.125, 1.5)
    for i in range(nsrc):
        res = eta[i] - orc.apply_D(f["U"], A, 0.125, X[i], -1)
        assert np.linalg.norm(res) / np.linalg.norm(eta[i]) <= 1e-10, (i, info[i])


def test_tuned_bricks_give_the_same_operator(ctx, orc, fields):
    """Every brick and block order the tuner may choose reorders the sweep only: the Schur
    operator is bitwise the same in FP64 (per-thread stencil) and in FP16 on the matrix cores
    (20 sources in one lane-interleaved group), and matches the oracle."""
    from paper_1405_4524_amd import a2a

    f = fields[1]
    print("[gpu] bricks", flush=True)
    rng = np.random.default_rng(9)
    shp = (20,) + tuple(f["dims"][::-1]) + (4, 3)
    psi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    A = orc.clover(f["U"], 0.125, 1.5)
    odd = (orc.parity_mask(f["dims"]) == 1)[..., None, None]
    want = orc.schur(f["U"], A, orc.invert_sites(A), 0.125, np.where(odd, psi[0], 0), -1)
    for prec, tol in ((a2a.F64, 1e-13), (a2a.F16_F32, 4e-3)):
        ref = ctx.dslash_clover(f["c"], 0.125, psi, op=a2a.OP_SCHUR, prec=prec)
        assert rel(ref[0], want) <= tol, (prec, rel(ref[0], want))
        for b in ctx.brick_choices(f["dims"]):
            for slab in (0, 1):
                ctx.set_option("brick", b[0] * 10000 + b[1] * 100 + b[2])
                ctx.set_option("mfma_slab", slab)
                try:
                    out = ctx.dslash_clover(f["c"], 0.125, psi, op=a2a.OP_SCHUR, prec=prec)
                finally:
                    ctx.set_option("brick", 0)
                    ctx.set_option("mfma_slab", 0)
                assert np.array_equal(out, ref), (prec, b, slab)


@pytest.mark.parametrize("il", [0, 1])
def test_engine_mixed_stream_matches_alone(ctx, orc, fields, il):
    ctx.set_option("interleave", il)
    try:
        _engine_mixed_stream(ctx, orc, fields)
    finally:
        ctx.set_option("interleave", 1)


def _engine_mixed_stream(ctx, orc, fields):
    import torch

    print("[gpu] engine mixed stream", flush=True)
    eng = ctx.engine_create('{"max_slots": 24, "check_every": 4}')
    reqs = []
    rng = np.random.default_rng(5)
    for k in range(7):
        f = fields[k % 2]
        kappa = float(rng.uniform(0.120, 0.130))
        nsrc = 20 if k in (1, 4) else int(rng.integers(1, 6))  # 20: a 16-lane group + 4 per slot
        prec = [2, 1, 3, 0][k % 4]
        eta = inputs.z2_noise(f["dims"], nsrc, seed=100 + k)
        src = torch.from_numpy(eta).cuda()
        sol = torch.zeros_like(src)
        reqs.append(dict(f=f, kappa=kappa, nsrc=nsrc, prec=prec, eta=eta, src=src, sol=sol, ticket=None))
    # staggered arrivals: two at first, then one more per step
    pending = list(reqs)
    for r in pending[:2]:
        r["ticket"] = eng.submit(r["f"]["c"], r["kappa"], r["src"], r["nsrc"], 1e-10, r["prec"], 20000, r["sol"])
    pending = pending[2:]
    for step in range(2000):
        if pending:
            r = pending.pop(0)
            r["ticket"] = eng.submit(r["f"]["c"], r["kappa"], r["src"], r["nsrc"], 1e-10, r["prec"], 20000, r["sol"])
        eng.step(8)
        if not pending and all(eng.poll(r["ticket"], r["nsrc"])[0] != 0 for r in reqs):
            break
    for r in reqs:
        done, info, rc = eng.poll(r["ticket"], r["nsrc"])
        assert done == 1 and rc == 0, (done, rc, info)
        X = r["sol"].cpu().numpy()
        A = orc.clover(r["f"]["U"], r["kappa"], 1.5)
        for i in range(r["nsrc"]):
            res = np.linalg.norm(r["eta"][i] - orc.apply_D(r["f"]["U"], A, r["kappa"], X[i], -1))
            assert res / np.linalg.norm(r["eta"][i]) <= 1e-10
            assert info[i]["converged"] == 1
        Xa, _, rc = ctx.solve_propagators(r["f"]["c"], r["eta"], r["kappa"], 1.5, tol=1e-10, prec=r["prec"])
        assert rel(X, Xa) < 1e-8
    eng.destroy()


def test_engine_admission_by_budget_and_cancel(orc, fields):
    """A context whose HBM budget fits one request at a time still serves all of them, one
    after another; a cancelled queued request is reported failed and never runs."""
    import torch

    from paper_1405_4524_amd import a2a

    print("[gpu] engine budget admission", flush=True)
    f = fields[0]
    dims = f["dims"]
    c2 = a2a.Context(0)
    try:
        g = c2.load_gauge(f["U"], -1)
        cl = c2.load_clover(g, 1.5)
        warm = inputs.z2_noise(dims, 1, seed=299)
        c2.dslash_clover(cl, 0.124, warm, prec=a2a.F32)  # builds the FP32 fields of this kappa
        hv = int(np.prod(dims)) // 2
        r256 = lambda b: (b + 255) // 256 * 256
        per_req = 12 * (8 * r256(hv * 24 * 4) + 7 * r256(hv * 24 * 8))
        c2.set_option("hbm_budget", c2.mem_in_use() + int(1.6 * per_req) + (256 << 10))
        eng = c2.engine_create('{"max_slots": 64}')
        tickets = []
        sols = []
        etas = []
        for k in range(3):
            eta = inputs.z2_noise(dims, 12, seed=300 + k)
            src = torch.from_numpy(eta).cuda()
            sol = torch.zeros_like(src)
            etas.append(eta)
            sols.append((src, sol))
            tickets.append(eng.submit(cl, 0.124, src, 12, 1e-10, 1, 20000, sol))
        eng.cancel(tickets[2])
        max_active = 0
        for _ in range(3000):
            act = eng.step(8)
            max_active = max(max_active, act)
            states = [eng.poll(t, 12)[0] for t in tickets[:2]]
            if all(s != 0 for s in states):
                break
        assert [eng.poll(t, 12)[0] for t in tickets] == [1, 1, -1]
        assert max_active == 12  # the budget admitted one request at a time
        A = orc.clover(f["U"], 0.124, 1.5)
        for k in range(2):
            X = sols[k][1].cpu().numpy()
            for i in range(12):
                r = etas[k][i] - orc.apply_D(f["U"], A, 0.124, X[i], -1)
                assert np.linalg.norm(r) / np.linalg.norm(etas[k][i]) <= 1e-10
        eng.destroy()
    finally:
        c2.finalize()


def test_engine_failed_admission_is_undone(ctx, orc, fields):
    """A request whose source preparation fails after its slots were allocated gives the slots,
    their ids and their memory back.  An out-of-memory failure while another request runs leaves
    it queued, and a later step admits it afresh; a device error fails that request alone.  The
    requests converge to their solutions alone, the engine's active count returns to zero and
    the context's live memory to its value before the engine was created.  The test has a
    context of its own, so that no clover fields of other kappas are left for an out-of-memory
    admission to evict (which would lower the live memory legitimately)."""
    from paper_1405_4524_amd import a2a

    print("[gpu] engine: failed admissions are undone", flush=True)
    f = dict(fields[0])
    cx = a2a.Context(0)
    try:
        _failed_admission_body(cx, orc, f, cx.load_clover(cx.load_gauge(f["U"], -1), 1.5))
    finally:
        cx.finalize()


def _failed_admission_body(ctx, orc, f, clover):
    import torch

    from paper_1405_4524_amd import a2a

    f["c"] = clover
    kappa = 0.127
    sizes = (5, 7, 4)
    etas = [inputs.z2_noise(f["dims"], n, seed=600 + k) for k, n in enumerate(sizes)]
    alone = []
    for eta in etas[:2]:
        Xa, _, rc = ctx.solve_propagators(f["c"], eta, kappa, 1.5, tol=1e-10, prec=a2a.F16_F32)
        assert rc == 0
        alone.append(Xa)
    # every sid the engine will hold at once was in use above: nothing context-wide grows
    ctx.solve_propagators(f["c"], np.concatenate(etas), kappa, 1.5, tol=1e-10, prec=a2a.F16_F32)
    mem0 = ctx.mem_in_use()
    eng = ctx.engine_create('{"max_slots": 64}')
    dev = []
    for e in etas:
        src = torch.from_numpy(e).cuda()
        dev.append((src, torch.zeros_like(src)))
    submit = lambda k: eng.submit(f["c"], kappa, dev[k][0], sizes[k], 1e-10, a2a.F16_F32, 20000, dev[k][1])
    tA = submit(0)
    assert eng.step(1) == sizes[0]
    ctx.set_option("fail_setup_enomem", 2)  # fails the first admission and an immediate retry
    tB = submit(1)
    admitted = False
    for _ in range(4):
        act = eng.step(1)
        assert eng.poll(tB, sizes[1])[0] != -1
        assert act in (sizes[0], sizes[0] + sizes[1]), act
        if act == sizes[0] + sizes[1]:
            admitted = True
            break
    assert admitted
    ctx.set_option("fail_setup_device", 1)
    tC = submit(2)
    act = eng.step(1)
    done, _, rc = eng.poll(tC, sizes[2])
    assert done == -1 and rc == a2a.EDEVICE, (done, rc)
    assert act == sizes[0] + sizes[1]
    for _ in range(3000):
        act = eng.step(8)
        if act == 0:
            break
    assert act == 0
    A = orc.clover(f["U"], kappa, 1.5)
    for k, t in enumerate((tA, tB)):
        done, info, rc = eng.poll(t, sizes[k])
        assert done == 1 and rc == 0, (k, done, rc)
        X = dev[k][1].cpu().numpy()
        for i in range(sizes[k]):
            r = etas[k][i] - orc.apply_D(f["U"], A, kappa, X[i], -1)
            assert np.linalg.norm(r) / np.linalg.norm(etas[k][i]) <= 1e-10
        assert rel(X, alone[k]) < 1e-8
    eng.destroy()
    assert ctx.mem_in_use() == mem0


@pytest.mark.parametrize("prec", [0, 2])
def test_repeat_solve_on_recycled_memory_is_bitwise_identical(ctx, orc, fields, prec):
    """The context hands freed device buffers to later allocations of the same size: solves
    and engine requests that run on recycled buffers (holding whatever the previous user left,
    with other-sized work in between) give bitwise the same solutions, iteration counts and
    residuals as the first solve on fresh memory."""
    import torch

    print(f"[gpu] repeat solve on recycled memory prec={prec}", flush=True)
    f = fields[0]
    eta = inputs.z2_noise(f["dims"], 20, seed=410)
    X0, info0, rc = ctx.solve_propagators(f["c"], eta, 0.124, 1.5, tol=1e-10, prec=prec)
    assert rc == 0
    other = inputs.z2_noise(f["dims"], 7, seed=411)  # different sizes in between
    ctx.solve_propagators(f["c"], other, 0.126, 1.5, tol=1e-10, prec=1)
    for _ in range(2):
        X1, info1, rc = ctx.solve_propagators(f["c"], eta, 0.124, 1.5, tol=1e-10, prec=prec)
        assert rc == 0
        assert np.array_equal(X1, X0)
        assert [x["iters"] for x in info1] == [x["iters"] for x in info0]
        assert [x["true_rel_residual"] for x in info1] == [x["true_rel_residual"] for x in info0]
    runs = []
    for k in range(2):  # the same request twice, a differently sized one in between
        eng = ctx.engine_create('{"max_slots": 64}')
        src = torch.from_numpy(eta).cuda()
        sol = torch.zeros_like(src)
        t = eng.submit(f["c"], 0.124, src, 20, 1e-10, prec, 20000, sol)
        for _ in range(3000):
            eng.step(4)
            if eng.poll(t, 20)[0] != 0:
                break
        done, info, rc = eng.poll(t, 20)
        assert done == 1 and rc == 0
        runs.append((sol.cpu().numpy(), [x["iters"] for x in info]))
        eng.destroy()
        ctx.solve_propagators(f["c"], other[:3], 0.126, 1.5, tol=1e-10, prec=1)
    assert np.array_equal(runs[0][0], runs[1][0]) and runs[0][1] == runs[1][1]


@pytest.mark.parametrize("prec", [2, 0])
def test_no_result_depends_on_unwritten_memory(orc, fields, prec):
    """With every buffer the context allocates or reuses filled with NaN bytes (option
    poison_memory), solves in interleaved groups with an idle lane (47 = 16 + 16 + 15 sources),
    a per-slot solve on reused buffers, CGNR, an engine request and the contractions give
    bitwise the results of a context without the poison: no kernel lets memory it did not
    write reach a result (an idle lane's 0 * NaN once reached the reductions of its column)."""
    import torch

    from paper_1405_4524_amd import a2a

    print(f"[gpu] poisoned memory prec={prec}", flush=True)
    f = fields[0]
    eta = inputs.z2_noise(f["dims"], 47, seed=420)
    res = []
    for poison in (0, 1):
        c2 = a2a.Context(0)
        try:
            c2.set_option("poison_memory", poison)
            g = c2.load_gauge(f["U"], -1)
            cl = c2.load_clover(g, 1.5)
            out = []
            for n, solver in ((47, a2a.SOLVER_BICGSTAB), (5, a2a.SOLVER_BICGSTAB), (20, a2a.SOLVER_CGNR)):
                c2.set_option("solver", solver)
                X, info, rc = c2.solve_propagators(cl, eta[:n], 0.124, 1.5, tol=1e-10, prec=prec, max_iter=20000)
                assert rc == 0 and all(x["converged"] == 1 for x in info)
                out += [X, np.array([x["iters"] for x in info])]
            c2.set_option("solver", a2a.SOLVER_BICGSTAB)
            eng = c2.engine_create('{"max_slots": 64}')
            src = torch.from_numpy(eta[:31]).cuda()
            sol = torch.zeros_like(src)
            t = eng.submit(cl, 0.123, src, 31, 1e-10, prec, 20000, sol)
            for _ in range(3000):
                eng.step(4)
                if eng.poll(t, 31)[0] != 0:
                    break
            assert eng.poll(t, 31)[0] == 1
            eng.destroy()
            out.append(sol.cpu().numpy())
            X = out[0]
            corr, O = c2.contract_pion_2pt(eta, X)
            d, v = c2.contract_pipi_2pt(eta[:16], X[:16])
            out += [corr, O, d, v]
            res.append(out)
        finally:
            c2.finalize()
    for k, (a, b) in enumerate(zip(*res)):
        assert np.array_equal(a, b), k


def test_trim_returns_cached_buffers(ctx, orc, fields):
    """a2a_trim hands the freed buffers kept for reuse back to the device: after a solve it
    releases some bytes, right after that none, live memory is untouched, and the next solve
    (on fresh buffers) gives bitwise the same solutions."""
    print("[gpu] trim", flush=True)
    f = fields[0]
    eta = inputs.z2_noise(f["dims"], 6, seed=430)
    X0, _, rc = ctx.solve_propagators(f["c"], eta, 0.124, 1.5, tol=1e-10, prec=2)
    assert rc == 0
    live = ctx.mem_in_use()
    assert ctx.trim() > 0
    assert ctx.trim() == 0
    assert ctx.mem_in_use() == live
    X1, _, rc = ctx.solve_propagators(f["c"], eta, 0.124, 1.5, tol=1e-10, prec=2)
    assert rc == 0 and np.array_equal(X0, X1)


def test_failures_do_not_affect_co_scheduled_work(ctx, orc, fields):
    """A request with a non-finite source fails with A2A_ENAN and one whose max_iter is too small
    with A2A_ENOTCONV, while the requests that share the engine with them (the same lattice and
    another one, two precisions) converge to their solutions alone; in one solve call the good
    sources of a batch that holds a non-finite source still converge."""
    import torch

    from paper_1405_4524_amd import a2a

    print("[gpu] failure isolation", flush=True)
    f0, f1 = fields
    eta0 = inputs.z2_noise(f0["dims"], 8, seed=440)
    eta1 = inputs.z2_noise(f1["dims"], 5, seed=441)
    bad = eta0[:3].copy()
    bad[1, 0, 0, 0, 0, 0, 0] = np.nan
    eng = ctx.engine_create('{"max_slots": 64}')
    jobs = [("good0", f0, eta0, 2, 20000), ("nan", f0, bad, 2, 20000), ("good1", f1, eta1, 1, 20000),
            ("short", f0, eta0[:2], 2, 3)]
    subs = {}
    for name, f, eta, prec, maxit in jobs:
        src = torch.from_numpy(eta).cuda()
        sol = torch.zeros_like(src)
        subs[name] = (eng.submit(f["c"], 0.124, src, len(eta), 1e-10, prec, maxit, sol), len(eta), src, sol)
    for _ in range(3000):
        eng.step(4)
        if all(eng.poll(t, n)[0] != 0 for t, n, _, _ in subs.values()):
            break
    res = {k: eng.poll(t, n) for k, (t, n, _, _) in subs.items()}
    assert res["nan"][0] == -1 and res["nan"][2] == a2a.ENAN
    assert res["short"][0] == -1 and res["short"][2] == a2a.ENOTCONV
    for name, f, eta, prec in (("good0", f0, eta0, 2), ("good1", f1, eta1, 1)):
        done, info, rc = res[name]
        assert done == 1 and rc == 0 and all(x["converged"] == 1 for x in info), name
        X = subs[name][3].cpu().numpy()
        Xa, _, rc = ctx.solve_propagators(f["c"], eta, 0.124, 1.5, tol=1e-10, prec=prec)
        assert rc == 0 and rel(X, Xa) < 1e-8, name
    eng.destroy()
    mixed = np.stack([eta0[0], bad[1], eta0[2]])
    # the host-pointer call validates its input first and rejects it whole
    with pytest.raises(a2a.A2AError) as e:
        ctx.solve_propagators(f0["c"], mixed, 0.124, 1.5, tol=1e-10, prec=2)
    assert e.value.code == a2a.ENAN
    # the device-pointer call fails the non-finite source only
    src = torch.from_numpy(mixed).cuda()
    sol = torch.zeros_like(src)
    info, rc = ctx.solve_propagators_dev(f0["c"], src, sol, 3, 0.124, 1.5, tol=1e-10, prec=2, allow=(a2a.ENAN,))
    assert rc == a2a.ENAN
    assert info[0]["converged"] == 1 and info[2]["converged"] == 1 and info[1]["converged"] == 0
    X = sol.cpu().numpy()  # a complex tensor: from_numpy keeps the complex dtype
    A = orc.clover(f0["U"], 0.124, 1.5)
    for i in (0, 2):
        r = mixed[i] - orc.apply_D(f0["U"], A, 0.124, X[i], -1)
        assert np.linalg.norm(r) / np.linalg.norm(mixed[i]) <= 1e-10


@pytest.mark.parametrize("prec,nsrc", [(2, 20), (2, 5), (3, 16), (1, 4)])
def test_reliable_update_correction_form(ctx, orc, fields, prec, nsrc):
    """Reliable updates in correction form (r64 -= M (sigma x_lo) from the stored low-precision
    correction, FP64 arithmetic; the default) and recomputed from the FP64 iterate (r64 = b -
    M x64) both solve to 1e-10 with the oracle's D, with agreeing solutions (FP16 in a lane-
    interleaved group and per slot, BF16, FP32)."""
    from paper_1405_4524_amd import a2a

    f = fields[1]
    print(f"[gpu] reliable-update forms prec={prec} nsrc={nsrc}", flush=True)
    eta = inputs.z2_noise(f["dims"], nsrc, seed=71)
    A = orc.clover(f["U"], 0.126, 1.5)
    out = {}
    for form in (1, 0):
        ctx.set_option("ru_correction", form)
        try:
            X, info, rc = ctx.solve_propagators(f["c"], eta, 0.126, 1.5, tol=1e-10, prec=prec)
        finally:
            ctx.set_option("ru_correction", 1)
        assert rc == 0
        assert all(x["reliable_updates"] >= 1 for x in info)
        for i in range(nsrc):
            res = eta[i] - orc.apply_D(f["U"], A, 0.126, X[i], -1)
            r = np.linalg.norm(res) / np.linalg.norm(eta[i])
            assert r <= 1e-10, (form, i, r)
            assert abs(r - info[i]["true_rel_residual"]) < 1e-13, (form, i, r, info[i])
        out[form] = X
    assert rel(out[1], out[0]) < 1e-8


def test_upload_staging_paths_are_bitwise(ctx, orc, fields):
    """Device tables uploaded through a tiny pinned staging buffer (uploads above a quarter of it
    take the waiting copy, the others fill it and force a synchronisation before reuse) give
    bitwise the solutions, residuals and iteration counts of the default staging."""
    f = fields[1]
    print("[gpu] upload staging paths", flush=True)
    eta = inputs.z2_noise(f["dims"], 20, seed=97)
    out = []
    for size in (0, 4096):
        ctx.set_option("upload_stage_bytes", size)
        try:
            X, info, rc = ctx.solve_propagators(f["c"], eta, 0.126, 1.5, tol=1e-10, prec=2)
        finally:
            ctx.set_option("upload_stage_bytes", 0)
        assert rc == 0
        out.append((X, [x["true_rel_residual"] for x in info], [x["iters"] for x in info]))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
    A = orc.clover(f["U"], 0.126, 1.5)
    res = eta[0] - orc.apply_D(f["U"], A, 0.126, out[1][0][0], -1)
    assert np.linalg.norm(res) / np.linalg.norm(eta[0]) <= 1e-10


@pytest.mark.parametrize("prec,nsrc", [(2, 20), (2, 5), (3, 16), (1, 4)])
def test_symmetric_schur_form(ctx, orc, fields, prec, nsrc):
    """BiCGStab on the symmetric Schur form (the default; FP16 in a lane-interleaved group on the
    matrix cores and per slot, BF16, FP32) and on the asymmetric form both solve to 1e-10 with
    the oracle's D, with agreeing solutions."""
    f = fields[1]
    print(f"[gpu] Schur forms prec={prec} nsrc={nsrc}", flush=True)
    eta = inputs.z2_noise(f["dims"], nsrc, seed=81)
    A = orc.clover(f["U"], 0.127, 1.5)
    out = {}
    for form in (1, 0):
        ctx.set_option("schur_sym", form)
        try:
            X, info, rc = ctx.solve_propagators(f["c"], eta, 0.127, 1.5, tol=1e-10, prec=prec)
        finally:
            ctx.set_option("schur_sym", 1)
        assert rc == 0
        for i in range(nsrc):
            res = eta[i] - orc.apply_D(f["U"], A, 0.127, X[i], -1)
            r = np.linalg.norm(res) / np.linalg.norm(eta[i])
            assert r <= 1e-10, (form, i, r)
            assert abs(r - info[i]["true_rel_residual"]) < 1e-13, (form, i, r, info[i])
        out[form] = X
    assert rel(out[1], out[0]) < 1e-8
