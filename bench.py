#!/usr/bin/env python3
"""Benchmark: solved RHS/s of the stochastic-propagator solve, and the stencil's HBM roofline.

One step is one pass of the whole hot path over one batch of synthetic input resident in HBM:
  gauge ingest (canonical FP64 links -> even-odd fields), clover build, per-kappa clover and
  inverse, even-odd source preparation, batched mixed-precision BiCGStab with FP64 reliable
  updates for every noise source to ||eta - D X|| <= 1e-10 ||eta||, reconstruction and FP64
  true residual, the stochastic-operator contraction, the pion and the pi-pi correlators.
value = sources solved per second over the timed steps (whole job, one GPU).

Beside it: the same solve in plain FP64 (FP64 storage and arithmetic, one source at a time)
and FP64 batched (all sources in one call), the stencil alone in GB/s, the roofline of the
dominant kernel measured with HIP events over the timed region, and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload l32t64] [--prec f16] [--no-cpu]

Studies (each prints its own JSON line): --serve (continuous batching under Poisson load),
--mixed (three lattices in one batch), --stencil-only, --fill (outer-product fill against the
Gram route), --dilution, --noise-study, --point-study, --ensemble N, --solver cgnr.
"""
import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash HBM GB/s; solved RHS/s at rel. residual 1e-10 (mixed+batched vs FP64)"
HBM_PEAK_GBS = 8000.0
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
STORAGE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}


# HBM bytes per launch of the dominant stencil from two rocprofv3 counter passes (FETCH_SIZE,
# WRITE_SIZE; KiB per dispatch), scaled by what the same counters read for a plain 1 GiB device
# copy (fetch x2.0, write x1.0). Valid only for the kernel sources they were taken on (hash of the
# stencil's sources) and for the same workload, precision, layout and kernel class.
TRAFFIC = {
    ("schur2", "l32t64", "f16", "il"): {"src": "8b0e066ee05a6155", "bytes": 1.5795e10,
                                        "profile": "profiles/bench_l32t64_f16_hbm_counters.txt"},
}
STENCIL_SOURCES = {"per-thread": ("hop.hip", "a2a_device.h", "a2a_reduce.h", "a2a_kernels.h"),
                   "mfma": ("hop_mfma.hip", "a2a_device.h", "a2a_reduce.h", "a2a_kernels.h")}


def stencil_src_hash(kind):
    import hashlib

    h = hashlib.sha256()
    for f in STENCIL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1405_4524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="l32t64")
    ap.add_argument("--prec", default="f16", choices=list(PREC))
    ap.add_argument("--rhs-block", type=int, default=2, help="per-thread RHS width when not autotuned")
    ap.add_argument("--rhs-block64", type=int, default=2,
                    help="FP64-stencil RHS width when not autotuned (1 or 2)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: tune the launch configuration (group width, brick, FP64 width) before the warmup")
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--interleave", type=int, default=1,
                    help="1: FP16/BF16 inner vectors in lane-interleaved groups (matrix-core stencil)")
    ap.add_argument("--mfma", type=int, default=1, help="0: interleaved groups use the per-thread stencil")
    ap.add_argument("--delta", type=float, default=0.03, help="reliable-update reduction factor")
    ap.add_argument("--delta-bf16", type=float, default=0.05, help="the same for BF16 storage")
    ap.add_argument("--target-frac", type=float, default=0.8,
                    help="Schur-residual target as a fraction of tol ||eta|| (the full residual decides)")
    ap.add_argument("--tail-checks", type=int, default=1, help="1: residual checks after every iteration in the tail")
    ap.add_argument("--schur-sym", type=int, default=1, help="1: BiCGStab on the symmetric Schur form")
    ap.add_argument("--ru-correction", type=int, default=1,
                    help="1: reliable updates as r64 -= M (sigma x_lo); 0: r64 = b - M x64 recomputed")
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "cgnr"],
                    help="inner Krylov method (cgnr: CG on the normal equations)")
    ap.add_argument("--fp64-sources", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and stencil side measurements")
    ap.add_argument("--stencil-only", action="store_true",
                    help="time only the one-parity hopping stencil and a plain copy (for counter runs)")
    ap.add_argument("--stencil-reps", type=int, default=20)
    ap.add_argument("--copy-calib", action="store_true",
                    help="after the timed steps, copy 1 GiB on the device (calibrates counter runs)")
    ap.add_argument("--serve", action="store_true",
                    help="serving run: Poisson request streams on resident 8^3x16, 16^3x32, 24^3x48 fields")
    ap.add_argument("--serve-rates", default="1,2,5,10,20,50")
    ap.add_argument("--serve-requests", type=int, default=40)
    ap.add_argument("--serve-policy", default='{"max_slots": 256, "check_every": 4}', help="engine policy JSON")
    ap.add_argument("--serve-step", type=int, default=4, help="solver iterations per engine step")
    ap.add_argument("--serve-cap", type=int, default=384,
                    help="RHS submitted to the engine at most at once; later arrivals wait on the client side")
    ap.add_argument("--mixed", action="store_true",
                    help="mixed-lattice batch: 8^3x16, 16^3x32, 24^3x48 with 8-32 sources each in one batch")
    ap.add_argument("--fill", action="store_true",
                    help="outer-product fill of the all-to-all propagator against the Gram-matrix route, "
                         "L^3 x 2L lattices, and the fill kernel's matrix-core roofline")
    ap.add_argument("--fill-sizes", default="4,6,8,10,12")
    ap.add_argument("--dilution", action="store_true",
                    help="time-spin-colour dilution against undiluted noise at the same number of solves, "
                         "with momentum-projected pion correlators (8^3x16)")
    ap.add_argument("--dil-noise", type=int, default=4, help="noise vectors of the diluted set")
    ap.add_argument("--noise-study", action="store_true",
                    help="one noise set for both propagators against two independent sets (4^3x8), "
                         "against the exact all-to-all from full dilution")
    ap.add_argument("--noise-counts", default="16,64,256,1024")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="pi-pi diagrams with vacuum subtraction over this many synthetic 8^3x16 configurations")
    ap.add_argument("--fill-sources", default="16,64,256,1024")
    ap.add_argument("--cpu-study", action="store_true",
                    help="the CPU oracle alone: FP64 hop GB/s at three shapes and full solves, all cores and one")
    ap.add_argument("--cpu-study-sources", type=int, default=4, help="16^3x32 sources solved on all cores")
    ap.add_argument("--serve-leg", default="5,20",
                    help="offered rates of the short serving leg of the default run ('' to skip)")
    ap.add_argument("--serve-leg-requests", type=int, default=40)
    ap.add_argument("--source-errors", default="",
                    help="workload whose every source is solved on the GPU (FP16 and BF16 inner) and by the oracle "
                         "(FP64, tol 1e-12 on the host): per-source propagator error and residual")
    ap.add_argument("--point-study", action="store_true",
                    help="pi-pi diagrams from point and stochastic propagators (4^3x8) against the exact "
                         "diagrams from full dilution, one noise set against two")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.cpu_study:
        cpu_study(args)
        return

    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a, inputs

    if args.serve or args.mixed:
        print(json.dumps(serve_or_mixed(args)), flush=True)
        return
    if args.fill:
        fill_study(args)
        return
    if args.dilution:
        dilution_study(args)
        return
    if args.noise_study:
        noise_study(args)
        return
    if args.ensemble:
        ensemble_study(args)
        return
    if args.point_study:
        point_study(args)
        return
    if args.source_errors:
        source_errors(args)
        return

    w = inputs.WORKLOADS[args.workload]
    dims, tbc, kappa, csw, nsrc, tol = w["dims"], w["tbc"], w["kappa"], w["csw"], w["nsrc"], w["tol"]
    X, Y, Z, T = dims
    V = X * Y * Z * T
    prec = PREC[args.prec]
    log(f"workload {args.workload}: {dims} V={V} nsrc={nsrc} kappa={kappa} csw={csw} prec={args.prec}")

    # ---- inputs, resident in HBM before timing
    t = time.time()
    links_np = inputs.gauge_field(dims, w["eps"], w["gauge_seed"])
    log(f"gauge field generated on host in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    links = torch.from_numpy(links_np.view(np.float64)).to(dev)
    src = torch.empty((nsrc, T, Z, Y, X, 4, 3, 2), dtype=torch.float64, device=dev)
    sol = torch.zeros_like(src)
    torch.cuda.synchronize()
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    ctx.z2_noise_dev(dims, w["noise_seed"], 0, nsrc, src)
    ctx.set_option("rhs_block", args.rhs_block)
    ctx.set_option("rhs_block64", args.rhs_block64)
    ctx.set_option("check_every", args.check_every)
    ctx.set_option("interleave", args.interleave)
    ctx.set_option("mfma", args.mfma)
    ctx.set_option("delta", args.delta)
    ctx.set_option("delta_bf16", args.delta_bf16)
    ctx.set_option("ru_correction", args.ru_correction)
    ctx.set_option("target_frac", args.target_frac)
    ctx.set_option("tail_checks", args.tail_checks)
    ctx.set_option("schur_sym", args.schur_sym)
    ctx.set_option("solver", a2a.SOLVER_CGNR if args.solver == "cgnr" else a2a.SOLVER_BICGSTAB)

    if args.stencil_only:
        stencil_only(args, ctx, links, dims, tbc, kappa, csw, V)
        return

    tuned = None
    if args.autotune:  # before the warmup, outside the timed region
        g = ctx.load_gauge_dev(links, dims, tbc)
        c = ctx.load_clover(g, csw)
        t = time.perf_counter()
        tuned = ctx.autotune(c, kappa, prec, nsrc)
        tuned["seconds"] = round(time.perf_counter() - t, 2)
        ctx.unload(g)
        ctx.set_option("autotune", 1)
        log(f"autotuned: {tuned}")

    infos = []
    last_corr = {}
    phases = ("load_gauge", "load_clover", "solve", "contract", "unload")

    def step():
        """One pass of the whole path; returns the host wall time of each phase (every call
        below returns only after its device work is done, so the phases add up to the step)."""
        ph = {}
        t = time.perf_counter()
        g = ctx.load_gauge_dev(links, dims, tbc)
        ph["load_gauge"], t = time.perf_counter() - t, time.perf_counter()
        c = ctx.load_clover(g, csw)
        ph["load_clover"], t = time.perf_counter() - t, time.perf_counter()
        info, rc = ctx.solve_propagators_dev(c, src, sol, nsrc, kappa, csw, tol=tol, prec=prec, allow=())
        ph["solve"], t = time.perf_counter() - t, time.perf_counter()
        if nsrc % 4 == 0 and nsrc <= 128:  # one pass over (eta, X): pi-pi pieces and the pion
            diag, vac, corr = ctx.contract_pipi_2pt_dev(src, sol, nsrc, dims, tbc, want_pion=True)
        else:
            corr, _ = ctx.contract_pion_2pt_dev(src, sol, nsrc, dims, tbc)
            diag = None
        ph["contract"], t = time.perf_counter() - t, time.perf_counter()
        ctx.unload(g)  # the fields' buffers go to the context's reuse cache
        ph["unload"] = time.perf_counter() - t
        infos.append(info)
        last_corr["pion"], last_corr["pipi"] = corr, diag
        return ph

    warm_s = []
    for i in range(args.warmup):
        ph = step()
        warm_s.append(sum(ph.values()))
        log(f"warmup step {i} {warm_s[-1]:.3f}s")
    # HIP events around every stencil and vector launch of the solves, on the context stream
    ctx.set_option("kernel_timing", 1)
    ctx.kernel_stats("schur2", reset=True)
    torch.cuda.synchronize()
    step_ph = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ph = step()
        step_ph.append(ph)
        log(f"timed step {i}: {sum(ph.values()):.3f}s (" + ", ".join(f"{k} {ph[k]:.3f}" for k in phases) + ")")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_option("kernel_timing", 0)
    elapsed = t1 - t0
    if args.copy_calib:
        copy_1gib(1)
    value = nsrc * args.steps / elapsed
    kstats = {k: ctx.kernel_stats(k) for k in ("schur1", "schur2", "xr", "p", "s")}
    timed = infos[args.warmup:]
    last = timed[-1]
    iters = [x["iters"] for x in last]
    resid = [x["true_rel_residual"] for inf in timed for x in inf]
    rus = [x["reliable_updates"] for x in last]
    all_conv = all(x["converged"] for inf in timed for x in inf)
    step_s = [sum(ph.values()) for ph in step_ph]
    log(f"{value:.2f} RHS/s; step median {1e3 * float(np.median(step_s)):.1f} ms, max {1e3 * max(step_s):.1f} ms; "
        f"iters {min(iters)}-{max(iters)}; max residual {max(resid):.2e}")

    # dominant kernel of the timed region
    dom = max(kstats, key=lambda k: kstats[k][1])
    n_l, ms_l, by_l = kstats[dom]
    achieved = by_l / (ms_l * 1e-3) / 1e9 if ms_l > 0 else 0.0
    mfma = bool(args.interleave and args.mfma and prec in (2, 3))
    layout = "il" if mfma else f"rb{args.rhs_block}"
    tr = TRAFFIC.get((dom, args.workload, args.prec, layout))
    kind = "mfma" if mfma else "per-thread"
    traffic = tr["bytes"] if tr and tr["src"] == stencil_src_hash(kind) else None
    sym = bool(args.schur_sym) and args.solver == "bicgstab"
    names = ({"schur1": "k_hop_mfma<.., EPI_INV> (H_eo + A_ee^-1, matrix cores)",
              "schur2": "k_hop_mfma<.., 3> (identity - A_oo^-1 H_oe + dot, matrix cores)" if sym else
                        "k_hop_mfma<.., EPI_CLOV> (H_oe + A_oo + axpy + dot, matrix cores)"} if mfma else
             {"schur1": "k_hop<.., EPI_INV> (H_eo + A_ee^-1)",
              "schur2": "k_hop<.., EPI_INVA> (identity - A_oo^-1 H_oe + dot)" if sym else
                        "k_hop<.., EPI_CLOV> (H_oe + A_oo + axpy + dot)"})
    if args.solver == "cgnr":
        names["xr"] = "k_vec_il<.., VK_CG_XR> (x += alpha p; r' -= alpha g5 q; |r'|^2)"
        names["p"] = "k_vec_il<.., VK_CG_P> (p = g5 u + beta p)"
    else:
        names["xr"] = "k_vec_il<.., VK_BICG_XR> (x += alpha p + omega s; r = s - omega t; dots)"
        names["p"] = "k_vec_il<.., VK_BICG_P> (p = r + beta (p - omega v))"
        names["s"] = "k_vec_il<.., VK_BICG_S> (s = r - alpha v)"
    roofline = {"bound": "hbm", "kernel": names[dom],
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "bytes/launch",
                "launches": n_l, "avg_launch_ms": round(ms_l / max(1, n_l), 4),
                "alg_bytes_per_launch": round(by_l / max(1, n_l))}
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 2),
                   "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None} for k, v in kstats.items()}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec else "f64",
           "storage": args.prec, "data": "synthetic",
           "config": {"workload": f"{args.workload}: {X}^3x{T}" if X == Y == Z else args.workload,
                      "dims": list(dims), "kappa": kappa, "c_sw": csw, "t_bc": tbc, "nsrc": nsrc,
                      "tol": tol, "links": f"exp(i {w['eps']} H), seed {w['gauge_seed']}",
                      "noise": f"complex Z2 splitmix64 seed {w['noise_seed']}",
                      "precision": f"inner {args.prec} storage / f32 arithmetic, f64 reliable updates"
                      if prec else "f64",
                      "rhs_block": (tuned["rhs_block"] or args.rhs_block) if tuned else args.rhs_block,
                      "autotuned": {k: tuned[k] for k in ("il_width", "brick", "xcd_slab", "rhs_block",
                                                          "rhs_block64", "brick64", "xcd64", "ms_schur",
                                                          "ms_schur64", "candidates", "seconds")}
                      if tuned else None,
                      "solver": args.solver,
                      "layout": "lane-interleaved groups, matrix-core stencil" if mfma else
                      ("lane-interleaved groups, per-thread stencil" if args.interleave and prec in (2, 3)
                       else "per-slot")},
           "solve": {"iters_min": min(iters), "iters_max": max(iters), "reliable_updates_max": max(rus),
                     "max_true_rel_residual": max(resid), "all_converged": all_conv},
           "step_ms": {"median": round(1e3 * float(np.median(step_s)), 1), "min": round(1e3 * min(step_s), 1),
                       "max": round(1e3 * max(step_s), 1),
                       "warmup_median_untimed_kernels": round(1e3 * float(np.median(warm_s)), 1) if warm_s else None,
                       "phases_median": {k: round(1e3 * float(np.median([ph[k] for ph in step_ph])), 1)
                                         for k in phases}},
           "roofline": roofline, "kernels": kernels,
           "correlators": correlator_summary(last_corr, T)}

    if not args.no_extras:
        ctx.set_option("autotune", 0)  # the side measurements keep their stated widths
        # ---- plain FP64: FP64 storage and arithmetic, one source at a time
        ctx.set_option("rhs_block", 1)
        g = ctx.load_gauge_dev(links, dims, tbc)
        c = ctx.load_clover(g, csw)
        nf = min(args.fp64_sources, nsrc)
        ctx.solve_propagators_dev(c, src[:1], sol[:1], 1, kappa, csw, tol=tol, prec=0)  # warm
        torch.cuda.synchronize()
        tf = time.perf_counter()
        f64_iters = []
        for i in range(nf):
            info, _ = ctx.solve_propagators_dev(c, src[i:i + 1], sol[i:i + 1], 1, kappa, csw, tol=tol, prec=0)
            f64_iters.append(info[0]["iters"])
        torch.cuda.synchronize()
        f64_rate = nf / (time.perf_counter() - tf)
        log(f"plain FP64: {f64_rate:.2f} RHS/s, iters {f64_iters}")
        out["fp64_plain"] = {"value": round(f64_rate, 3), "unit": "RHS/s", "sources": nf, "iters": f64_iters,
                             "note": "FP64 storage+arithmetic, rhs_block 1, one source per solve"}
        out["speedup_vs_fp64_plain"] = round(value / f64_rate, 2)
        # ---- FP64 batched: FP64 storage and arithmetic, all sources in one call (the gain of
        # batching alone); the second of two calls is timed (the first allocates the buffers)
        ctx.set_option("rhs_block", args.rhs_block)
        for _ in range(2):
            tb = time.perf_counter()
            info, _ = ctx.solve_propagators_dev(c, src, sol, nsrc, kappa, csw, tol=tol, prec=0)
            torch.cuda.synchronize()
            tb = time.perf_counter() - tb
        b64_rate = nsrc / tb
        log(f"batched FP64: {b64_rate:.2f} RHS/s")
        out["fp64_batched"] = {"value": round(b64_rate, 3), "unit": "RHS/s", "sources": nsrc,
                               "iters_max": max(x["iters"] for x in info),
                               "note": f"FP64 storage+arithmetic, all sources in one call, rhs_block {args.rhs_block}"}
        out["speedup_vs_fp64_batched"] = round(value / b64_rate, 2)
        # ---- the hopping stencil alone (one parity, H_eo), compulsory bytes (V/2)(8l + 2 n s)/launch
        ds = {}
        for key, p, n, il in (("f64_n1", 0, 1, 0), ("f32_n1", 1, 1, 0), ("f16_n1", 2, 1, 0),
                              ("f16_n16_per_slot", 2, 16, 0), ("f16_n48_matrix_cores", 2, 48, 1)):
            ctx.set_option("rhs_block", 4 if n > 1 else 1)
            ctx.set_option("interleave", il)
            ms = ctx.bench_stencil(c, kappa, a2a.OP_HOP_EO, p, n, 20)
            sb = STORAGE_BYTES[p]
            byts = (V // 2) * (8 * 18 * sb + 2 * n * 24 * sb)
            ds[key] = {"ms": round(ms, 4), "GBps": round(byts / (ms * 1e-3) / 1e9, 1),
                       "frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
        ctx.set_option("rhs_block", args.rhs_block)
        ctx.set_option("interleave", args.interleave)
        log(f"stencil: {ds}")
        out["dslash_hop_eo"] = ds
        ctx.unload(g)

    ctx.finalize()
    del src, sol
    torch.cuda.empty_cache()

    if args.serve_leg and not args.no_extras:
        # a short serving leg: Poisson request streams on three resident lattices (engine)
        import copy

        sa = copy.copy(args)
        sa.serve, sa.mixed = True, False
        sa.serve_rates, sa.serve_requests = args.serve_leg, args.serve_leg_requests
        sv = serve_or_mixed(sa)
        out["serving"] = {"rates": sv["rates"], "iters_per_step": sv["iters_per_step"], "cap_rhs": sv["cap_rhs"],
                          "precision": sv["precision"],
                          "requests": "lattice uniform over 8^3x16 / 16^3x32 / 24^3x48, kappa ~ U[0.120, 0.130], "
                                      "1-64 sources, tol 1e-10"}
        torch.cuda.empty_cache()
    if not args.no_cpu:
        del links
        out["cpu_baseline"] = cpu_baseline(w, links_np)
    print(json.dumps(out), flush=True)


def correlator_summary(last, T):
    """Real parts of the last timed step's pion correlator C(dt) and pi-pi pieces D0..D3 (dt <= T/2)."""
    out = {}
    if last.get("pion") is not None:
        out["pion_C"] = [float(f"{v.real:.6e}") for v in last["pion"][:T // 2 + 1]]
    if last.get("pipi") is not None:
        out["pipi_D0_D1_D2_D3"] = [[float(f"{v.real:.6e}") for v in d[:T // 2 + 1]] for d in last["pipi"]]
    return out


SERVE_LATTICES = [((8, 8, 8, 16), 11), ((16, 16, 16, 32), 12), ((24, 24, 24, 48), 13)]


FP64_PEAK_TFS = 78.6  # MI355X dense FP64 (matrix and vector)


def fill_study(args):
    """The paper's outer-product fill (Sec. 7, eq. Sfill) on the FP64 matrix cores against the
    stochastic-operator route, for the same quantity C(t) = sum_{z,x} tr[S1 S2^dag] (source
    timeslice 0, two independent sets of N sources / solutions) on L^3 x 2L lattices.  The fill
    route costs 2 x 8 T M^2 N flop (M = 12 L^3), the Gram route 8 (T + 1) M N^2 + 8 T N^2, so
    the fill wins only when N > ~M.  Fields are synthetic (counter-hash noise, also for the
    "solutions": the cost does not depend on the values); both routes are checked to agree.
    Also times one fill of S at 8^3x16 with 1024 sources for the kernel's roofline."""
    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a

    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    out = {"mode": "fill", "quantity": "C(t) = sum_{z,x} tr[S1(t,z;0,x) S2(t,z;0,x)^dag], FP64",
           "peak_fp64_tflops": FP64_PEAK_TFS, "rows": []}

    def fields(L, N, seed):
        dims = (L, L, L, 2 * L)
        fs = []
        for k in range(4):
            f = torch.empty((N, 2 * L, L, L, L, 4, 3, 2), dtype=torch.float64, device="cuda")
            ctx.z2_noise_dev(dims, seed + k, 0, N, f)
            fs.append(f)
        torch.cuda.synchronize()
        return dims, fs

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    for L in [int(x) for x in args.fill_sizes.split(",")]:
        for N in [int(x) for x in args.fill_sources.split(",")]:
            M, T = 12 * L ** 3, 2 * L
            if 4 * N * M * T * 16 > 64e9:
                continue
            dims, (X1, e1, X2, e2) = fields(L, N, 100)
            fl_fill = 2 * 8 * T * M * M * N
            fl_gram = 8 * (T + 1) * M * N * N + 8 * T * N * N
            reps_f = 1 if fl_fill > 2e13 else 3
            tf, cf = timed(lambda: ctx.contract_fill_2pt_dev(X1, e1, X2, e2, N, dims, 0, method="fill"), reps_f)
            tg, cg = timed(lambda: ctx.contract_fill_2pt_dev(X1, e1, X2, e2, N, dims, 0, method="gram"), 3)
            agree = float(np.max(np.abs(cf - cg)) / np.max(np.abs(cg)))
            row = {"L": L, "N": N, "M": M, "fill_s": round(tf, 5), "gram_s": round(tg, 5),
                   "fill_over_gram": round(tf / tg, 2), "fill_tflops": round(fl_fill / tf / 1e12, 2),
                   "gram_tflops": round(fl_gram / tg / 1e12, 2), "rel_diff": agree}
            out["rows"].append(row)
            log(f"fill study L={L} N={N}: fill {tf:.4f}s gram {tg:.4f}s ({row['fill_tflops']} / "
                f"{row['gram_tflops']} TF/s), agree {agree:.1e}")
            del X1, e1, X2, e2
            torch.cuda.empty_cache()
    # the fill kernel alone: one S at 8^3x16 from 1024 sources
    L, N = 8, 1024
    dims, (X1, e1, _, _) = fields(L, N, 200)
    M = 12 * L ** 3
    S = torch.empty((M, M, 2), dtype=torch.float64, device="cuda")
    ts, _ = timed(lambda: ctx.fill_propagator_dev(X1, e1, N, dims, 0, 3, S), 10)
    fl = 8 * M * M * N
    byts = 2 * M * N * 16 + M * M * 16
    out["fill_kernel"] = {"workload": "S(t=3, z; 0, x) at 8^3x16 from 1024 sources", "M": M, "K": N,
                          "ms": round(ts * 1e3, 4), "flop": fl, "compulsory_bytes": byts,
                          "roofline": {"bound": "mfma", "achieved": round(fl / ts / 1e12, 2),
                                       "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                                       "frac": round(fl / ts / 1e12 / FP64_PEAK_TFS, 4)}}
    log(f"fill kernel: {ts * 1e3:.3f} ms, {fl / ts / 1e12:.2f} TF/s")
    print(json.dumps(out))


DIL_MOMS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 1, 1)]


def dilution_study(args):
    """Time-spin-colour dilution (Sec. 7) at 8^3x16 (kappa 0.125, c_sw 1.2, links exp(i 0.3 H)):
    n noise vectors, each split into 12 T = 192 pieces, are solved (FP16 inner, FP64 reliable
    updates, tol 1e-10) and contracted into pion correlators at six momenta; an undiluted set of
    as many noise vectors as there are diluted pieces is solved and contracted the same way.
    Reported: solve and contraction times, and the jackknife error of C(dt, p = 0) over noise
    vectors for both sets, i.e. the statistical error at equal cost in solves."""
    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a, inputs

    dims, kappa, csw, tbc, eps = (8, 8, 8, 16), 0.125, 1.2, -1, 0.3
    X, Y, Z, T = dims
    nv = args.dil_noise
    D = 12 * T
    n = nv * D
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_option("rhs_block", args.rhs_block)
    g = ctx.load_gauge(inputs.gauge_field(dims, eps, 1), tbc)
    c = ctx.load_clover(g, csw)
    shape = (T, Z, Y, X, 4, 3, 2)
    out = {"mode": "dilution", "dims": list(dims), "kappa": kappa, "c_sw": csw, "noise_vectors": nv,
           "pieces_per_noise_vector": D, "solves_per_set": n, "moms": DIL_MOMS}

    def solve(src):
        sol = torch.zeros_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, rc = ctx.solve_propagators_dev(c, src, sol, src.shape[0], kappa, csw, tol=1e-10, prec=a2a.F16_F32,
                                             allow=())
        torch.cuda.synchronize()
        return sol, time.perf_counter() - t0, max(x["true_rel_residual"] for x in info)

    noise = torch.empty((nv,) + shape, dtype=torch.float64, device="cuda")
    ctx.z2_noise_dev(dims, 51, 0, nv, noise)
    src_d = torch.empty((n,) + shape, dtype=torch.float64, device="cuda")
    ctx.dilute_dev(noise, nv, dims, a2a.DILUTE_TSC, src_d)
    sol_d, ts_d, res_d = solve(src_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C_d = ctx.contract_pion_mom_dev(src_d, sol_d, n, dims, DIL_MOMS, scheme=a2a.DILUTE_TSC)
    tc_d = time.perf_counter() - t0
    loo = []
    for k in range(nv):  # jackknife over noise vectors
        keep = torch.cat([src_d[i * D:(i + 1) * D] for i in range(nv) if i != k])
        keepx = torch.cat([sol_d[i * D:(i + 1) * D] for i in range(nv) if i != k])
        loo.append(ctx.contract_pion_mom_dev(keep, keepx, n - D, dims, DIL_MOMS[:1], scheme=a2a.DILUTE_TSC)[0])
        del keep, keepx
    loo = np.array(loo)
    err_d = np.sqrt((nv - 1) / nv * np.sum(np.abs(loo - loo.mean(axis=0)) ** 2, axis=0))
    del src_d, sol_d
    torch.cuda.empty_cache()

    src_u = torch.empty((n,) + shape, dtype=torch.float64, device="cuda")
    ctx.z2_noise_dev(dims, 52, 0, n, src_u)
    sol_u, ts_u, res_u = solve(src_u)
    t0 = time.perf_counter()
    C_u, O = ctx.contract_pion_2pt_dev(src_u, sol_u, n, dims, want_O=True)
    tc_u = time.perf_counter() - t0
    # leave-one-out from O: remove the pairs that involve source k
    P = np.stack([np.einsum("tab,tba->", np.roll(O, -dt, axis=0), O) for dt in range(T)])  # all pairs
    diagp = np.stack([np.einsum("taa,taa->a", np.roll(O, -dt, axis=0), O) for dt in range(T)])  # a == b
    rowk = np.stack([np.einsum("tkb,tbk->k", np.roll(O, -dt, axis=0), O) for dt in range(T)])  # a == k
    colk = np.stack([np.einsum("tak,tka->k", np.roll(O, -dt, axis=0), O) for dt in range(T)])  # b == k
    tot = P - diagp.sum(axis=1)
    loo_u = (tot[:, None] - (rowk - diagp) - (colk - diagp)) / (T * (n - 1) * (n - 2))
    err_u = np.sqrt((n - 1) / n * np.sum(np.abs(loo_u - loo_u.mean(axis=1, keepdims=True)) ** 2, axis=1))
    rows = []
    for dt in range(1, T // 2 + 1):
        rows.append({"dt": dt, "C_diluted": round(C_d[0][dt].real, 8), "err_diluted": float(f"{err_d[dt]:.3e}"),
                     "C_undiluted": round(C_u[dt].real, 8), "err_undiluted": float(f"{err_u[dt]:.3e}"),
                     "error_ratio": round(float(err_u[dt] / err_d[dt]), 2)})
    out.update({"solve_s_diluted": round(ts_d, 3), "solve_s_undiluted": round(ts_u, 3),
                "rhs_per_s": round(n / ts_d, 1), "max_true_rel_residual": max(res_d, res_u),
                "contract_s_diluted_6_moms": round(tc_d, 3), "contract_s_undiluted_p0": round(tc_u, 3),
                "pion_p0": rows,
                "pion_moms_dt1": {str(p): round(C_d[m][1].real, 8) for m, p in enumerate(DIL_MOMS)}})
    log(f"dilution: {n} solves {ts_d:.2f}s / {ts_u:.2f}s; contraction {tc_d:.3f}s (6 momenta) / {tc_u:.3f}s")
    for r in rows[:6]:
        log(f"  dt {r['dt']}: diluted {r['C_diluted']:.4e} +- {r['err_diluted']:.1e}, undiluted "
            f"{r['C_undiluted']:.4e} +- {r['err_undiluted']:.1e}")
    ctx.unload(g)
    print(json.dumps(out))


def noise_study(args):
    """The paper's comparison of one noise set for both propagators against two independent sets
    (Sec. 7, Figs. rel1k / rel20k), on the synthetic 4^3x8 field (eps 0.2, kappa 0.120, c_sw 1.0):
    Q(t) = sum_{z, x} tr[S(t, z; 0, x) S(t, z; 0, x)^dag], the all-to-all piece of diagram 0.
    Exact: full dilution of timeslice 0 (12 L^3 unit sources, solved to 1e-10), for which the
    raw sum is exact.  Stochastic: S1, S2 from N_r complex-Z2 noise vectors each; E1 uses S1 for
    both propagators, E2 the independent S2 for the second.  Reported: relative error
    |Q_est - Q| / Q averaged over t, for each N_r, on the GPU path end to end."""
    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a, inputs

    w = inputs.WORKLOADS["tiny_4c8"]
    dims, tbc, kappa, csw = w["dims"], w["tbc"], w["kappa"], w["csw"]
    X, Y, Z, T = dims
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    g = ctx.load_gauge(inputs.gauge_field(dims, w["eps"], w["gauge_seed"]), tbc)
    c = ctx.load_clover(g, csw)
    shape = (T, Z, Y, X, 4, 3, 2)

    def solve(src):
        sol = torch.zeros_like(src)
        info, rc = ctx.solve_propagators_dev(c, src, sol, src.shape[0], kappa, csw, tol=1e-10, prec=a2a.F16_F32,
                                             allow=())
        return sol

    M = 12 * X * Y * Z
    unit = torch.zeros((M,) + shape, dtype=torch.float64, device="cuda")
    unit.view(M, T, M, 2)[torch.arange(M), 0, torch.arange(M), 0] = 1.0  # e_k on timeslice 0
    t0 = time.perf_counter()
    Xu = solve(unit)
    exact = M * M * ctx.contract_fill_2pt_dev(Xu, unit, Xu, unit, M, dims, 0, method="gram").real
    t_exact = time.perf_counter() - t0
    rows = []
    seed = 300
    for nr in [int(x) for x in args.noise_counts.split(",")]:
        e1 = torch.empty((nr,) + shape, dtype=torch.float64, device="cuda")
        e2 = torch.empty_like(e1)
        ctx.z2_noise_dev(dims, seed, 0, nr, e1)
        ctx.z2_noise_dev(dims, seed + 1, 0, nr, e2)
        seed += 2
        X1, X2 = solve(e1), solve(e2)
        q1 = ctx.contract_fill_2pt_dev(X1, e1, X1, e1, nr, dims, 0, method="gram").real
        q2 = ctx.contract_fill_2pt_dev(X1, e1, X2, e2, nr, dims, 0, method="gram").real
        r1 = float(np.mean(np.abs(q1 - exact) / np.abs(exact)))
        r2 = float(np.mean(np.abs(q2 - exact) / np.abs(exact)))
        rows.append({"N_r": nr, "rel_err_one_set": round(r1, 4), "rel_err_two_sets": round(r2, 4),
                     "ratio": round(r1 / r2, 2)})
        log(f"noise study N_r={nr}: one set {r1:.4f}, two sets {r2:.4f}")
        del e1, e2, X1, X2
    out = {"mode": "noise_study", "dims": list(dims), "kappa": kappa, "c_sw": csw,
           "quantity": "sum_{z,x} tr[S(t,z;0,x) S(t,z;0,x)^dag], mean over t of the relative error",
           "exact_solves": M, "exact_s": round(t_exact, 3), "exact_Q": [round(float(v), 6) for v in exact],
           "rows": rows}
    ctx.unload(g)
    print(json.dumps(out))


def point_study(args):
    """The pi-pi diagrams of Sec. 8 from point propagators at the origin (12 solves) and
    stochastic all-to-all propagators, on the synthetic 4^3x8 field (eps 0.2, kappa 0.120,
    c_sw 1.0): D0 = Cp Cs, D1 = L Cp(0), D2 (D3 = conj D2).  Exact: every unit source of the
    lattice (12 V = 6144 solves, tol 1e-10), for which the stochastic formulas are exact.
    Stochastic: N_r complex-Z2 noise vectors per set; one set used for both propagators (E1)
    against two independent sets (E2).  Reported per N_r and diagram: |D_est - D| / |D| with
    the norm over dt (Sec. 7's comparison with point propagators, extended to every diagram)."""
    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a, inputs

    w = inputs.WORKLOADS["tiny_4c8"]
    dims, tbc, kappa, csw = w["dims"], w["tbc"], w["kappa"], w["csw"]
    X, Y, Z, T = dims
    NV = 12 * X * Y * Z * T
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    g = ctx.load_gauge(inputs.gauge_field(dims, w["eps"], w["gauge_seed"]), tbc)
    c = ctx.load_clover(g, csw)
    shape = (T, Z, Y, X, 4, 3, 2)

    def solve(src):
        sol = torch.zeros_like(src)
        ctx.solve_propagators_dev(c, src, sol, src.shape[0], kappa, csw, tol=1e-10, prec=a2a.F16_F32, allow=())
        return sol

    t_start = time.perf_counter()
    psrc = torch.empty((12,) + shape, dtype=torch.float64, device="cuda")
    ctx.point_sources_dev(dims, 0, (0, 0, 0), psrc)
    Sp = solve(psrc)
    unit = torch.zeros((NV,) + shape, dtype=torch.float64, device="cuda")
    unit.view(NV, NV, 2)[torch.arange(NV), torch.arange(NV), 0] = 1.0
    Xu = solve(unit)
    t_solve = time.perf_counter() - t_start
    d_ex, p_ex = ctx.contract_pipi_mixed_dev(Sp, 0, unit, Xu, NV, unit, Xu, NV, dims)
    d_ex, p_ex = d_ex * NV * NV, p_ex.copy()
    p_ex[1:] *= NV * NV
    t_exact = time.perf_counter() - t_start
    del unit, Xu
    torch.cuda.empty_cache()
    names = ("D0", "D1", "D2")

    def errs(d):
        return {k: round(float(np.linalg.norm(d[i] - d_ex[i]) / np.linalg.norm(d_ex[i])), 4) for i, k in enumerate(names)}

    rows = []
    seed = 500
    for nr in [int(x) for x in args.noise_counts.split(",")]:
        e1 = torch.empty((nr,) + shape, dtype=torch.float64, device="cuda")
        e2 = torch.empty_like(e1)
        ctx.z2_noise_dev(dims, seed, 0, nr, e1)
        ctx.z2_noise_dev(dims, seed + 1, 0, nr, e2)
        seed += 2
        X1, X2 = solve(e1), solve(e2)
        tc = time.perf_counter()
        d1, _ = ctx.contract_pipi_mixed_dev(Sp, 0, e1, X1, nr, e1, X1, nr, dims)
        d2, _ = ctx.contract_pipi_mixed_dev(Sp, 0, e1, X1, nr, e2, X2, nr, dims)
        tc = (time.perf_counter() - tc) / 2
        rows.append({"N_r": nr, "one_set": errs(d1), "two_sets": errs(d2), "contract_ms": round(1e3 * tc, 2)})
        log(f"point study N_r={nr}: one set {rows[-1]['one_set']}, two sets {rows[-1]['two_sets']}")
        del e1, e2, X1, X2
    out = {"mode": "point_study", "dims": list(dims), "kappa": kappa, "c_sw": csw, "point": [0, 0, 0, 0],
           "quantity": "|D_est - D| / |D| over dt for D0 = Cp Cs, D1 = L Cp(0), D2",
           "exact_solves": NV + 12, "exact_solve_s": round(t_solve, 3), "exact_total_s": round(t_exact, 3),
           "exact": {k: [[round(float(v.real), 6), round(float(v.imag), 6)] for v in d_ex[i]]
                     for i, k in enumerate(names)},
           "point_pion": [round(float(v.real), 6) for v in p_ex[0]], "rows": rows}
    ctx.unload(g)
    print(json.dumps(out))


def ensemble_study(args):
    """Zero-momentum pi-pi correlator over an ensemble of synthetic configurations (8^3x16,
    eps 0.3, kappa 0.125, c_sw 1.2, seeds 1000 + k): per configuration 64 complex-Z2 sources in
    four independent groups are solved (FP16 inner, tol 1e-10) and contracted into diagrams
    D0..D3, the timeslice loop L(t, t) and the pion; the vacuum part of diagram 1 is subtracted
    with the ensemble average of the loop: C(dt) = <D0 + D1 - D2 - D3> - <L>^2 (Secs. 5 and 8).
    Jackknife errors over configurations.  The fields are not a thermalised ensemble: this
    exercises the machinery, it is not a physics result."""
    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a, inputs

    dims, kappa, csw, tbc, eps, nsrc = (8, 8, 8, 16), 0.125, 1.2, -1, 0.3, 64
    X, Y, Z, T = dims
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    src = torch.empty((nsrc, T, Z, Y, X, 4, 3, 2), dtype=torch.float64, device="cuda")
    sol = torch.zeros_like(src)
    D, V, Pn = [], [], []
    t0 = time.perf_counter()
    for k in range(args.ensemble):
        g = ctx.load_gauge(inputs.gauge_field(dims, eps, 1000 + k), tbc)
        c = ctx.load_clover(g, csw)
        ctx.z2_noise_dev(dims, 2000 + k, 0, nsrc, src)
        sol.zero_()
        info, rc = ctx.solve_propagators_dev(c, src, sol, nsrc, kappa, csw, tol=1e-10, prec=a2a.F16_F32, allow=())
        d, v, pc = ctx.contract_pipi_2pt_dev(src, sol, nsrc, dims, tbc, want_pion=True)
        D.append(d.real)
        V.append(v.real)
        Pn.append(pc.real)
        ctx.unload(g)
    el = time.perf_counter() - t0
    D, V, Pn = np.array(D), np.array(V), np.array(Pn)
    n = len(D)

    def est(idx):
        d = D[idx].mean(axis=0)
        vac = V[idx].mean()
        return d[0] + d[1] - d[2] - d[3] - vac * vac, d[1] - vac * vac, Pn[idx].mean(axis=0)

    full = est(np.arange(n))
    loo = [est(np.array([j for j in range(n) if j != k])) for k in range(n)]
    errs = [np.sqrt((n - 1) / n * np.sum([(l[q] - np.mean([m[q] for m in loo], axis=0)) ** 2 for l in loo],
                                         axis=0)) for q in range(3)]
    rows = [{"dt": dt, "pipi": float(f"{full[0][dt]:.6e}"), "pipi_err": float(f"{errs[0][dt]:.2e}"),
             "D1_subtracted": float(f"{full[1][dt]:.4e}"), "pion": float(f"{full[2][dt]:.6e}"),
             "pion_err": float(f"{errs[2][dt]:.2e}")} for dt in range(T // 2 + 1)]
    out = {"mode": "ensemble", "configurations": n, "dims": list(dims), "sources_per_config": nsrc,
           "seconds": round(el, 2), "loop_mean": float(V.mean()), "rows": rows}
    log(f"ensemble of {n}: {el:.1f}s; <L> = {V.mean():.4e}")
    print(json.dumps(out))


def serve_or_mixed(args):
    """Continuous batching through the engine (a2a_engine_*).

    --mixed: one batch of the three lattices with 8-32 sources each (seed 4), all submitted
    at once, against the same sources solved lattice by lattice with solve_propagators.
    --serve: for each Poisson rate, N requests (seed 3 + rate): lattice uniform over the
    three resident fields, kappa ~ U[0.120, 0.130], 1-64 sources, tol 1e-10, FP16/FP32 +
    FP64 reliable updates.  Requests are submitted at their arrival times while the engine
    steps; latency = completion - arrival on the host clock; p50/p99 and RHS/s per rate."""
    import numpy as np
    import torch

    from paper_1405_4524_amd import a2a, inputs

    csw, tbc, eps, prec = 1.5, -1, 0.35, PREC[args.prec]
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_option("rhs_block", args.rhs_block)
    fields = []
    for dims, seed in SERVE_LATTICES:
        g = ctx.load_gauge(inputs.gauge_field(dims, eps, seed), tbc)
        fields.append(dict(dims=dims, c=ctx.load_clover(g, csw), V=int(np.prod(dims))))
    log("resident fields loaded")
    next_src = [0]

    def make_sources(f, n):
        X, Y, Z, T = f["dims"]
        src = torch.empty((n, T, Z, Y, X, 4, 3, 2), dtype=torch.float64, device="cuda")
        ctx.z2_noise_dev(f["dims"], 7, next_src[0], n, src)
        next_src[0] += n
        return src, torch.zeros_like(src)

    out = {"mode": "mixed" if args.mixed else "serve", "precision": args.prec, "rhs_block": args.rhs_block}
    if not args.mixed:
        out.update(policy=json.loads(args.serve_policy), iters_per_step=args.serve_step, cap_rhs=args.serve_cap)
    if args.mixed:
        rng = np.random.default_rng(4)
        jobs = []
        for f in fields:
            n = int(rng.integers(8, 33))
            src, sol = make_sources(f, n)
            jobs.append((f, n, src, sol))
        kappa = 0.13
        # lattice by lattice
        torch.cuda.synchronize()
        t = time.perf_counter()
        for f, n, src, sol in jobs:
            ctx.solve_propagators_dev(f["c"], src, sol, n, kappa, csw, tol=1e-10, prec=prec)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t
        ref = [sol.clone() for _, _, _, sol in jobs]
        # one batch through the engine
        eng = ctx.engine_create('{"max_slots": 256}')
        for _, _, _, sol in jobs:
            sol.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        tickets = [eng.submit(f["c"], kappa, src, n, 1e-10, prec, 100000, sol) for f, n, src, sol in jobs]
        while True:
            eng.step(8)
            if all(eng.poll(tk, n)[0] != 0 for tk, (_, n, _, _) in zip(tickets, jobs)):
                break
        torch.cuda.synchronize()
        t_mix = time.perf_counter() - t
        ntot = sum(n for _, n, _, _ in jobs)
        diff = max(float(torch.linalg.vector_norm(sol - r) / torch.linalg.vector_norm(r))
                   for (_, _, _, sol), r in zip(jobs, ref))
        eng.destroy()
        out.update({"lattices": [list(f["dims"]) for f, _, _, _ in jobs], "sources": [n for _, n, _, _ in jobs],
                    "rhs_per_s_one_batch": round(ntot / t_mix, 2), "rhs_per_s_lattice_by_lattice": round(ntot / t_seq, 2),
                    "max_rel_diff_batch_vs_alone": diff})
        log(f"mixed batch {ntot / t_mix:.1f} RHS/s vs lattice by lattice {ntot / t_seq:.1f} RHS/s, diff {diff:.2e}")
    else:
        eng = ctx.engine_create(args.serve_policy)
        results = []
        for rate in [float(x) for x in args.serve_rates.split(",")]:
            rng = np.random.default_rng(3 + int(rate))
            nreq = args.serve_requests
            arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
            spec = [(int(rng.integers(0, 3)), float(rng.uniform(0.120, 0.130)), int(rng.integers(1, 65)))
                    for _ in range(nreq)]
            live, lat, nrhs_done = {}, [], 0
            # arrived requests wait on the client side while the sources already submitted
            # exceed serve_cap RHS (their device arrays and the engine's state bound the HBM in
            # use); latency runs from arrival either way
            backlog, outstanding, max_backlog = collections.deque(), 0, 0
            k = 0
            t0 = time.perf_counter()
            while k < nreq or live or backlog:
                now = time.perf_counter() - t0
                while k < nreq and arrivals[k] <= now:
                    backlog.append(k)
                    k += 1
                max_backlog = max(max_backlog, len(backlog))
                while backlog and (not live or outstanding + spec[backlog[0]][2] <= args.serve_cap):
                    j = backlog.popleft()
                    li, kappa, n = spec[j]
                    f = fields[li]
                    src, sol = make_sources(f, n)
                    tk = eng.submit(f["c"], kappa, src, n, 1e-10, prec, 100000, sol)
                    live[tk] = (arrivals[j], n, src, sol)
                    outstanding += n
                if live:
                    eng.step(args.serve_step)
                else:
                    time.sleep(max(0.0, min(0.01, arrivals[k] - now)))
                for tk in list(live):
                    done, info, rc = eng.poll(tk, live[tk][1])
                    if done:
                        if done < 0 or not all(x["converged"] for x in info):
                            raise RuntimeError(f"request {tk} failed: {rc}")
                        lat.append(time.perf_counter() - t0 - live[tk][0])
                        nrhs_done += live[tk][1]
                        outstanding -= live[tk][1]
                        del live[tk]
                        if len(lat) % 50 == 0:
                            log(f"serve rate {rate}: {len(lat)} of {nreq} requests done")
            span = time.perf_counter() - t0
            r = {"rate_req_per_s": rate, "requests": nreq, "p50_s": round(float(np.percentile(lat, 50)), 4),
                 "p99_s": round(float(np.percentile(lat, 99)), 4), "rhs_per_s": round(nrhs_done / span, 2),
                 "makespan_s": round(span, 2), "hbm_in_use_GB": round(ctx.mem_in_use() / 1e9, 2),
                 "max_client_backlog": max_backlog}
            results.append(r)
            log(f"serve {r}")
        eng.destroy()
        out["rates"] = results
    ctx.finalize()
    return out


def stencil_only(args, ctx, links, dims, tbc, kappa, csw, V):
    """H_eo alone in each precision, plus a plain device copy of 1 GiB whose counters calibrate
    FETCH_SIZE / WRITE_SIZE (a copy reads and writes exactly its size)."""
    import torch

    from paper_1405_4524_amd import a2a

    g = ctx.load_gauge_dev(links, dims, tbc)
    c = ctx.load_clover(g, csw)
    res = {}
    for key, p, n, rb, il, op in (("f64_n1", 0, 1, 1, 0, a2a.OP_HOP_EO), ("f32_n1", 1, 1, 1, 0, a2a.OP_HOP_EO),
                                  ("f16_n1", 2, 1, 1, 0, a2a.OP_HOP_EO),
                                  ("f16_n16_per_slot", 2, 16, 2, 0, a2a.OP_HOP_EO),
                                  ("f16_n48_matrix_cores", 2, 48, 2, 1, a2a.OP_HOP_EO),
                                  ("f16_n48_matrix_cores_schur", 2, 48, 2, 1, a2a.OP_SCHUR)):
        ctx.set_option("rhs_block", rb)
        ctx.set_option("interleave", il)
        ms = ctx.bench_stencil(c, kappa, op, p, n, args.stencil_reps)
        sb = STORAGE_BYTES[p]
        byts = (V // 2) * (8 * 18 * sb + 2 * n * 24 * sb)
        if op == a2a.OP_SCHUR:  # H_eo + A_ee^-1, then H_oe + A_oo: two hops, clover twice, aux input
            byts = 2 * byts + (V // 2) * (2 * 72 * sb + n * 24 * sb)
        res[key] = {"ms": round(ms, 4), "alg_bytes": byts, "GBps": round(byts / (ms * 1e-3) / 1e9, 1)}
        log(f"stencil {key}: {ms:.4f} ms, {res[key]['GBps']} GB/s")
    ms = copy_1gib(args.stencil_reps)
    res["copy_1GiB"] = {"ms": round(ms, 4), "GBps": round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1)}
    log(f"copy 1 GiB: {ms:.4f} ms")
    ctx.unload(g)
    ctx.finalize()
    print(json.dumps({"stencil_only": res, "workload": args.workload}), flush=True)


def copy_1gib(reps):
    """A plain device copy of 1 GiB (reads and writes exactly its size): the known traffic that
    scales the FETCH_SIZE / WRITE_SIZE counters. Returns ms per copy."""
    import torch

    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    torch.cuda.empty_cache()
    return ms


def host_info():
    """CPU model, the cores this process may run on, and the oracle's OpenMP threads."""
    import oracle

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0)), "omp_threads": oracle.num_threads()}


def source_errors(args):
    """Every source of one workload, solved on the GPU in the benchmark's configuration (all
    sources in one call, FP16 and BF16 storage, FP64 reliable updates, tol 1e-10) and by the
    oracle (FP64 BiCGStab on the full system to 1e-12, host cores): per source, the propagator's
    relative error ||X - X_O|| / ||X_O||, the residual ||eta - D X|| / ||eta|| recomputed with
    the oracle's D, and the residual the library reports.  The oracle's inputs are the host
    generators' (the device noise equals them bitwise, which is checked per source)."""
    import numpy as np
    import torch

    import oracle
    from paper_1405_4524_amd import a2a, inputs

    w = inputs.WORKLOADS[args.source_errors]
    dims, tbc, kappa, csw, n = w["dims"], w["tbc"], w["kappa"], w["csw"], w["nsrc"]
    X, Y, Z, T = dims
    U = inputs.gauge_field(dims, w["eps"], w["gauge_seed"])
    ctx = a2a.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_option("autotune", 1)
    links = torch.from_numpy(U.view(np.float64)).cuda()
    g = ctx.load_gauge_dev(links, dims, tbc)
    c = ctx.load_clover(g, csw)
    src = torch.empty((n, T, Z, Y, X, 4, 3, 2), dtype=torch.float64, device="cuda")
    ctx.z2_noise_dev(dims, w["noise_seed"], 0, n, src)
    sols, infos = {}, {}
    for name, p in (("f16", a2a.F16_F32), ("bf16", a2a.BF16_F32)):
        sol = torch.zeros_like(src)
        t = time.perf_counter()
        info, _ = ctx.solve_propagators_dev(c, src, sol, n, kappa, csw, tol=w["tol"], prec=p, allow=())
        torch.cuda.synchronize()
        log(f"source errors: GPU {name} solve of {n} sources {time.perf_counter() - t:.2f}s")
        sols[name] = sol.cpu().numpy().view(np.complex128).reshape(n, T, Z, Y, X, 4, 3)
        infos[name] = info
        del sol
    dev_eta = src.cpu().numpy().view(np.complex128).reshape(n, T, Z, Y, X, 4, 3)
    ctx.unload(g)
    ctx.finalize()
    del src, links
    torch.cuda.empty_cache()
    A = oracle.clover(U, kappa, csw)
    rows = []
    t0 = time.perf_counter()
    for i in range(n):
        eta = inputs.z2_noise(dims, 1, w["noise_seed"], src_offset=i)[0]
        assert np.array_equal(eta, dev_eta[i]), i
        Xo, io = oracle.solve(U, A, kappa, eta, tbc, tol=1e-12)
        row = {"source": i, "oracle_iters": int(io[0, 0]), "oracle_residual": float(f"{io[0, 3]:.3e}")}
        ne = np.linalg.norm(eta)
        for name in ("f16", "bf16"):
            Xg = sols[name][i]
            row[f"{name}_prop_err"] = float(f"{np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo):.3e}")
            row[f"{name}_residual"] = float(
                f"{np.linalg.norm(eta - oracle.apply_D(U, A, kappa, Xg, tbc)) / ne:.3e}")
            row[f"{name}_reported"] = float(f"{infos[name][i]['true_rel_residual']:.3e}")
            row[f"{name}_iters"] = infos[name][i]["iters"]
        rows.append(row)
        log(f"source errors: {row} ({time.perf_counter() - t0:.0f}s)")
    summary = {}
    for name in ("f16", "bf16"):
        e = [r[f"{name}_prop_err"] for r in rows]
        res = [r[f"{name}_residual"] for r in rows]
        summary[name] = {"prop_err_max": max(e), "prop_err_median": float(np.median(e)), "residual_max": max(res)}
    print(json.dumps({"mode": "source_errors", "workload": args.source_errors, "nsrc": n, "tol": w["tol"],
                      "oracle_tol": 1e-12, "summary": summary, "rows": rows}), flush=True)


def cpu_baseline(w, links_np):
    """The FP64 CPU oracle on a bounded sample of the same workload: one full solve (source 0 of
    the workload's noise set, the oracle's BiCGStab on the un-preconditioned system with
    true-residual restarts) to the workload's tolerance, on all of the host's cores; RHS/s is
    one over its wall time (the clover build is timed separately and not counted)."""
    import oracle
    from paper_1405_4524_amd import inputs

    dims, tbc, kappa, csw = w["dims"], w["tbc"], w["kappa"], w["csw"]
    hi = host_info()
    t = time.perf_counter()
    A = oracle.clover(links_np, kappa, csw)
    t_clover = time.perf_counter() - t
    eta = inputs.z2_noise(dims, 1, w["noise_seed"])[0]
    t = time.perf_counter()
    _, info = oracle.solve(links_np, A, kappa, eta, tbc, tol=w["tol"])
    t_solve = time.perf_counter() - t
    iters, res = int(info[0, 0]), float(info[0, 3])
    del A
    log(f"oracle: clover {t_clover:.1f}s; one full solve {t_solve:.1f}s ({iters} iterations, residual {res:.2e}) "
        f"on {hi['omp_threads']} threads of {hi['cpu_model']}")
    X, Y, Z, T = dims
    return {"value": 1.0 / t_solve, "unit": "RHS/s", "cores": hi["omp_threads"], "kind": "oracle",
            "sample": f"source 0 of the {w['nsrc']} sources of {X}^3x{T} (a 1-of-{w['nsrc']} subset), solved by the "
                      f"oracle to ||eta - D X|| <= {w['tol']:g} ||eta|| ({iters} BiCGStab iterations on the full "
                      f"system, true residual {res:.2e}); clover build {t_clover:.1f} s not counted",
            "solve_s": round(t_solve, 2), "iters": iters, "secs_per_iter": round(t_solve / max(1, iters), 3),
            **hi}


def cpu_study(args):
    """The oracle on the host cores (no GPU): the FP64 hopping term in GB/s at the 16^3x32,
    24^3x48 and 32^3x64 shapes, and full solves of the small workloads, on all cores and on one.
    Hop bytes are the compulsory ones of the full-lattice operator: V x (4 links + spinor in +
    spinor out) = 960 B per site."""
    import numpy as np

    import oracle
    from paper_1405_4524_amd import inputs

    hi = host_info()
    nthreads = hi["omp_threads"]
    out = {"mode": "cpu_study", **hi, "hop": [], "solves": []}
    for name in ("l16t32", "l24t48", "l32t64"):
        w = inputs.WORKLOADS[name]
        U = inputs.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
        psi = inputs.z2_noise(w["dims"], 1, w["noise_seed"])[0]
        V = inputs.volume(w["dims"])
        for th in (nthreads, 1):
            oracle.set_num_threads(th)
            oracle.hop(U, psi, w["tbc"])
            reps = 3 if th > 1 else 1
            t = time.perf_counter()
            for _ in range(reps):
                oracle.hop(U, psi, w["tbc"])
            dt = (time.perf_counter() - t) / reps
            row = {"workload": name, "threads": th, "s": round(dt, 4), "GBps": round(V * 960 / dt / 1e9, 2)}
            out["hop"].append(row)
            log(f"cpu hop {row}")
        del U, psi
    oracle.set_num_threads(nthreads)
    for name, n_all, n_one in (("tiny_4c8", 4, 4), ("l16t32", args.cpu_study_sources, 1)):
        w = inputs.WORKLOADS[name]
        U = inputs.gauge_field(w["dims"], w["eps"], w["gauge_seed"])
        A = oracle.clover(U, w["kappa"], w["csw"])
        for th, n in ((nthreads, n_all), (1, n_one)):
            oracle.set_num_threads(th)
            eta = inputs.z2_noise(w["dims"], n, w["noise_seed"])
            t = time.perf_counter()
            _, info = oracle.solve(U, A, w["kappa"], eta, w["tbc"], tol=w["tol"])
            dt = time.perf_counter() - t
            row = {"workload": name, "threads": th, "sources": n, "of": w["nsrc"], "s": round(dt, 3),
                   "rhs_per_s": round(n / dt, 5), "iters": [int(x) for x in info[:, 0]],
                   "max_residual": float(info[:, 3].max())}
            out["solves"].append(row)
            log(f"cpu solve {row}")
        del U, A
    oracle.set_num_threads(nthreads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
