/*
 * a2a.h -- C ABI of liba2a: stochastic all-to-all propagators for lattice QCD on one
 * AMD Instinct MI355X (gfx950).
 *
 * What is computed (Giedt & Howarth, "Stochastic propagators for multi-pion correlation
 * functions in lattice QCD with GPUs", arXiv:1405.4524):
 *   - Sec. 7, eq. (Sfill): the all-to-all propagator is estimated from noise sources,
 *     S ~ (1/N_r) sum_i X_i eta_i^dag, with X_i = D^{-1} eta_i.  This library solves
 *     D X_i = eta_i for many complex-Z2 sources at once (a2a_solve_propagators).
 *   - D is the clover-improved Wilson "lattice fermion matrix" of Sec. 7 with the
 *     tree-level coefficient c_SW of Sec. 8, written in the hopping-parameter form
 *         D = A - kappa H,
 *         (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu),
 *         A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu(x),
 *     with F the four-leaf clover field strength (Q - Q^dag)/8, sigma_munu = (i/2)[gamma_mu,
 *     gamma_nu], Hermitian gamma matrices in the chiral basis
 *         gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1,1,-1,-1),
 *     periodic links and a fermion sign t_bc on hops that wrap around in time.
 *   - Sec. 7, eq. (stoop): stochastic operators O_ij(t) = sum_{y in t} eta_i^dag(y) gamma_5 X_j(y)
 *     and the zero-momentum pion correlator built from them (a2a_contract_pion_2pt); the
 *     pi-pi diagram pieces of Secs. 5 and 8 from the same operators with independent noise
 *     groups (a2a_contract_pipi_2pt).
 *
 * Canonical host/device layouts (complex128 = two doubles, real first):
 *   links    [t][z][y][x][mu][row][col]          mu = 0..3 for x, y, z, t
 *   spinors  [src][t][z][y][x][spin][colour]
 *   site index inside a field: ((t*Z + z)*Y + y)*X + x  (x fastest)
 *
 * Conventions for every call:
 *   - return value 0 (A2A_OK) or a negative A2A_E* code; a2a_last_error() describes the
 *     last failure on that context.  No exception crosses the ABI.
 *   - the caller owns every buffer it passes; host buffers are not kept after a call
 *     returns.  *_dev calls take device pointers (for instance torch data_ptr()) and run
 *     on the context's stream; their buffers must stay alive until that stream is
 *     synchronised (the synchronous calls synchronise before returning).
 *   - the context owns resident fields (gauge and clover handles) until a2a_unload or
 *     a2a_finalize; all its device memory counts against the HBM budget given at
 *     a2a_init, and a call that would exceed it fails with A2A_ENOMEM before allocating.
 *   - a context is not thread-safe; use one per host thread.
 */
#ifndef A2A_H
#define A2A_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define A2A_OK 0
#define A2A_EINVAL (-1)      /* bad argument: odd or < 2 extents, nrhs <= 0, kappa <= 0, tol <= 0, ... */
#define A2A_ENOMEM (-2)      /* the HBM budget (or the device) cannot hold the request; nothing allocated */
#define A2A_ENOTCONV (-3)    /* max_iter reached; solutions hold the best iterate, info the residuals */
#define A2A_EBREAKDOWN (-4)  /* the Krylov solver broke down repeatedly after restarts */
#define A2A_ENAN (-5)        /* non-finite input */
#define A2A_EHANDLE (-6)     /* unknown or wrong-kind handle */
#define A2A_EDEVICE (-7)     /* a HIP runtime error; the message carries the HIP error string */
#define A2A_EAGAIN (-8)      /* engine: queue full, retry after a step */

/* ---- precision modes: storage / arithmetic of the inner Krylov solve ----------------- */
#define A2A_F64 0        /* FP64 storage and arithmetic throughout ("plain" solver)          */
#define A2A_F32 1        /* FP32 storage and arithmetic, FP64 reliable updates               */
#define A2A_F16_F32 2    /* FP16 storage, FP32 arithmetic, FP64 reliable updates             */
#define A2A_BF16_F32 3   /* BF16 storage, FP32 arithmetic, FP64 reliable updates             */

/* ---- inner Krylov methods (option "solver") ------------------------------------------ */
#define A2A_SOLVER_BICGSTAB 0  /* BiCGStab on the Schur system (van der Vorst 1992)             */
#define A2A_SOLVER_CGNR 1      /* CG on the normal equations M^dag M x = M^dag b, with M^dag =
                                  gamma_5 M gamma_5 (the Schur operator is gamma_5-hermitian)  */

/* ---- operator selectors for a2a_dslash_clover ---------------------------------------- */
#define A2A_OP_FULL_D 0  /* out = D in on the full lattice                                  */
#define A2A_OP_SCHUR 1   /* odd sites: out_o = (A_oo - kappa^2 H_oe A_ee^{-1} H_eo) in_o; out_e = 0 */
#define A2A_OP_HOP_EO 2  /* out_e = (H in)_e from in_o; out_o = 0                           */
#define A2A_OP_HOP_OE 3  /* out_o = (H in)_o from in_e; out_e = 0                           */

/* ---- dilution schemes (a2a_dilute_dev) ----------------------------------------------- */
#define A2A_DILUTE_NONE 0  /* D = 1: the noise vector itself                                  */
#define A2A_DILUTE_T 1     /* D = T: one timeslice per piece, d = t                            */
#define A2A_DILUTE_SC 2    /* D = 12: one spin-colour component per piece, d = 3 spin + colour */
#define A2A_DILUTE_TSC 3   /* D = 12 T: both, d = 12 t + 3 spin + colour                       */

/* ---- correlator normalisation modes -------------------------------------------------- */
#define A2A_PION_UNBIASED 0   /* C(dt) = 1/(T N (N-1)) sum_t0 sum_{a != b} O_ab(t0+dt) O_ba(t0) */
#define A2A_PION_ALL_PAIRS 1  /* C(dt) = 1/(T N^2) sum_t0 sum_{a, b} ... (the printed Sec. 7 form)  */

typedef struct a2a_ctx a2a_ctx;
typedef struct a2a_engine a2a_engine;

typedef struct {
  int dims[4]; /* X, Y, Z, T: each even and >= 2 */
  int t_bc;    /* +1 periodic or -1 antiperiodic fermion boundary in time */
} a2a_geom;

typedef struct {
  int iters;             /* inner Krylov iterations                                     */
  int reliable_updates;  /* FP64 true-residual recomputations                           */
  int converged;         /* 1 if ||eta - D X|| <= tol ||eta|| was verified in FP64       */
  int restarts;          /* Krylov restarts after a breakdown                           */
  double true_rel_residual; /* ||eta - D X||_2 / ||eta||_2 on the full lattice, in FP64  */
  double seconds;        /* wall time from admission to completion                      */
  int solver;            /* A2A_SOLVER_* that finished the source (CGNR after a fallback) */
  int reserved;
} a2a_solve_info;

/* ---- context ------------------------------------------------------------------------- */
/* Create a context on HIP device `device`.  hbm_budget_bytes = 0 means 90% of the free
 * device memory.  hip_stream = NULL creates a private stream owned by the context;
 * otherwise all work is queued on the given hipStream_t (not owned). */
int a2a_init(a2a_ctx **ctx, int device, size_t hbm_budget_bytes, void *hip_stream);
/* Release every handle, engine and allocation of the context. */
int a2a_finalize(a2a_ctx *ctx);
/* Message for the last failed call on ctx (never NULL; empty after success). */
const char *a2a_last_error(const a2a_ctx *ctx);
/* Tuning knobs: "rhs_block" (1, 2, 4: RHS per thread in the stencil), "rhs_block64" (1, 2:
 * RHS per thread in the FP64 stencils of set-up, reliable updates and reconstruction; default
 * 2), "check_every" (iterations between residual checks), "delta" (reliable-update reduction
 * factor for FP16 / FP32 storage, default 0.03), "delta_bf16" (the same for BF16, default 0.05),
 * "delta_cgnr" (the same for CGNR with FP16 storage, default 0.1),
 * "delta64" (the same for the FP64-only mode, default 1e-3),
 * "xcd_order" (0/1), "kernel_timing" (0/1), "autotune" (0/1), "hbm_budget" (bytes; resets
 * the budget given at a2a_init), "interleave" (0/1, default 1: FP16 / BF16 inner vectors of
 * the sources of one call or request in lane-interleaved groups of up to 48, which the stencil
 * applies on the matrix cores), "mfma" (0/1: 0 makes interleaved groups use the per-thread
 * stencil), "solver" (A2A_SOLVER_BICGSTAB (default) or A2A_SOLVER_CGNR: the inner method of
 * later solve calls and engine submissions), "cgnr_fallback" (0/1, default 1: in solve calls,
 * sources whose BiCGStab broke down repeatedly are solved again by CGNR from their current
 * iterate; iterations count against the same max_iter), "force_breakdown" (0/1, default 0:
 * a test hook that makes every BiCGStab source of a solve call report a breakdown at its first
 * reliable update, so that the fallback runs), "poison_memory" (0/1, default 0: a test hook that
 * fills every device buffer the context allocates or reuses with 0xFF bytes, NaN in every
 * floating format, so that a read of memory not written first shows in the results),
 * "fail_setup_enomem" / "fail_setup_device" (n >= 0, default 0: test hooks that make the next
 * n source preparations of solve calls and engine admissions fail with A2A_ENOMEM /
 * A2A_EDEVICE, so that the clean-up of a failed admission can be checked), "il_width" (16, 32
 * or 48, default 48: RHS per lane-interleaved group), "brick" (by * 10000 + bz * 100 + bt:
 * the stencil brick of later calls on lattices it tiles, 0 = each lattice's default; a brick
 * orders the stencil's sweep only, results are unchanged), "mfma_slab" (0/1, default 0: the
 * matrix-core stencil's blocks in XCD slabs, XCD k taking the k-th eighth of the bricks),
 * "ru_correction" (0/1, default 1: mixed-precision reliable updates compute the FP64 residual
 * as r64 -= M (sigma x_lo) from the stored low-precision correction, in FP64 arithmetic; 0
 * recomputes r64 = b - M x64 from the FP64 iterate), "target_frac" (in (0, 1], default 0.8: a
 * source's iteration stops when its odd-site Schur residual reaches target_frac tol ||eta||;
 * the reconstruction then computes the full-system FP64 residual, which decides convergence,
 * and a source it does not accept continues with a tenfold tighter target), "tail_checks" (0/1,
 * default 1: once at most a quarter of the most sources a solve has run at once are still
 * iterating, their residuals are checked after every iteration instead of every check_every),
 * "schur_sym" (0/1, default 1: BiCGStab iterates the symmetric Schur form
 * 1 - kappa^2 A_oo^{-1} H_oe A_ee^{-1} H_eo on A_oo^{-1} b, which has the same solution; the FP64
 * residuals, reliable updates and reconstruction stay in the form A_oo - kappa^2 H_oe A_ee^{-1}
 * H_eo; CGNR always uses that form), "upload_stage_bytes" (size of the pinned host buffer through
 * which the context uploads its device tables without waiting; 0 = 64 MiB; uploads larger than a
 * quarter of it wait for their copy).
 * Returns A2A_EINVAL for an unknown key. */
int a2a_set_option(a2a_ctx *ctx, const char *key, double value);
/* Bytes of device memory in the context's live buffers.  Freed buffers are kept for reuse
 * (same-size requests take them without hipMalloc) and are released whenever an allocation
 * would otherwise not fit the budget or the device; they are not counted here. */
size_t a2a_mem_in_use(const a2a_ctx *ctx);
/* Return the freed buffers kept for reuse to the device (hipFree, which waits for the device);
 * *released (may be NULL) receives their bytes.  a2a_engine_destroy and a2a_finalize do
 * this too; solve calls and a2a_unload keep the buffers, so that the next call of the same
 * shape (a solve, or the fields of the next gauge configuration) allocates nothing. */
int a2a_trim(a2a_ctx *ctx, size_t *released);

/* ---- resident fields (Sec. 7 "inversions in the background of the gauge field") ------ */
/* Upload a gauge field (canonical layout) and convert it to the even-odd device layout in
 * every precision; *gauge_h receives a handle.  Links must be finite. */
int a2a_load_gauge(a2a_ctx *ctx, const a2a_geom *geom, const double *links_host, int *gauge_h);
int a2a_load_gauge_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *links_dev, int *gauge_h);
/* Build the kappa-independent clover field for c_sw (Sec. 8, c_SW) on a gauge handle.
 * A(kappa) and A^{-1}(kappa) are made and cached on first use of each kappa. */
int a2a_load_clover(a2a_ctx *ctx, int gauge_h, double c_sw, int *clover_h);
/* Free a gauge or clover handle (a gauge handle also frees its clover handles).  The
 * buffers go to the context's reuse cache (see a2a_trim), not back to the device: a loop over
 * configurations that loads, solves and unloads allocates nothing after its first pass. */
int a2a_unload(a2a_ctx *ctx, int handle);

/* ---- operator application (parity tests and the stencil benchmark) -------------------- */
/* out = op(in) for nrhs spinor fields in canonical layout, computed in precision `prec`
 * (inputs are rounded to that storage precision first).  dagger = 1 applies op^dag
 * through gamma_5 hermiticity (gamma_5 op gamma_5).  Host and device variants. */
int a2a_dslash_clover(a2a_ctx *ctx, int clover_h, double kappa, int op, int dagger, int prec,
                      const double *in_host, double *out_host, int nrhs);
int a2a_dslash_clover_dev(a2a_ctx *ctx, int clover_h, double kappa, int op, int dagger, int prec,
                          const double *in_dev, double *out_dev, int nrhs);
/* Time `reps` applications of one stencil launch (op = A2A_OP_HOP_EO or A2A_OP_SCHUR) on
 * nrhs device-resident fields already converted to the device layout; returns the mean
 * kernel milliseconds per application measured with HIP events on the context stream. */
int a2a_bench_stencil(a2a_ctx *ctx, int clover_h, double kappa, int op, int prec, int nrhs, int reps,
                      double *ms_per_apply);

/* Launch configuration chosen by the autotuner for one workload. */
typedef struct {
  int il_width;      /* RHS per lane-interleaved group on the matrix cores: 16, 32 or 48 (0: not used) */
  int brick[3];      /* stencil brick extents in y, z, t (the x extent is the whole checkerboard row) */
  int rhs_block;     /* RHS per thread of the per-thread stencil: 1, 2 or 4 (0: the context option) */
  int rhs_block64;   /* RHS per thread of the FP64 stencils of reliable updates: 1 or 2 */
  double ms_schur;   /* best time of the inner-precision Schur operator (both stencils), ms; -1 if cached */
  double ms_schur64; /* best time of the FP64 stencils the solves run, ms: the correction-form
                        reliable-update pair for FP16 / BF16 / FP32 storage, else the FP64 Schur
                        operator; -1 if cached */
  int candidates;    /* configurations timed (0: taken from the cache) */
  int xcd_slab;      /* matrix-core blocks: 1 in XCD slabs, 0 in brick order, -1 not used */
  int brick64[3];    /* brick of the FP64 stencils of reliable updates (y, z, t) */
  int xcd64;         /* FP64 stencil blocks: 1 in XCD slabs, 0 not */
} a2a_tune_result;

/* Autotune the launch configuration of the batched stencils (the multi-RHS batching of the
 * solve) for this lattice, precision and number of sources, by a coordinate search that times
 * the Schur operator on min(nrhs, 64) sources: first the RHS width (the lane-interleaved group
 * width 16 / 32 / 48 for FP16 / BF16 storage on the matrix cores, else the per-thread width
 * 1 / 2 / 4), then the stencil brick (up to six shapes that tile the lattice) together with
 * the order of the matrix-core blocks over the XCDs (brick order or XCD slabs), then for the
 * FP64 stencils of the reliable updates their width 1 / 2 and their own brick and block order
 * (FP64 Schur operator on min(nrhs, 24) sources).  The result is kept in
 * the context and in the JSON file named by the environment variable A2A_TUNE_CACHE, keyed by
 * arch, lattice, precision and RHS bucket (the next power of two, at most 64); a cached key
 * is returned without timing.  With option "autotune" = 1 solve calls tune on first use of a
 * key and run in the tuned configuration.  result may be NULL.  Temporary device buffers of
 * up to min(nrhs, 64) sources are allocated (and kept in the context's buffer cache). */
int a2a_autotune(a2a_ctx *ctx, int clover_h, double kappa, int prec, int nrhs, a2a_tune_result *result);
/* The stencil bricks (y, z, t extents) the autotuner may choose for a lattice, in order of
 * preference (the first is the default), as out[3 k + 0..2], at most maxn of them.  Host only;
 * returns their number, or A2A_EINVAL for a bad geometry. */
int a2a_brick_choices(const a2a_geom *geom, int *out, int maxn);

/* ---- solves (Sec. 7: X_i = D^{-1} eta_i) --------------------------------------------- */
/* Solve D X_i = eta_i for nrhs sources with even-odd preconditioning (odd-site Schur
 * complement A_oo - kappa^2 H_oe A_ee^{-1} H_eo), batched BiCGStab (or CGNR, option
 * "solver") in precision `prec` and FP64 reliable updates, until the FP64 true residual of the full system satisfies
 * ||eta - D X||_2 <= tol ||eta||_2 for every source.  c_sw must equal the clover handle's.
 * x0_or_null: optional initial guess (resume); info: nrhs records (may be NULL).
 * A zero source gives X = 0, converged, residual 0.  Returns A2A_ENOTCONV if some source
 * did not converge within max_iter (solutions hold the best iterates).  A non-finite value in
 * the sources: the host-pointer call rejects the call before any work (A2A_ENAN); the
 * device-pointer call fails that source only (info converged = 0), solves the others and
 * returns A2A_ENAN.  Requests of more than
 * 2048 sources run as consecutive batches of 2048 (the return code is the worst batch's). */
int a2a_solve_propagators(a2a_ctx *ctx, int clover_h, const double *sources_host, int nrhs, double kappa,
                          double c_sw, double tol, int prec, int max_iter, const double *x0_or_null,
                          double *solutions_host, a2a_solve_info *info);
int a2a_solve_propagators_dev(a2a_ctx *ctx, int clover_h, const double *sources_dev, int nrhs, double kappa,
                              double c_sw, double tol, int prec, int max_iter, const double *x0_dev_or_null,
                              double *solutions_dev, a2a_solve_info *info);

/* ---- contractions (Sec. 7, eq. stoop; Secs. 5 and 8 diagrams) ------------------------ */
/* O[t][a][b] = sum_{y in t} eta_a(y)^dag gamma_5 X_b(y) (complex [T][nrhs][nrhs], optional)
 * and corr[dt] (complex [T]) in the given mode.  nrhs >= 2 for the unbiased mode. */
int a2a_contract_pion_2pt(a2a_ctx *ctx, const a2a_geom *geom, const double *sources_host,
                          const double *solutions_host, int nrhs, int mode, double *corr, double *O_or_null);
int a2a_contract_pion_2pt_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *sources_dev,
                              const double *solutions_dev, int nrhs, int mode, double *corr_host,
                              double *O_host_or_null);
/* The same contraction for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc,
 * hipFree or allocating library routine.  Inputs and outputs are device pointers owned by the
 * caller: sources_dev and solutions_dev as for a2a_contract_pion_2pt_dev, corr_dev complex
 * [T], O_dev_or_null complex [T][nrhs][nrhs] (if null, O is kept in the scratch only).  The
 * partial sums of the timeslice products live in a static 32 MiB device array per GPU, held
 * from the library's first use on that GPU until the process ends; its device address is
 * looked up once per device in a2a_init.  Limit: 16 T nrhs^2 bytes (twice that without
 * O_dev) must fit in 32 MiB, i.e. nrhs <= 181 at T = 64 with O_dev, else A2A_EINVAL and
 * nothing is launched.  Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU (two contexts, two host threads) race and give wrong results.  The array keeps the
 * last call's contents; nothing in it needs to start at zero.  Returns after the stream has
 * finished the call's kernels. */
int a2a_contract_pion_2pt_noalloc(a2a_ctx *ctx, const a2a_geom *geom, const double *sources_dev,
                                  const double *solutions_dev, int nrhs, int mode, double *corr_dev,
                                  double *O_dev_or_null);
/* Zero-momentum pi-pi pieces from four disjoint noise groups (nrhs = 4m, 1 <= m <= 32):
 * diagrams complex [4][T] = D0 (direct), D1 (vacuum, unsubtracted), D2, D3 (single quark
 * loop through the four points, both orientations); vac_pieces complex [T] = the
 * timeslice loop L(t, t) of groups 1 and 2.  The total is D0 + D1 - D2 - D3 (Sec. 8).
 * pion_or_null (complex [T]): the unbiased pion correlator from the same O, so one pass
 * over (eta, X) serves both. */
int a2a_contract_pipi_2pt(a2a_ctx *ctx, const a2a_geom *geom, const double *sources_host,
                          const double *solutions_host, int nrhs, double *diagrams, double *vac_pieces,
                          double *pion_or_null);
int a2a_contract_pipi_2pt_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *sources_dev,
                              const double *solutions_dev, int nrhs, double *diagrams_host,
                              double *vac_pieces_host, double *pion_or_null);

/* ---- outer-product fill of the all-to-all propagator (Sec. 7, eq. Sfill) -------------- */
/* All three take device arrays in the canonical spinor layout: sol = solutions X_i, src =
 * sources eta_i, nrhs of each.  M = 12 X Y Z (spin-colour components of a timeslice).
 *
 * S (device, complex [M][M], owned by the caller) receives, for sink timeslice t and source
 * timeslice t_src, S(t, z; t_src, x)_{ab} = (1/nrhs) sum_i X_i(t, z)_a conj(eta_i(t_src, x)_b)
 * at row 12 z + a, column 12 x + b (z, x spatial site indices, x fastest; a = 3 spin + colour);
 * with dagger = 1 every 12 x 12 block is replaced by its spin-colour dagger (Sec. 7: the
 * paper's "S_s^dag fill").  Computed on the FP64 matrix cores. */
int a2a_fill_propagator_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *sol_dev, const double *src_dev,
                            int nrhs, int t_src, int t, int dagger, double *S_dev);
/* corr (host, complex [T]) = sum_{z, x} tr[S1(t, z; t_src, x) S2(t, z; t_src, x)^dag] for every t,
 * with S1 from (sol1, src1) and S2 from an independent set (sol2, src2) (the paper's
 * "sum_x sum_z tr S_s S_s^dag" with independent noise for the two propagators, Sec. 7).
 * _fill_ builds each product tile by tile on the matrix cores (cost ~ 8 T M^2 nrhs flop) without
 * storing S; _gram_ evaluates the same sum as (1/nrhs^2) sum_ij <eta1_i, eta2_j>_{t_src}
 * <X2_j, X1_i>_t (cost ~ 8 T M nrhs^2 flop).  The two agree to rounding. */
int a2a_contract_fill_2pt_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *sol1_dev, const double *src1_dev,
                              const double *sol2_dev, const double *src2_dev, int nrhs, int t_src, double *corr_host);
int a2a_contract_gram_2pt_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *sol1_dev, const double *src1_dev,
                              const double *sol2_dev, const double *src2_dev, int nrhs, int t_src, double *corr_host);

/* ---- dilution and momentum projection (Sec. 7 dilution; Sec. 5 momentum states) -------- */
/* out (device, canonical, nnoise * D sources) = every noise vector split into D pieces with
 * disjoint supports (scheme A2A_DILUTE_*; pieces of noise vector i are sources i D .. i D + D-1,
 * in the order of d).  The pieces of one noise vector sum to it. */
int a2a_dilute_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *noise_dev, int nnoise, int scheme,
                   double *out_dev);
/* Pion correlator projected onto momentum p = 2 pi (n_x / X, n_y / Y, n_z / Z) for each of the
 * nmom integer triples in moms (host, [nmom][3]):
 *   O_ab(t, p) = sum_{y in t} exp(-i p.y) eta_a(y)^dag gamma_5 X_b(y),
 *   corr[m][dt] = sum_t0 sum_{a, b} O_ab(t0 + dt, p) O_ba(t0, -p)
 * over pairs of sources from different noise vectors, the sources being the output of
 * a2a_dilute_dev with this scheme (nrhs = n D; sources a and b belong to noise vectors a / D
 * and b / D), normalised by 1 / (T n (n - 1)) (mode 0), or over all pairs without
 * normalisation (mode 3, e.g. for full dilution).  With time dilution (A2A_DILUTE_T, _TSC)
 * only the pieces on timeslice t enter O(t), which cuts the work by T.  corr: host complex
 * [nmom][T].  With A2A_DILUTE_NONE, p = 0 and mode 0 this is a2a_contract_pion_2pt's
 * unbiased correlator. */
int a2a_contract_pion_mom_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *sources_dev,
                              const double *solutions_dev, int nrhs, int scheme, int nmom, const int *moms,
                              int mode, double *corr_host);

/* ---- point-source propagators and the pi-pi diagrams that use them (Sec. 8) ------------ */
/* out (device, canonical, 12 sources) = the unit sources at the site (t0, x0[0..2] = x, y, z):
 * source k = 3 spin + colour is 1 in component k there and 0 elsewhere.  Solving them gives
 * the point propagator S_p(w) = S(w; t0, x0), column k = solution k.  A2A_EINVAL if the point
 * is outside the lattice. */
int a2a_point_sources_dev(a2a_ctx *ctx, const a2a_geom *geom, int t0, const int *x0, double *out_dev);
/* The pi-pi diagrams of Sec. 8 from point propagators (point_sol: the 12 solutions of
 * a2a_point_sources_dev at timeslice t0) and stochastic all-to-all propagators
 * S1 = (1/n1) sum_i X1_i eta1_i^dag and S2 = (1/n2) sum_j X2_j eta2_j^dag (eq. Sfill) of two
 * noise sets (pass the same set twice for the paper's one-set variant), for t = t0 + dt:
 *   pieces[0][dt] = Cp = sum_y tr[S_p(t, y) S_p(t, y)^dag]                    point pion
 *   pieces[1][dt] = Cs = sum_{z, x} tr[S1(t, z; t0, x) S2(t, z; t0, x)^dag]   all-to-all pion
 *   pieces[2][dt] = L  = sum_{z, y} tr[S1(t, z; t, y) S2(t, z; t, y)^dag]     loop at t
 *   diagrams[0][dt] = Cp Cs,  diagrams[1][dt] = L Cp(0)  (both unsubtracted)
 *   diagrams[2][dt] = sum_{x, y, z} tr[S_p(t0, x)^dag S1(t0, x; t, z) S2(t, y; t, z)^dag S_p(t, y)]
 *   diagrams[3][dt] = conj(diagrams[2][dt])
 * (daggers on spin and colour only; total D0 + D1 - D2 - D3 after the ensemble subtractions).
 * Evaluated from timeslice Gram matrices of the inputs (FP64, no propagator is stored; work
 * ~ 8 T 12 X Y Z (n1 n2 + 12 (n1 + n2)) flop).  All arrays are canonical device spinors;
 * diagrams (complex [4][T]) and pieces (complex [3][T], or NULL) are host arrays.  Temporary
 * device memory ~ 16 T n1 n2 x (2 + a chunk factor) bytes.  A2A_EINVAL for n1 or n2 < 1 or t0
 * outside [0, T); A2A_ENOMEM when the temporaries do not fit the budget. */
int a2a_contract_pipi_mixed_dev(a2a_ctx *ctx, const a2a_geom *geom, const double *point_sol_dev, int t0,
                                const double *src1_dev, const double *sol1_dev, int n1, const double *src2_dev,
                                const double *sol2_dev, int n2, double *diagrams_host, double *pieces_host);

/* ---- synthetic inputs ---------------------------------------------------------------- */
/* Complex-Z2 noise (Sec. 7 "Z2 noise", here (+-1 +- i)/sqrt 2) written to a canonical
 * device array of nsrc sources: component k of the flattened array (global source index
 * src_offset + s) uses h = splitmix64(seed * 2^48 + k), real sign from bit 0 and
 * imaginary sign from bit 1 of h. */
int a2a_z2_noise_dev(a2a_ctx *ctx, const a2a_geom *geom, unsigned long long seed, long long src_offset, int nsrc,
                     double *out_dev);

/* ---- serving engine: continuous batching of propagator requests ---------------------- */
/* policy_json keys (all optional): "max_slots" (RHS resident at once), "max_queue",
 * "check_every".  Requests of any resident lattice, kappa and precision share the device;
 * a request is admitted when its memory fits the context's HBM budget, and its sources
 * join the running batch at the next step.  sources_dev / solutions_dev must stay valid
 * until a2a_engine_poll reports the ticket done.  Each request runs with the inner method
 * (option "solver") set when it was submitted; unlike a2a_solve_propagators, the engine has
 * no CGNR fallback: a source whose BiCGStab breaks down repeatedly fails its request with
 * A2A_EBREAKDOWN (its sources share lane groups with sources still iterating), and the caller
 * may submit it again with "solver" = A2A_SOLVER_CGNR. */
int a2a_engine_create(a2a_ctx *ctx, const char *policy_json, a2a_engine **eng);
int a2a_engine_submit(a2a_engine *eng, int clover_h, double kappa, const double *sources_dev, int nsrc, double tol,
                      int prec, int max_iter, double *solutions_dev, long long *ticket);
/* Run `iters` solver iterations for every active slot (all lattices and precisions), then
 * admit queued requests and retire converged ones.  *active receives the number of active
 * RHS after the step (may be NULL). */
int a2a_engine_step(a2a_engine *eng, int iters, int *active);
/* done: 0 queued or running, 1 finished (info filled, nsrc records), -1 failed */
int a2a_engine_poll(a2a_engine *eng, long long ticket, int *done, a2a_solve_info *info);
int a2a_engine_cancel(a2a_engine *eng, long long ticket);
int a2a_engine_destroy(a2a_engine *eng);

/* ---- instrumentation ------------------------------------------------------------------ */
/* With option "kernel_timing" = 1 the solver brackets every inner-solver launch with HIP
 * events on the context stream.  For kernel class `name` ("schur1": hop to even sites with
 * the A_ee^{-1} epilogue; "schur2": hop to odd sites with the A_oo, axpy and dot-product
 * epilogue; "xr", "p", "s": the BiCGStab updates of x and r, of p, of s (CGNR's x/r and p
 * updates count as "xr" and "p"); "blas": the three updates together) returns the launches, their total
 * milliseconds and their total algorithmic bytes (links and clover once per site, each
 * spinor stream once per right-hand side) since the last reset; resets if reset != 0. */
int a2a_kernel_stats(a2a_ctx *ctx, const char *name, long long *launches, double *total_ms, double *alg_bytes,
                     int reset);

#ifdef __cplusplus
}
#endif

#endif /* A2A_H */
