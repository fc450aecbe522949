"""ctypes binding of liba2a (C ABI in include/a2a.h): argument marshalling only.

Every computation runs in the HIP library; if ``_build/liba2a.so`` is missing this module
raises on first use (there is no fallback).  Method names follow the C functions without the
``a2a_`` prefix.  Host-array methods take and return numpy complex128 arrays in the canonical
layouts; ``*_dev`` methods take torch tensors on the GPU (complex128, or float64 with a
trailing dimension of 2) and run on the stream the context was created with.

    links    (T, Z, Y, X, 4, 3, 3)      spinors  (nsrc, T, Z, Y, X, 4, 3)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "liba2a.so")

OK, EINVAL, ENOMEM, ENOTCONV, EBREAKDOWN, ENAN, EHANDLE, EDEVICE, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32, F16_F32, BF16_F32 = 0, 1, 2, 3
OP_FULL_D, OP_SCHUR, OP_HOP_EO, OP_HOP_OE = 0, 1, 2, 3
PION_UNBIASED, PION_ALL_PAIRS = 0, 1
SOLVER_BICGSTAB, SOLVER_CGNR = 0, 1
DILUTE_NONE, DILUTE_T, DILUTE_SC, DILUTE_TSC = 0, 1, 2, 3
PREC_NAMES = {F64: "f64", F32: "f32", F16_F32: "f16/f32", BF16_F32: "bf16/f32"}
ERR_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ENOTCONV: "ENOTCONV", EBREAKDOWN: "EBREAKDOWN", ENAN: "ENAN",
             EHANDLE: "EHANDLE", EDEVICE: "EDEVICE", EAGAIN: "EAGAIN"}


class A2AError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("t_bc", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("il_width", ctypes.c_int), ("brick", ctypes.c_int * 3), ("rhs_block", ctypes.c_int),
                ("rhs_block64", ctypes.c_int), ("ms_schur", ctypes.c_double), ("ms_schur64", ctypes.c_double),
                ("candidates", ctypes.c_int), ("xcd_slab", ctypes.c_int), ("brick64", ctypes.c_int * 3),
                ("xcd64", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["brick"] = list(self.brick)
        d["brick64"] = list(self.brick64)
        return d


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("restarts", ctypes.c_int), ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("solver", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
P, I, D, SZ, LL, ULL = (ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_longlong,
                        ctypes.c_ulonglong)
_SIG = {
    "a2a_init": (I, [ctypes.POINTER(P), I, SZ, P]),
    "a2a_finalize": (I, [P]),
    "a2a_last_error": (ctypes.c_char_p, [P]),
    "a2a_set_option": (I, [P, ctypes.c_char_p, D]),
    "a2a_mem_in_use": (SZ, [P]),
    "a2a_trim": (I, [P, ctypes.POINTER(SZ)]),
    "a2a_load_gauge": (I, [P, ctypes.POINTER(Geom), P, ctypes.POINTER(I)]),
    "a2a_load_gauge_dev": (I, [P, ctypes.POINTER(Geom), P, ctypes.POINTER(I)]),
    "a2a_load_clover": (I, [P, I, D, ctypes.POINTER(I)]),
    "a2a_unload": (I, [P, I]),
    "a2a_dslash_clover": (I, [P, I, D, I, I, I, P, P, I]),
    "a2a_dslash_clover_dev": (I, [P, I, D, I, I, I, P, P, I]),
    "a2a_bench_stencil": (I, [P, I, D, I, I, I, I, ctypes.POINTER(D)]),
    "a2a_autotune": (I, [P, I, D, I, I, P]),
    "a2a_brick_choices": (I, [ctypes.POINTER(Geom), P, I]),
    "a2a_solve_propagators": (I, [P, I, P, I, D, D, D, I, I, P, P, P]),
    "a2a_solve_propagators_dev": (I, [P, I, P, I, D, D, D, I, I, P, P, P]),
    "a2a_contract_pion_2pt": (I, [P, ctypes.POINTER(Geom), P, P, I, I, P, P]),
    "a2a_contract_pion_2pt_dev": (I, [P, ctypes.POINTER(Geom), P, P, I, I, P, P]),
    "a2a_contract_pion_2pt_noalloc": (I, [P, ctypes.POINTER(Geom), P, P, I, I, P, P]),
    "a2a_contract_pipi_2pt": (I, [P, ctypes.POINTER(Geom), P, P, I, P, P, P]),
    "a2a_contract_pipi_2pt_dev": (I, [P, ctypes.POINTER(Geom), P, P, I, P, P, P]),
    "a2a_z2_noise_dev": (I, [P, ctypes.POINTER(Geom), ULL, LL, I, P]),
    "a2a_fill_propagator_dev": (I, [P, ctypes.POINTER(Geom), P, P, I, I, I, I, P]),
    "a2a_dilute_dev": (I, [P, ctypes.POINTER(Geom), P, I, I, P]),
    "a2a_contract_pion_mom_dev": (I, [P, ctypes.POINTER(Geom), P, P, I, I, I, P, I, P]),
    "a2a_contract_fill_2pt_dev": (I, [P, ctypes.POINTER(Geom), P, P, P, P, I, I, P]),
    "a2a_contract_gram_2pt_dev": (I, [P, ctypes.POINTER(Geom), P, P, P, P, I, I, P]),
    "a2a_point_sources_dev": (I, [P, ctypes.POINTER(Geom), I, P, P]),
    "a2a_contract_pipi_mixed_dev": (I, [P, ctypes.POINTER(Geom), P, I, P, P, I, P, P, I, P, P]),
    "a2a_engine_create": (I, [P, ctypes.c_char_p, ctypes.POINTER(P)]),
    "a2a_engine_submit": (I, [P, I, D, P, I, D, I, I, P, ctypes.POINTER(LL)]),
    "a2a_engine_step": (I, [P, I, ctypes.POINTER(I)]),
    "a2a_engine_poll": (I, [P, LL, ctypes.POINTER(I), P]),
    "a2a_engine_cancel": (I, [P, LL]),
    "a2a_engine_destroy": (I, [P]),
    "a2a_kernel_stats": (I, [P, ctypes.c_char_p, ctypes.POINTER(LL), ctypes.POINTER(D), ctypes.POINTER(D), I]),
}
EXPORTS = tuple(_SIG)


def lib():
    """Load liba2a.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1405_4524_amd.build` first")
        # torch ships its own HIP runtime (soname libamdhip64.so.7); loading it first makes
        # liba2a bind to that same runtime, so the process has one HIP runtime and torch's
        # device memory and streams are usable by the library.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _np_c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(P)


def _tptr(t):
    """data pointer of a contiguous torch tensor on the GPU (complex128 or float64)."""
    import torch

    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if t.dtype not in (torch.complex128, torch.float64):
        raise ValueError("expected complex128 or float64")
    return ctypes.c_void_p(t.data_ptr())


def geom(dims, t_bc):
    g = Geom()
    for i in range(4):
        g.dims[i] = int(dims[i])
    g.t_bc = int(t_bc)
    return g


def dims_of_spinor(a):
    """(X, Y, Z, T) of a (nsrc, T, Z, Y, X, 4, 3) array or tensor."""
    s = tuple(a.shape)
    if len(s) >= 7 and s[-1] == 2:
        s = s[:-1]
    return (s[-3], s[-4], s[-5], s[-6])


class Engine:
    """Continuous-batching engine of one context (a2a_engine_*)."""

    def __init__(self, ctx, policy_json=""):
        self.ctx = ctx
        self._e = P()
        ctx._chk(lib().a2a_engine_create(ctx._c, policy_json.encode(), ctypes.byref(self._e)))

    def submit(self, clover_h, kappa, sources_dev, nsrc, tol, prec, max_iter, solutions_dev):
        t = LL()
        self.ctx._chk(lib().a2a_engine_submit(self._e, int(clover_h), float(kappa), _tptr(sources_dev), int(nsrc),
                                              float(tol), int(prec), int(max_iter), _tptr(solutions_dev),
                                              ctypes.byref(t)))
        return t.value

    def step(self, iters):
        a = I()
        self.ctx._chk(lib().a2a_engine_step(self._e, int(iters), ctypes.byref(a)))
        return a.value

    def poll(self, ticket, nsrc):
        done = I()
        info = (SolveInfo * max(1, nsrc))()
        rc = lib().a2a_engine_poll(self._e, int(ticket), ctypes.byref(done), info)
        return done.value, [x.as_dict() for x in info[:nsrc]], rc

    def cancel(self, ticket):
        self.ctx._chk(lib().a2a_engine_cancel(self._e, int(ticket)))

    def destroy(self):
        if self._e:
            lib().a2a_engine_destroy(self._e)
            self._e = P()


class Context:
    """An a2a context on one GPU (a2a_init ... a2a_finalize)."""

    def __init__(self, device=0, hbm_budget=0, stream=None):
        self._c = P()
        s = P(stream) if stream else P()
        rc = lib().a2a_init(ctypes.byref(self._c), int(device), ctypes.c_size_t(int(hbm_budget)), s)
        if rc:
            raise A2AError(rc, "a2a_init failed")

    # ---- plumbing
    def _chk(self, rc, allow=()):
        if rc and rc not in allow:
            raise A2AError(rc, self.last_error())
        return rc

    def finalize(self):
        if self._c:
            lib().a2a_finalize(self._c)
            self._c = P()

    close = finalize

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.finalize()

    def last_error(self):
        m = lib().a2a_last_error(self._c)
        return m.decode() if m else ""

    def set_option(self, key, value):
        self._chk(lib().a2a_set_option(self._c, key.encode(), float(value)))

    def mem_in_use(self):
        return int(lib().a2a_mem_in_use(self._c))

    def trim(self):
        """Return cached device buffers to the device; returns their bytes."""
        n = SZ()
        self._chk(lib().a2a_trim(self._c, ctypes.byref(n)))
        return int(n.value)

    # ---- fields
    def load_gauge(self, links, t_bc):
        links, p = _np_c128(links)
        T, Z, Y, X = links.shape[:4]
        g = geom((X, Y, Z, T), t_bc)
        h = I()
        self._chk(lib().a2a_load_gauge(self._c, ctypes.byref(g), p, ctypes.byref(h)))
        return h.value

    def load_gauge_dev(self, links_t, dims, t_bc):
        g = geom(dims, t_bc)
        h = I()
        self._chk(lib().a2a_load_gauge_dev(self._c, ctypes.byref(g), _tptr(links_t), ctypes.byref(h)))
        return h.value

    def load_clover(self, gauge_h, csw):
        h = I()
        self._chk(lib().a2a_load_clover(self._c, int(gauge_h), float(csw), ctypes.byref(h)))
        return h.value

    def unload(self, handle):
        self._chk(lib().a2a_unload(self._c, int(handle)))

    # ---- operators
    def dslash_clover(self, clover_h, kappa, psi, op=OP_FULL_D, dagger=False, prec=F64):
        single = psi.ndim == 6
        x, p = _np_c128(psi[None] if single else psi)
        out = np.empty_like(x)
        self._chk(lib().a2a_dslash_clover(self._c, int(clover_h), float(kappa), int(op), int(bool(dagger)), int(prec),
                                          p, out.ctypes.data_as(P), x.shape[0]))
        return out[0] if single else out

    def dslash_clover_dev(self, clover_h, kappa, in_t, out_t, nrhs, op=OP_FULL_D, dagger=False, prec=F64):
        self._chk(lib().a2a_dslash_clover_dev(self._c, int(clover_h), float(kappa), int(op), int(bool(dagger)),
                                              int(prec), _tptr(in_t), _tptr(out_t), int(nrhs)))

    def bench_stencil(self, clover_h, kappa, op, prec, nrhs, reps):
        ms = D()
        self._chk(lib().a2a_bench_stencil(self._c, int(clover_h), float(kappa), int(op), int(prec), int(nrhs),
                                          int(reps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, clover_h, kappa, prec, nrhs):
        """Tune (or look up) the launch configuration of this workload; returns it as a dict:
        il_width, brick [by, bz, bt], rhs_block, rhs_block64, ms_schur, ms_schur64, candidates."""
        r = TuneResult()
        self._chk(lib().a2a_autotune(self._c, int(clover_h), float(kappa), int(prec), int(nrhs), ctypes.byref(r)))
        return r.as_dict()

    @staticmethod
    def brick_choices(dims, t_bc=-1):
        """The stencil bricks (by, bz, bt) the tuner may choose for a lattice, default first."""
        g = geom(dims, t_bc)
        out = (I * 48)()
        n = lib().a2a_brick_choices(ctypes.byref(g), out, 16)
        if n < 0:
            raise A2AError(n, "bad lattice geometry")
        return [tuple(out[3 * k:3 * k + 3]) for k in range(n)]

    # ---- solves
    def solve_propagators(self, clover_h, sources, kappa, csw, tol=1e-10, prec=F64, max_iter=100000, x0=None,
                          allow=(ENOTCONV,)):
        single = sources.ndim == 6
        s, ps = _np_c128(sources[None] if single else sources)
        n = s.shape[0]
        X = np.empty_like(s)
        info = (SolveInfo * n)()
        px0 = None
        if x0 is not None:
            x0a, px0 = _np_c128(x0[None] if single else x0)
        rc = lib().a2a_solve_propagators(self._c, int(clover_h), ps, n, float(kappa), float(csw), float(tol),
                                         int(prec), int(max_iter), px0, X.ctypes.data_as(P), info)
        self._chk(rc, allow)
        inf = [x.as_dict() for x in info]
        return (X[0] if single else X), inf, rc

    def solve_propagators_dev(self, clover_h, src_t, sol_t, nrhs, kappa, csw, tol=1e-10, prec=F64, max_iter=100000,
                              x0_t=None, allow=(ENOTCONV,)):
        info = (SolveInfo * nrhs)()
        rc = lib().a2a_solve_propagators_dev(self._c, int(clover_h), _tptr(src_t), int(nrhs), float(kappa),
                                             float(csw), float(tol), int(prec), int(max_iter),
                                             _tptr(x0_t) if x0_t is not None else None, _tptr(sol_t), info)
        self._chk(rc, allow)
        return [x.as_dict() for x in info], rc

    # ---- contractions
    def contract_pion_2pt(self, sources, solutions, t_bc=-1, mode=PION_UNBIASED, want_O=True):
        s, ps = _np_c128(sources)
        x, px = _np_c128(solutions)
        n = s.shape[0]
        g = geom(dims_of_spinor(s), t_bc)
        T = g.dims[3]
        corr = np.empty(T, np.complex128)
        O = np.empty((T, n, n), np.complex128) if want_O else None
        self._chk(lib().a2a_contract_pion_2pt(self._c, ctypes.byref(g), ps, px, n, int(mode),
                                              corr.ctypes.data_as(P), O.ctypes.data_as(P) if want_O else None))
        return corr, O

    def contract_pion_2pt_dev(self, src_t, sol_t, nrhs, dims, t_bc=-1, mode=PION_UNBIASED, want_O=False):
        g = geom(dims, t_bc)
        T = g.dims[3]
        corr = np.empty(T, np.complex128)
        O = np.empty((T, nrhs, nrhs), np.complex128) if want_O else None
        self._chk(lib().a2a_contract_pion_2pt_dev(self._c, ctypes.byref(g), _tptr(src_t), _tptr(sol_t), int(nrhs),
                                                  int(mode), corr.ctypes.data_as(P),
                                                  O.ctypes.data_as(P) if want_O else None))
        return corr, O

    def contract_pion_2pt_noalloc(self, src_t, sol_t, nrhs, dims, corr_t, O_t=None, t_bc=-1, mode=PION_UNBIASED):
        """The allocation-free contraction: corr_t (complex128 [T]) and O_t (complex128 [T][n][n] or
        None) are caller-owned device tensors; the library allocates nothing."""
        g = geom(dims, t_bc)
        self._chk(lib().a2a_contract_pion_2pt_noalloc(self._c, ctypes.byref(g), _tptr(src_t), _tptr(sol_t),
                                                      int(nrhs), int(mode), _tptr(corr_t),
                                                      _tptr(O_t) if O_t is not None else None))

    def contract_pipi_2pt(self, sources, solutions, t_bc=-1, want_pion=False):
        """(diagrams[4, T], vac[T]) and, with want_pion, also the unbiased pion correlator."""
        s, ps = _np_c128(sources)
        x, px = _np_c128(solutions)
        n = s.shape[0]
        g = geom(dims_of_spinor(s), t_bc)
        T = g.dims[3]
        d = np.empty((4, T), np.complex128)
        v = np.empty(T, np.complex128)
        pc = np.empty(T, np.complex128) if want_pion else None
        self._chk(lib().a2a_contract_pipi_2pt(self._c, ctypes.byref(g), ps, px, n, d.ctypes.data_as(P),
                                              v.ctypes.data_as(P), pc.ctypes.data_as(P) if want_pion else None))
        return (d, v, pc) if want_pion else (d, v)

    def contract_pipi_2pt_dev(self, src_t, sol_t, nrhs, dims, t_bc=-1, want_pion=False):
        g = geom(dims, t_bc)
        T = g.dims[3]
        d = np.empty((4, T), np.complex128)
        v = np.empty(T, np.complex128)
        pc = np.empty(T, np.complex128) if want_pion else None
        self._chk(lib().a2a_contract_pipi_2pt_dev(self._c, ctypes.byref(g), _tptr(src_t), _tptr(sol_t), int(nrhs),
                                                  d.ctypes.data_as(P), v.ctypes.data_as(P),
                                                  pc.ctypes.data_as(P) if want_pion else None))
        return (d, v, pc) if want_pion else (d, v)

    # ---- inputs
    def z2_noise_dev(self, dims, seed, src_offset, nsrc, out_t):
        g = geom(dims, 1)
        self._chk(lib().a2a_z2_noise_dev(self._c, ctypes.byref(g), ctypes.c_ulonglong(int(seed)),
                                         ctypes.c_longlong(int(src_offset)), int(nsrc), _tptr(out_t)))

    # ---- outer-product fill (device tensors in the canonical spinor layout)
    def fill_propagator_dev(self, sol_t, src_t, nrhs, dims, t_src, t, S_t, dagger=False, t_bc=-1):
        g = geom(dims, t_bc)
        self._chk(lib().a2a_fill_propagator_dev(self._c, ctypes.byref(g), _tptr(sol_t), _tptr(src_t), int(nrhs),
                                                int(t_src), int(t), int(bool(dagger)), _tptr(S_t)))

    def contract_fill_2pt_dev(self, sol1_t, src1_t, sol2_t, src2_t, nrhs, dims, t_src, t_bc=-1, method="fill"):
        g = geom(dims, t_bc)
        corr = np.empty(dims[3], np.complex128)
        f = lib().a2a_contract_fill_2pt_dev if method == "fill" else lib().a2a_contract_gram_2pt_dev
        self._chk(f(self._c, ctypes.byref(g), _tptr(sol1_t), _tptr(src1_t), _tptr(sol2_t), _tptr(src2_t), int(nrhs),
                    int(t_src), corr.ctypes.data_as(P)))
        return corr

    # ---- dilution and momentum projection (device tensors in the canonical spinor layout)
    def dilute_dev(self, noise_t, nnoise, dims, scheme, out_t, t_bc=-1):
        g = geom(dims, t_bc)
        self._chk(lib().a2a_dilute_dev(self._c, ctypes.byref(g), _tptr(noise_t), int(nnoise), int(scheme),
                                       _tptr(out_t)))

    def contract_pion_mom_dev(self, src_t, sol_t, nrhs, dims, moms, scheme=DILUTE_NONE, mode=PION_UNBIASED, t_bc=-1):
        g = geom(dims, t_bc)
        m = np.ascontiguousarray(np.asarray(moms, dtype=np.int32).reshape(-1, 3))
        corr = np.empty((m.shape[0], dims[3]), np.complex128)
        self._chk(lib().a2a_contract_pion_mom_dev(self._c, ctypes.byref(g), _tptr(src_t), _tptr(sol_t), int(nrhs),
                                                  int(scheme), m.shape[0], m.ctypes.data_as(P), int(mode),
                                                  corr.ctypes.data_as(P)))
        return corr

    # ---- point-source propagators and the pi-pi diagrams that use them
    def point_sources_dev(self, dims, t0, x0, out_t, t_bc=-1):
        g = geom(dims, t_bc)
        x = (ctypes.c_int * 3)(*[int(v) for v in x0])
        self._chk(lib().a2a_point_sources_dev(self._c, ctypes.byref(g), int(t0), x, _tptr(out_t)))

    def contract_pipi_mixed_dev(self, point_sol_t, t0, src1_t, sol1_t, n1, src2_t, sol2_t, n2, dims, t_bc=-1):
        """(diagrams[4, T] = D0..D3, pieces[3, T] = point pion, all-to-all pion, loop)."""
        g = geom(dims, t_bc)
        T = dims[3]
        d = np.empty((4, T), np.complex128)
        pc = np.empty((3, T), np.complex128)
        self._chk(lib().a2a_contract_pipi_mixed_dev(self._c, ctypes.byref(g), _tptr(point_sol_t), int(t0),
                                                    _tptr(src1_t), _tptr(sol1_t), int(n1), _tptr(src2_t),
                                                    _tptr(sol2_t), int(n2), d.ctypes.data_as(P),
                                                    pc.ctypes.data_as(P)))
        return d, pc

    # ---- engine / instrumentation
    def engine_create(self, policy_json=""):
        return Engine(self, policy_json)

    def kernel_stats(self, name, reset=False):
        """(launches, total ms, total algorithmic bytes) of a timed kernel class."""
        n = LL()
        ms = D()
        by = D()
        self._chk(lib().a2a_kernel_stats(self._c, name.encode(), ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(by), int(bool(reset))))
        return n.value, ms.value, by.value
