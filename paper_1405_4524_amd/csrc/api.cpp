// api.cpp -- the extern "C" entry points of liba2a (declared in include/a2a.h) and the
// continuous-batching serving engine.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <mutex>

#include "a2a_contract.h"
#include "runtime.h"

using namespace a2a;

struct a2a_ctx {
  Ctx c;
};

static int autotune_cfg(Ctx* c, int clover_h, double kappa, int prec, int nrhs, TuneCfg* out,
                        a2a_tune_result* res);
static void tune_load(Ctx* c);

namespace {

constexpr int SID_CAP = 4096;

int check_prec(int prec) { return (prec >= 0 && prec <= 3) ? A2A_OK : A2A_EINVAL; }

long long volume_of(const Geo& g) { return 2LL * g.hv; }

// allocate the arenas and stable id of one slot
int slot_alloc(Ctx* c, Slot* s, int prec, long hv, int nblk, int nlo, int nhi) {
  A2A_TRY(c->alloc_sid(nblk, &s->sid));
  const size_t bl = [&] {
    size_t b = prec == 0 ? SpinorF<double>::bytes(hv)
               : prec == 1 ? SpinorF<float>::bytes(hv)
               : prec == 2 ? SpinorF<_Float16>::bytes(hv)
                           : SpinorF<bf16_t>::bytes(hv);
    return (b + 255) & ~(size_t)255;
  }();
  const size_t bh = (SpinorF<double>::bytes(hv) + 255) & ~(size_t)255;
  s->lo_stride = bl;
  s->hi_stride = bh;
  void* p = nullptr;
  if (nlo) {
    int rc = c->dalloc(&p, bl * nlo);
    if (rc) {
      c->free_sid(s->sid);
      s->sid = -1;
      return rc;
    }
    s->lo = (char*)p;
    s->lo_alloc = s->lo;
  }
  s->lss = 16;
  s->lcs = 16LL * hv;
  s->lss_x = 16;
  s->lxoff = 0;
  if (nhi) {
    int rc = c->dalloc(&p, bh * nhi);
    if (rc) {
      c->dfree(s->lo_alloc);
      s->lo = s->lo_alloc = nullptr;
      c->free_sid(s->sid);
      s->sid = -1;
      return rc;
    }
    s->hi = (char*)p;
  }
  return A2A_OK;
}

void slot_free(Ctx* c, Slot* s) {
  c->dfree(s->lo_alloc);
  c->dfree(s->hi);
  s->lo = s->hi = s->lo_alloc = s->il_base = nullptr;
  if (s->sid >= 0) c->free_sid(s->sid);
  s->sid = -1;
}

// Interleaved inner layout (FP16 / BF16 storage): consecutive slots form groups of up to
// IL_LANES lanes (tiles of 16) sharing one arena [vector][site][tile][3 chunks][16 lanes] of
// 16-byte chunks.  Lane 0 of each group owns the arena.  Groups never span calls or requests,
// so a group's arena is freed together with all of its slots.
constexpr int IL_MAX = IL_LANES;

bool use_interleave(const Ctx* c, int prec) { return c->interleave && (prec == 2 || prec == 3); }

int il_alloc(Ctx* c, Slot* slots, int n, long hv, int nlo, int width) {
  for (int g0 = 0; g0 < n; g0 += width) {
    const int m = std::min(width, n - g0);
    const int nt = (m + 15) / 16;
    const size_t vs = ((size_t)hv * nt * 768 + 255) & ~(size_t)255;
    void* p = nullptr;
    A2A_TRY(c->dalloc(&p, vs * nlo));
    for (int j = 0; j < m; ++j) {
      Slot& s = slots[g0 + j];
      const int tile = j / 16, lane = j % 16;
      s.lo = (char*)p + tile * 768 + lane * 16;
      s.lo_alloc = j == 0 ? (char*)p : nullptr;
      s.lo_stride = vs;
      s.lss = 768LL * nt;
      s.lcs = 256;
      s.lss_x = s.lss;  // the inner iterate in the storage format, laid out like the other vectors
      s.lxoff = 0;
      s.il_base = (char*)p;
      s.il_nt = nt;
      s.il_lane = j;
    }
  }
  return A2A_OK;
}

// arenas of n slots of one operator: per slot, or interleaved groups for FP16 / BF16.  Whole
// 16-lane tiles go to interleaved groups; a remainder of at least IL_REM_MIN sources gets a
// tile of its own, a smaller one stays per slot (a tile costs the same whatever its fill: the
// per-thread stencil is cheaper per RHS below about 12 of 16 lanes).
constexpr int IL_REM_MIN = 12;

// ilw: RHS per interleaved group (16, 32 or 48; 0 = the context's option)
int slots_alloc(Ctx* c, Slot* slots, int n, int prec, long hv, int nblk, int nlo, int nhi, int ilw = 0) {
  const bool il = use_interleave(c, prec) && nlo > 0;
  int width = ilw > 0 ? ilw : c->il_width;
  if (width != 16 && width != 32) width = IL_MAX;
  int n_il = 0;
  if (il) {
    n_il = n / 16 * 16;
    if (n - n_il >= IL_REM_MIN) n_il = n;
  }
  int rc = A2A_OK;
  int k = 0;
  for (; k < n && !rc; ++k) rc = slot_alloc(c, &slots[k], prec, hv, nblk, k < n_il ? 0 : nlo, nhi);
  if (!rc && n_il > 0) rc = il_alloc(c, slots, n_il, hv, nlo, width);
  if (rc)
    for (int j = 0; j < k; ++j) slot_free(c, &slots[j]);
  return rc;
}

int effective_R(Ctx* c, int prec) {
  int R = c->rhs_block;
  if (R != 1 && R != 2 && R != 4) R = 1;
  if (prec == 0 && R > 2) R = 2;
  return R;
}

// resolve clover handle -> (gauge, clover, kappa op with prec fields, links in prec and FP64)
int resolve_op(Ctx* c, int clover_h, double kappa, int prec, GaugeField** gf, CloverField** cf, KappaOp** kop) {
  *cf = c->clover(clover_h);
  if (!*cf) return c->fail(A2A_EHANDLE, "unknown clover handle " + std::to_string(clover_h));
  *gf = c->gauge((*cf)->gauge);
  if (!*gf) return c->fail(A2A_EHANDLE, "clover handle refers to an unloaded gauge field");
  if (!(kappa > 0.0) || !std::isfinite(kappa)) return c->fail(A2A_EINVAL, "kappa must be positive and finite");
  void *u0, *u1;
  A2A_TRY(c->gauge_links(*gf, 0, &u0, &u1));
  A2A_TRY(c->gauge_links(*gf, prec, &u0, &u1));
  A2A_TRY(c->kappa_op(*cf, kappa, prec, kop));
  if (use_interleave(c, prec) && c->mfma) {  // fields of the matrix-core stencil
    A2A_TRY(c->hop_links(*gf, prec));
    A2A_TRY(c->clover_full(*kop, prec, (*gf)->g.hv));
  }
  return A2A_OK;
}

// Sources whose BiCGStab broke down repeatedly start again with CG on the normal equations
// (whose residual decreases monotonically and which needs no bi-orthogonality), from the
// iterate the first pass wrote to their solution buffer when it is finite, else from zero.
// Runs after the first pass has finished, so no slot is live in two solvers.
static int cgnr_fallback(Ctx* c, Solver& first, std::vector<Slot>& slots, int clover_h, double kappa, KappaOp* kop,
                         GaugeField* gf) {
  std::vector<int> idx;
  for (int i = 0; i < (int)slots.size(); ++i)
    if (slots[i].state == SS_FAIL && slots[i].err == A2A_EBREAKDOWN && slots[i].iters < slots[i].max_iter)
      idx.push_back(i);
  if (idx.empty()) return A2A_OK;
  A2A_TRY(c->sync());
  Solver sv(c, first.prec, first.R);
  sv.method = SOLVER_CGNR;
  const int op = sv.op_index(clover_h, kappa, kop, gf);
  for (int k = 0; k < (int)idx.size(); ++k) {
    Slot& s = slots[idx[k]];
    s.op = op;
    s.x0 = std::isfinite(s.info.true_rel_residual) ? s.sol : nullptr;
    s.state = SS_NEW;
    s.err = A2A_OK;
    s.restarts = s.stagn = 0;
    s.last_r64 = INFINITY;
    sv.add_slot(&s);
  }
  std::vector<int> all(idx.size());
  for (int k = 0; k < (int)idx.size(); ++k) all[k] = k;
  A2A_TRY(sv.setup(all));
  std::vector<int> early;
  for (int k : all)
    if (sv.live[k]->state == SS_RUN && sv.live[k]->last_r64 <= sv.live[k]->target) early.push_back(k);
  if (!early.empty()) {
    A2A_TRY(sv.finalize(early));
    for (int k : early) sv.live[k]->state = sv.live[k]->info.converged ? SS_DONE : SS_RUN;
  }
  return sv.run_until_done(1 << 30);
}

static int solve_batch(Ctx* c, int clover_h, const double* src, int nrhs, double kappa, double csw, double tol,
                       int prec, int max_iter, const double* x0, double* sol, a2a_solve_info* info) {
  if (nrhs <= 0) return c->fail(A2A_EINVAL, "nrhs must be positive");
  if (!(tol > 0.0)) return c->fail(A2A_EINVAL, "tol must be positive");
  if (max_iter <= 0) return c->fail(A2A_EINVAL, "max_iter must be positive");
  if (check_prec(prec)) return c->fail(A2A_EINVAL, "unknown precision mode");
  if (!src || !sol) return c->fail(A2A_EINVAL, "null source or solution pointer");
  GaugeField* gf;
  CloverField* cf;
  KappaOp* kop;
  A2A_TRY(resolve_op(c, clover_h, kappa, prec, &gf, &cf, &kop));
  if (std::fabs(csw - cf->csw) > 1e-12 * std::max(1.0, std::fabs(cf->csw)))
    return c->fail(A2A_EINVAL, "c_sw does not match the clover handle");
  const long hv = gf->g.hv;
  const long long V = volume_of(gf->g);
  TuneCfg tc{};
  if (c->autotune) A2A_TRY(autotune_cfg(c, clover_h, kappa, prec, nrhs, &tc, nullptr));
  const int R = tc.R ? tc.R : effective_R(c, prec);
  Solver sv(c, prec, R);
  if (tc.R64) sv.R64 = tc.R64;
  if (tc.slab >= 0) sv.mfma_slab = tc.slab;
  if (tc.by > 0) {
    sv.by = tc.by;
    sv.bz = tc.bz;
    sv.bt = tc.bt;
  }
  sv.by64 = tc.by64;
  sv.bz64 = tc.bz64;
  sv.bt64 = tc.bt64;
  sv.xcd_sub = tc.xcd64;
  sv.method = c->solver;
  const int op = sv.op_index(clover_h, kappa, kop, gf);
  std::vector<Slot> slots(nrhs);
  int rc = A2A_OK;
  const double t0 = now_seconds();
  for (int i = 0; i < nrhs && !rc; ++i) {
    Slot& s = slots[i];
    s.op = op;
    s.src = src + (size_t)i * 24 * V;
    s.sol = sol + (size_t)i * 24 * V;
    s.x0 = x0 ? x0 + (size_t)i * 24 * V : nullptr;
    s.tol = tol;
    s.max_iter = max_iter;
    s.t_submit = t0;
  }
  rc = slots_alloc(c, slots.data(), nrhs, prec, hv, sv.ops[op].nblk, NVEC_LO, NVEC_HI, tc.il_width);
  if (!rc) {
    std::vector<int> idx;
    for (int i = 0; i < nrhs; ++i) {
      sv.add_slot(&slots[i]);
      idx.push_back(i);
    }
    rc = sv.setup(idx);
    if (!rc) {  // zero sources and good initial guesses finish without iterating
      std::vector<int> early;
      for (int i = 0; i < nrhs; ++i)
        if (slots[i].state == SS_RUN && slots[i].last_r64 <= slots[i].target) early.push_back(i);
      if (!early.empty()) {
        rc = sv.finalize(early);
        for (int i : early) slots[i].state = slots[i].info.converged ? SS_DONE : SS_RUN;
      }
    }
    if (!rc) rc = sv.run_until_done(1 << 30);
    if (!rc && sv.method == SOLVER_BICGSTAB && c->cgnr_fallback) rc = cgnr_fallback(c, sv, slots, clover_h, kappa, kop, gf);
  }
  int worst = A2A_OK;
  for (int i = 0; i < nrhs; ++i) {
    Slot& s = slots[i];
    if (info) info[i] = s.info;
    if (s.state == SS_FAIL && worst == A2A_OK) worst = s.err;
    if (s.state == SS_FAIL && s.err == A2A_ENAN) worst = A2A_ENAN;
  }
  int rs = c->sync();
  for (auto& s : slots) slot_free(c, &s);
  if (rc) return rc;
  if (rs) return rs;
  if (worst == A2A_ENOTCONV) c->fail(A2A_ENOTCONV, "some sources did not converge within max_iter");
  if (worst == A2A_EBREAKDOWN) c->fail(A2A_EBREAKDOWN, "the Krylov solver broke down repeatedly");
  if (worst == A2A_ENAN) c->fail(A2A_ENAN, "non-finite source");
  return worst;
}

// Requests of more than SOLVE_BATCH sources run as consecutive batches (each batch iterates in
// lock step; the slot ids a batch holds leave room for a concurrent engine on the context).
constexpr int SOLVE_BATCH = SID_CAP / 2;

int solve_core(Ctx* c, int clover_h, const double* src, int nrhs, double kappa, double csw, double tol, int prec,
               int max_iter, const double* x0, double* sol, a2a_solve_info* info) {
  if (nrhs <= SOLVE_BATCH) return solve_batch(c, clover_h, src, nrhs, kappa, csw, tol, prec, max_iter, x0, sol, info);
  if (check_prec(prec)) return c->fail(A2A_EINVAL, "unknown precision mode");
  GaugeField* gf;
  CloverField* cf;
  KappaOp* kop;
  A2A_TRY(resolve_op(c, clover_h, kappa, prec, &gf, &cf, &kop));
  const size_t per = (size_t)24 * volume_of(gf->g);  // doubles per spinor field
  int worst = A2A_OK;
  for (int i0 = 0; i0 < nrhs; i0 += SOLVE_BATCH) {
    const int n = std::min(SOLVE_BATCH, nrhs - i0);
    const size_t off = (size_t)i0 * per;
    const int rc = solve_batch(c, clover_h, src + off, n, kappa, csw, tol, prec, max_iter, x0 ? x0 + off : nullptr,
                               sol + off, info ? info + i0 : nullptr);
    if (rc != A2A_OK && rc != A2A_ENOTCONV && rc != A2A_EBREAKDOWN && rc != A2A_ENAN) return rc;
    if (rc != A2A_OK && (worst == A2A_OK || rc == A2A_ENAN)) worst = rc;
  }
  return worst;
}

int dslash_core(Ctx* c, int clover_h, double kappa, int opk, int dagger, int prec, const double* in, double* out,
                int nrhs) {
  if (nrhs <= 0) return c->fail(A2A_EINVAL, "nrhs must be positive");
  if (opk < 0 || opk > 3) return c->fail(A2A_EINVAL, "unknown operator");
  if (check_prec(prec)) return c->fail(A2A_EINVAL, "unknown precision mode");
  GaugeField* gf;
  CloverField* cf;
  KappaOp* kop;
  A2A_TRY(resolve_op(c, clover_h, kappa, prec, &gf, &cf, &kop));
  const long hv = gf->g.hv;
  const long long V = volume_of(gf->g);
  Solver sv(c, prec, effective_R(c, prec));
  const int op = sv.op_index(clover_h, kappa, kop, gf);
  std::vector<Slot> slots(nrhs);
  int rc = A2A_OK;
  for (int i = 0; i < nrhs && !rc; ++i) {
    Slot& s = slots[i];
    s.op = op;
    s.src = in + (size_t)i * 24 * V;
    s.sol = out + (size_t)i * 24 * V;
  }
  rc = slots_alloc(c, slots.data(), nrhs, prec, hv, sv.ops[op].nblk, 5, 0);
  if (!rc)
    for (auto& s : slots) sv.add_slot(&s);
  if (!rc) rc = sv.rebuild();
  if (!rc) {
    const int H = sv.n_hop_tiles, Vn = sv.n_vec_tiles, R = sv.R;
    // vectors: 0 in_e, 1 in_o, 2 out_e, 3 out_o, 4 tmp
    rc = sv.layout_in(false, Vn, 0, 0, prec, 0, 1, dagger, RED_NONE);
    if (!rc) switch (opk) {
        case A2A_OP_FULL_D:
          rc = sv.hop(false, H, R, 0, prec, 0, 1, 2, -1, 0, -1, 0, 1.0, -1.0, 1, 0, RED_NONE, nullptr);
          if (!rc) rc = sv.hop(false, H, R, 0, prec, 1, 0, 3, -1, 1, -1, 0, 1.0, -1.0, 1, 0, RED_NONE, nullptr);
          break;
        case A2A_OP_SCHUR:
          rc = sv.hop(false, H, R, 0, prec, 0, 1, 4, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, nullptr);
          if (!rc) rc = sv.hop(false, H, R, 0, prec, 1, 4, 3, -1, 1, -1, 0, 1.0, -1.0, 2, 0, RED_NONE, nullptr);
          if (!rc) rc = sv.vec(false, Vn, VK_ZERO_LO, 0, 0, -1, 2);
          break;
        case A2A_OP_HOP_EO:
          rc = sv.hop(false, H, R, 0, prec, 0, 1, 2, -1, -1, -1, 0, 0, 1.0, 0, 0, RED_NONE, nullptr);
          if (!rc) rc = sv.vec(false, Vn, VK_ZERO_LO, 0, 0, -1, 3);
          break;
        default:
          rc = sv.hop(false, H, R, 0, prec, 1, 0, 3, -1, -1, -1, 0, 0, 1.0, 0, 0, RED_NONE, nullptr);
          if (!rc) rc = sv.vec(false, Vn, VK_ZERO_LO, 0, 0, -1, 2);
          break;
      }
    if (!rc) rc = sv.layout_out(false, Vn, 0, prec, 2, 3, dagger);
  }
  int rs = c->sync();
  for (auto& s : slots) slot_free(c, &s);
  return rc ? rc : rs;
}

int contract_ops(Ctx* c, const Geo& g, const double* src, const double* sol, int n, double** O_dev) {
  const int V3 = g.X * g.Y * g.Z;
  const long K = 12L * V3;
  const int ntb = (n + 63) / 64;
  long want = 4096 / std::max(1, g.T * ntb * ntb);
  int nchunk = (int)std::max(1L, std::min(want, (K + 255) / 256));
  void *part = nullptr, *O = nullptr;
  A2A_TRY(c->dalloc(&part, sizeof(double) * 2 * (size_t)g.T * nchunk * n * n));
  int rc = c->dalloc(&O, sizeof(double) * 2 * (size_t)g.T * n * n);
  if (rc) {
    c->dfree(part);
    return rc;
  }
  launch_stoch_ops(g, n, src, sol, (double*)part, nchunk, (double*)O, c->stream);
  hipError_t e = hipGetLastError();
  rc = c->sync();
  c->dfree(part);
  if (e != hipSuccess) {
    c->dfree(O);
    return c->fail(A2A_EDEVICE, std::string("stochastic operators: ") + hipGetErrorString(e));
  }
  if (rc) {
    c->dfree(O);
    return rc;
  }
  *O_dev = (double*)O;
  return A2A_OK;
}

int copy_to_host(Ctx* c, void* dst, const void* src, size_t n) {
  A2A_HIP(c, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, c->stream));
  return c->sync();
}

// tiny JSON number lookup: "key": value
double json_num(const char* js, const char* key, double dflt) {
  if (!js) return dflt;
  std::string k = std::string("\"") + key + "\"";
  const char* p = std::strstr(js, k.c_str());
  if (!p) return dflt;
  p = std::strchr(p + k.size(), ':');
  if (!p) return dflt;
  return std::strtod(p + 1, nullptr);
}

}  // namespace

// =========================================================================================
// scratch of the allocation-free pion contraction
// =========================================================================================
// The stochastic-operator partial sums (and O itself when the caller passes no O buffer) of
// a2a_contract_pion_2pt_noalloc live in this array.  Every GPU the library runs on holds its
// own copy at its own address, from the first use of the library on that device until the
// process ends.  Host code never passes the array's name to a kernel or a copy (on the host it
// is only a stand-in symbol): it uses the device address looked up once per device below.
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex scratch_mu;
void* scratch_dev[NOALLOC_MAX_DEVICES];

// with `device` current: the device address of that device's copy of the array
int scratch_lookup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return A2A_EINVAL;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_dev[device]) return A2A_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return A2A_EDEVICE;
  scratch_dev[device] = p;
  return A2A_OK;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  return (device >= 0 && device < NOALLOC_MAX_DEVICES) ? scratch_dev[device] : nullptr;
}
}  // namespace

// =========================================================================================
// context
// =========================================================================================
extern "C" int a2a_init(a2a_ctx** out, int device, size_t budget, void* stream) {
  if (!out) return A2A_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return A2A_EDEVICE;
  if (device < 0 || device >= ndev) return A2A_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return A2A_EDEVICE;
  if (scratch_lookup(device) != A2A_OK) return A2A_EDEVICE;
  auto* h = new a2a_ctx();
  Ctx* c = &h->c;
  c->device = device;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete h;
      return A2A_EDEVICE;
    }
    c->own_stream = true;
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    delete h;
    return A2A_EDEVICE;
  }
  c->budget = budget ? budget : (size_t)(0.9 * (double)fr);
  c->sid_cap = SID_CAP;
  const char* dbg = std::getenv("A2A_DEBUG");
  c->debug = dbg && dbg[0] == '1';
  const char* tc = std::getenv("A2A_TUNE_CACHE");
  if (tc && tc[0]) {
    c->tune_path = tc;
    tune_load(c);
  }
  void* p = nullptr;
  if (c->dalloc(&p, sizeof(double) * NSCAL * SID_CAP) ||
      hipMemset(p, 0, sizeof(double) * NSCAL * SID_CAP) != hipSuccess) {
    delete h;
    return A2A_ENOMEM;
  }
  c->scal_pool = (double*)p;
  if (hipHostMalloc((void**)&c->scal_host, sizeof(double) * NSCAL * SID_CAP, hipHostMallocDefault) != hipSuccess) {
    delete h;
    return A2A_ENOMEM;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    delete h;
    return A2A_EDEVICE;
  }
  *out = h;
  return A2A_OK;
}

extern "C" int a2a_finalize(a2a_ctx* h) {
  if (!h) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  c->timing_collect();
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  std::vector<int> hs;
  for (auto& kv : c->gauges) hs.push_back(kv.first);
  for (int g : hs) a2a_unload(h, g);
  for (auto& kv : c->sizes) (void)hipFree(kv.first);
  c->sizes.clear();
  c->release_cache();
  (void)hipStreamSynchronize(c->stream);  // no copy out of the staging buffer is pending
  if (c->scal_host) (void)hipHostFree(c->scal_host);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete h;
  return A2A_OK;
}

extern "C" const char* a2a_last_error(const a2a_ctx* h) { return h ? h->c.err.c_str() : "null context"; }

extern "C" int a2a_set_option(a2a_ctx* h, const char* key, double v) {
  if (!h || !key) return A2A_EINVAL;
  Ctx* c = &h->c;
  std::string k(key);
  if (k == "rhs_block") {
    int r = (int)v;
    if (r != 1 && r != 2 && r != 4) return c->fail(A2A_EINVAL, "rhs_block must be 1, 2 or 4");
    c->rhs_block = r;
  } else if (k == "rhs_block64") {
    int r = (int)v;
    if (r != 1 && r != 2) return c->fail(A2A_EINVAL, "rhs_block64 must be 1 or 2");
    c->rhs_block64 = r;
  } else if (k == "check_every") {
    if (v < 1) return c->fail(A2A_EINVAL, "check_every must be >= 1");
    c->check_every = (int)v;
  } else if (k == "delta") {
    if (!(v > 0 && v < 1)) return c->fail(A2A_EINVAL, "delta must be in (0, 1)");
    c->delta_lo = v;
  } else if (k == "delta_bf16") {
    if (!(v > 0 && v < 1)) return c->fail(A2A_EINVAL, "delta_bf16 must be in (0, 1)");
    c->delta_bf16 = v;
  } else if (k == "delta_cgnr") {
    if (!(v > 0 && v < 1)) return c->fail(A2A_EINVAL, "delta_cgnr must be in (0, 1)");
    c->delta_cgnr = v;
  } else if (k == "delta64") {
    if (!(v > 0 && v < 1)) return c->fail(A2A_EINVAL, "delta64 must be in (0, 1)");
    c->delta_64 = v;
  } else if (k == "xcd_order") {
    c->xcd_order = v != 0;
  } else if (k == "kernel_timing") {
    c->timing = v != 0;
  } else if (k == "autotune") {
    c->autotune = v != 0;
  } else if (k == "mfma_slab") {
    c->mfma_slab = v != 0;
  } else if (k == "ru_correction") {
    c->ru_correction = v != 0;
  } else if (k == "schur_sym") {
    c->schur_sym = v != 0;
  } else if (k == "upload_stage_bytes") {
    if (!(v >= 0 && v <= (double)((size_t)1 << 32))) return c->fail(A2A_EINVAL, "upload_stage_bytes must be in [0, 4 GiB]");
    if (c->stage) {  // the next upload allocates the new size
      A2A_TRY(c->sync());
      (void)hipHostFree(c->stage);
      c->stage = nullptr;
    }
    c->stage_cap = c->stage_off = 0;
    c->stage_failed = false;
    c->stage_req = (size_t)v;
  } else if (k == "tail_checks") {
    c->tail_checks = v != 0;
  } else if (k == "target_frac") {
    if (!(v > 0.0 && v <= 1.0)) return c->fail(A2A_EINVAL, "target_frac must be in (0, 1]");
    c->target_frac = v;
  } else if (k == "il_width") {
    if (v != 16 && v != 32 && v != 48) return c->fail(A2A_EINVAL, "il_width must be 16, 32 or 48");
    c->il_width = (int)v;
  } else if (k == "brick") {  // by * 10000 + bz * 100 + bt, 0 = each lattice's default
    const long b = (long)v;
    if (b < 0 || (double)b != v) return c->fail(A2A_EINVAL, "brick must be by * 10000 + bz * 100 + bt or 0");
    const int by = (int)(b / 10000), bz = (int)(b / 100 % 100), bt = (int)(b % 100);
    if (b != 0 && (by < 1 || bz < 1 || bt < 1 || by * bz * bt > BS))
      return c->fail(A2A_EINVAL, "brick extents must be >= 1 with by bz bt <= 256");
    c->brick_by = by;
    c->brick_bz = bz;
    c->brick_bt = bt;
  } else if (k == "interleave") {
    c->interleave = v != 0;
  } else if (k == "mfma") {
    c->mfma = v != 0;
  } else if (k == "solver") {
    if (v != A2A_SOLVER_BICGSTAB && v != A2A_SOLVER_CGNR) return c->fail(A2A_EINVAL, "solver must be 0 or 1");
    c->solver = (int)v;
  } else if (k == "cgnr_fallback") {
    c->cgnr_fallback = v != 0;
  } else if (k == "force_breakdown") {
    c->force_breakdown = v != 0;
  } else if (k == "poison_memory") {
    c->poison = v != 0;
  } else if (k == "fail_setup_enomem") {
    if (v < 0) return c->fail(A2A_EINVAL, "fail_setup_enomem must be >= 0");
    c->fail_setup_enomem = (int)v;
  } else if (k == "fail_setup_device") {
    if (v < 0) return c->fail(A2A_EINVAL, "fail_setup_device must be >= 0");
    c->fail_setup_device = (int)v;
  } else if (k == "hbm_budget") {
    if (!(v > 0)) return c->fail(A2A_EINVAL, "hbm_budget must be positive");
    c->budget = (size_t)v;
  } else {
    return c->fail(A2A_EINVAL, "unknown option " + k);
  }
  return A2A_OK;
}

extern "C" size_t a2a_mem_in_use(const a2a_ctx* h) { return h ? h->c.used : 0; }

// =========================================================================================
// resident fields
// =========================================================================================
static int load_gauge_impl(a2a_ctx* h, const a2a_geom* geom, const double* links, int* gauge_h, bool dev) {
  if (!h || !links || !gauge_h) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "lattice extents must be even and >= 2, t_bc = +-1");
  const size_t n = (size_t)2 * g.hv * 72;
  if (!dev)
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(links[i])) return c->fail(A2A_ENAN, "non-finite gauge link");
  auto gf = std::make_unique<GaugeField>();
  gf->geom = *geom;
  gf->g = g;
  void* p = nullptr;
  A2A_TRY(c->dalloc(&p, n * sizeof(double)));
  gf->canon = (double*)p;
  A2A_HIP(c, hipMemcpyAsync(gf->canon, links, n * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            c->stream));
  gf->handle = c->next_handle++;
  GaugeField* raw = gf.get();
  c->gauges[gf->handle] = std::move(gf);
  void *u0, *u1;
  int rc = c->gauge_links(raw, 0, &u0, &u1);
  if (!rc) rc = c->sync();
  if (rc) {
    a2a_unload(h, raw->handle);
    return rc;
  }
  *gauge_h = raw->handle;
  return A2A_OK;
}

extern "C" int a2a_load_gauge(a2a_ctx* h, const a2a_geom* geom, const double* links, int* gauge_h) {
  return load_gauge_impl(h, geom, links, gauge_h, false);
}

extern "C" int a2a_load_gauge_dev(a2a_ctx* h, const a2a_geom* geom, const double* links, int* gauge_h) {
  return load_gauge_impl(h, geom, links, gauge_h, true);
}

extern "C" int a2a_load_clover(a2a_ctx* h, int gauge_h, double csw, int* clover_h) {
  if (!h || !clover_h) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  GaugeField* gf = c->gauge(gauge_h);
  if (!gf) return c->fail(A2A_EHANDLE, "unknown gauge handle");
  if (!std::isfinite(csw)) return c->fail(A2A_EINVAL, "c_sw must be finite");
  auto cf = std::make_unique<CloverField>();
  cf->gauge = gauge_h;
  cf->csw = csw;
  const size_t cb = clover_bytes<double>(gf->g.hv);
  void *p0 = nullptr, *p1 = nullptr;
  A2A_TRY(c->dalloc(&p0, cb));
  int rc = c->dalloc(&p1, cb);
  if (rc) {
    c->dfree(p0);
    return rc;
  }
  cf->G[0] = (double*)p0;
  cf->G[1] = (double*)p1;
  launch_clover_field(gf->g, gf->canon, cf->G, c->stream);
  A2A_HIP(c, hipGetLastError());
  A2A_TRY(c->sync());
  cf->handle = c->next_handle++;
  *clover_h = cf->handle;
  c->clovers[cf->handle] = std::move(cf);
  return A2A_OK;
}

static void free_clover(Ctx* c, CloverField* cf) {
  for (auto& k : cf->kops) {
    for (int p = 0; p < 2; ++p) {
      c->dfree(k->A64[p]);
      c->dfree(k->Ai64[p]);
      for (int q = 1; q < 4; ++q) {
        c->dfree(k->Alo[q][p]);
        c->dfree(k->Ailo[q][p]);
      }
    }
  }
  c->dfree(cf->G[0]);
  c->dfree(cf->G[1]);
}

extern "C" int a2a_unload(a2a_ctx* h, int handle) {
  if (!h) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipStreamSynchronize(c->stream);
  if (auto* cf = c->clover(handle)) {
    free_clover(c, cf);
    c->clovers.erase(handle);
    return A2A_OK;
  }
  if (auto* gf = c->gauge(handle)) {
    std::vector<int> dead;
    for (auto& kv : c->clovers)
      if (kv.second->gauge == handle) dead.push_back(kv.first);
    for (int d : dead) {
      free_clover(c, c->clover(d));
      c->clovers.erase(d);
    }
    c->dfree(gf->canon);
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < 2; ++p) {
        c->dfree(gf->U[q][p]);
        c->dfree(gf->HL[q][p]);
      }
    c->gauges.erase(handle);
    return A2A_OK;
  }
  return c->fail(A2A_EHANDLE, "unknown handle");
}

// =========================================================================================
// operator application
// =========================================================================================
extern "C" int a2a_dslash_clover_dev(a2a_ctx* h, int clover_h, double kappa, int op, int dagger, int prec,
                                     const double* in, double* out, int nrhs) {
  if (!h || !in || !out) return A2A_EINVAL;
  (void)hipSetDevice(h->c.device);
  return dslash_core(&h->c, clover_h, kappa, op, dagger ? 1 : 0, prec, in, out, nrhs);
}

extern "C" int a2a_dslash_clover(a2a_ctx* h, int clover_h, double kappa, int op, int dagger, int prec,
                                 const double* in, double* out, int nrhs) {
  if (!h || !in || !out) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  CloverField* cf = c->clover(clover_h);
  if (!cf) return c->fail(A2A_EHANDLE, "unknown clover handle");
  if (nrhs <= 0) return c->fail(A2A_EINVAL, "nrhs must be positive");
  const size_t n = (size_t)nrhs * 24 * volume_of(c->gauge(cf->gauge)->g) * sizeof(double);
  void *di = nullptr, *dout = nullptr;
  A2A_TRY(c->dalloc(&di, n));
  int rc = c->dalloc(&dout, n);
  if (!rc) {
    if (hipMemcpyAsync(di, in, n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      rc = c->fail(A2A_EDEVICE, "host to device copy failed");
  }
  if (!rc) rc = dslash_core(c, clover_h, kappa, op, dagger ? 1 : 0, prec, (const double*)di, (double*)dout, nrhs);
  if (!rc) rc = copy_to_host(c, out, dout, n);
  c->sync();
  c->dfree(di);
  c->dfree(dout);
  return rc;
}

// mean milliseconds of one stencil application (HOP_EO, or the two launches of the Schur
// operator) on nrhs device-layout fields in launch configuration tc (per-thread width, brick,
// interleaved group width), timed with HIP events
static int stencil_time(Ctx* c, int clover_h, double kappa, int opk, int prec, int nrhs, int reps,
                        const TuneCfg& tc, double* ms) {
  GaugeField* gf;
  CloverField* cf;
  KappaOp* kop;
  A2A_TRY(resolve_op(c, clover_h, kappa, prec, &gf, &cf, &kop));
  Solver sv(c, prec, tc.R ? tc.R : effective_R(c, prec));
  if (tc.slab >= 0) sv.mfma_slab = tc.slab;
  sv.xcd_hop = tc.xcd64;
  if (tc.by > 0) {
    sv.by = tc.by;
    sv.bz = tc.bz;
    sv.bt = tc.bt;
  }
  const int op = sv.op_index(clover_h, kappa, kop, gf);
  std::vector<Slot> slots(nrhs);
  int rc = A2A_OK;
  for (int i = 0; i < nrhs; ++i) slots[i].op = op;
  rc = slots_alloc(c, slots.data(), nrhs, prec, gf->g.hv, sv.ops[op].nblk, 5, 0, tc.il_width);
  if (!rc)
    for (auto& s : slots) sv.add_slot(&s);
  if (!rc) rc = sv.rebuild();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) {
    const int H = sv.n_hop_tiles, Vn = sv.n_vec_tiles, R = sv.R;
    rc = sv.vec(false, Vn, VK_FILL_LO, 0, 0, -1, 0);
    if (!rc) rc = sv.vec(false, Vn, VK_FILL_LO, 0, 0, -1, 1);
    auto once = [&]() -> int {
      if (opk == A2A_OP_HOP_EO)
        return sv.hop(false, H, R, 0, prec, 0, 1, 2, -1, -1, -1, 0, 0, 1.0, 0, 0, RED_NONE, nullptr);
      int r = sv.hop(false, H, R, 0, prec, 0, 1, 4, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, nullptr);
      if (!r) r = sv.hop(false, H, R, 0, prec, 1, 4, 3, -1, 1, -1, 0, 1.0, -1.0, 2, 0, RED_NONE, nullptr);
      return r;
    };
    for (int w = 0; w < 2 && !rc; ++w) rc = once();
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
      rc = c->fail(A2A_EDEVICE, "hipEventCreate failed");
    if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = c->fail(A2A_EDEVICE, "hipEventRecord failed");
    for (int w = 0; w < reps && !rc; ++w) rc = once();
    if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = c->fail(A2A_EDEVICE, "hipEventRecord failed");
    if (!rc) rc = c->sync();
    float t = 0;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = c->fail(A2A_EDEVICE, "hipEventElapsedTime failed");
    if (!rc) *ms = t / reps;
  }
  c->sync();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (auto& s : slots) slot_free(c, &s);
  return rc;
}

// Time the FP64 stencil pair of a correction-form reliable update (te = A_ee^-1 H_eo (sigma x_lo),
// r64 -= M (sigma x_lo), the hopping input and the clover input read from the inner arena) for
// nrhs sources stored in precision prec (interleaved groups of il.il_width lanes), with the FP64
// stencils in configuration f64: width f64.R, brick f64.by/bz/bt, XCD order f64.xcd64.  This is
// the FP64 work of the solves of FP16 / BF16 / FP32 storage; values are arbitrary (timing only).
static int ru_time(Ctx* c, int clover_h, double kappa, int prec, int nrhs, int reps, const TuneCfg& il,
                   const TuneCfg& f64, double* ms) {
  GaugeField* gf;
  CloverField* cf;
  KappaOp* kop;
  A2A_TRY(resolve_op(c, clover_h, kappa, prec, &gf, &cf, &kop));
  Solver sv(c, prec, il.R ? il.R : effective_R(c, prec));
  sv.R64 = f64.R;
  if (il.by > 0) {
    sv.by = il.by;
    sv.bz = il.bz;
    sv.bt = il.bt;
  }
  sv.by64 = f64.by;
  sv.bz64 = f64.bz;
  sv.bt64 = f64.bt;
  sv.xcd_sub = f64.xcd64;
  const int op = sv.op_index(clover_h, kappa, kop, gf);
  std::vector<Slot> slots(nrhs);
  int rc = A2A_OK;
  for (int i = 0; i < nrhs; ++i) slots[i].op = op;
  rc = slots_alloc(c, slots.data(), nrhs, prec, gf->g.hv, sv.ops[op].nblk, NVEC_LO, NVEC_HI, il.il_width);
  if (!rc)
    for (auto& s : slots) sv.add_slot(&s);
  if (!rc) rc = sv.rebuild();
  std::vector<int> all(nrhs);
  for (int i = 0; i < nrhs; ++i) all[i] = i;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) {
    const int Vn = sv.n_vec_tiles;
    rc = sv.vec(false, Vn, VK_FILL_LO, 0, 0, -1, VL_X);
    if (!rc) rc = sv.vec(false, Vn, VK_ZERO_HI, 0, 0, -1, VH_R);
    if (!rc) rc = sv.upload_subset(all, sv.R64);
    if (!rc) rc = sv.true_residual_corr(all);  // warmup
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
      rc = c->fail(A2A_EDEVICE, "hipEventCreate failed");
    if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = c->fail(A2A_EDEVICE, "hipEventRecord failed");
    for (int w = 0; w < reps && !rc; ++w) rc = sv.true_residual_corr(all);
    if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = c->fail(A2A_EDEVICE, "hipEventRecord failed");
    if (!rc) rc = c->sync();
    float t = 0;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = c->fail(A2A_EDEVICE, "hipEventElapsedTime failed");
    if (!rc) *ms = t / reps;
  }
  c->sync();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (auto& s : slots) slot_free(c, &s);
  return rc;
}

extern "C" int a2a_bench_stencil(a2a_ctx* h, int clover_h, double kappa, int opk, int prec, int nrhs, int reps,
                                 double* ms) {
  if (!h || !ms || nrhs <= 0 || reps <= 0) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  if (check_prec(prec)) return c->fail(A2A_EINVAL, "unknown precision mode");
  if (opk != A2A_OP_HOP_EO && opk != A2A_OP_SCHUR) return c->fail(A2A_EINVAL, "op must be HOP_EO or SCHUR");
  return stencil_time(c, clover_h, kappa, opk, prec, nrhs, reps, TuneCfg{}, ms);
}

// ---- autotuner: launch configuration per (arch, lattice, precision, RHS bucket)
static std::string tune_key(const Geo& g, int prec, int nrhs) {
  int b = 1;
  while (b < nrhs && b < 64) b <<= 1;
  return "gfx950:" + std::to_string(g.X) + "x" + std::to_string(g.Y) + "x" + std::to_string(g.Z) + "x" +
         std::to_string(g.T) + ":p" + std::to_string(prec) + ":n" + std::to_string(b);
}

static void tune_save(Ctx* c) {
  if (c->tune_path.empty()) return;
  const std::string tmp = c->tune_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{");
  bool first = true;
  for (auto& kv : c->tuned) {
    const TuneCfg& t = kv.second;
    std::fprintf(f,
                 "%s\n  \"%s\": {\"il_width\": %d, \"by\": %d, \"bz\": %d, \"bt\": %d, \"slab\": %d, \"R\": %d, "
                 "\"R64\": %d, \"by64\": %d, \"bz64\": %d, \"bt64\": %d, \"xcd64\": %d}",
                 first ? "" : ",", kv.first.c_str(), t.il_width, t.by, t.bz, t.bt, t.slab, t.R, t.R64, t.by64, t.bz64,
                 t.bt64, t.xcd64);
    first = false;
  }
  std::fprintf(f, "\n}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), c->tune_path.c_str());
}

static void tune_load(Ctx* c) {
  if (c->tune_path.empty()) return;
  FILE* f = std::fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char key[400];
    TuneCfg t;
    if (std::sscanf(line,
                    " \"%399[^\"]\": {\"il_width\": %d, \"by\": %d, \"bz\": %d, \"bt\": %d, \"slab\": %d, \"R\": %d, "
                    "\"R64\": %d, \"by64\": %d, \"bz64\": %d, \"bt64\": %d, \"xcd64\": %d",
                    key, &t.il_width, &t.by, &t.bz, &t.bt, &t.slab, &t.R, &t.R64, &t.by64, &t.bz64, &t.bt64,
                    &t.xcd64) != 12)
      continue;
    const bool ok = (t.il_width == 0 || t.il_width == 16 || t.il_width == 32 || t.il_width == 48) &&
                    (t.R == 0 || t.R == 1 || t.R == 2 || t.R == 4) && (t.R64 == 0 || t.R64 == 1 || t.R64 == 2) &&
                    t.by >= 0 && t.bz >= 0 && t.bt >= 0 && t.by <= 64 && t.bz <= 64 && t.bt <= 64 &&
                    t.slab >= -1 && t.slab <= 1 && t.xcd64 >= -1 && t.xcd64 <= 1 && t.by64 >= 0 && t.bz64 >= 0 &&
                    t.bt64 >= 0 && t.by64 <= 64 && t.bz64 <= 64 && t.bt64 <= 64;
    if (ok) c->tuned[key] = t;  // a brick that does not tile the lattice is ignored at use
  }
  std::fclose(f);
}

// Coordinate search over the knobs of the path the solve runs, each timed on the Schur
// operator (both stencil launches) with min(nrhs, 64) sources:
//   1. the interleaved group width 16 / 32 / 48 (FP16 / BF16 storage on the matrix cores), or the
//      per-thread RHS width 1 / 2 / 4 (FP32, FP64, or FP16 / BF16 without interleaving);
//   2. the stencil brick (y, z, t extents; up to six shapes that tile the lattice);
//   3. the RHS width 1 / 2 of the FP64 stencils of setup, reliable updates and reconstruction,
//      timed as the FP64 Schur operator on min(nrhs, 24) sources with the chosen brick.
// The result is cached in the context and in the JSON file named by A2A_TUNE_CACHE.
static int autotune_cfg(Ctx* c, int clover_h, double kappa, int prec, int nrhs, TuneCfg* out,
                        a2a_tune_result* res) {
  CloverField* cf = c->clover(clover_h);
  if (!cf) return c->fail(A2A_EHANDLE, "unknown clover handle");
  const Geo g = c->gauge(cf->gauge)->g;
  const std::string key = tune_key(g, prec, nrhs);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    *out = it->second;
    if (res) {
      std::memset(res, 0, sizeof *res);
      res->il_width = out->il_width;
      res->brick[0] = out->by;
      res->brick[1] = out->bz;
      res->brick[2] = out->bt;
      res->rhs_block = out->R;
      res->rhs_block64 = out->R64;
      res->xcd_slab = out->slab;
      res->brick64[0] = out->by64 ? out->by64 : out->by;
      res->brick64[1] = out->by64 ? out->bz64 : out->bz;
      res->brick64[2] = out->by64 ? out->bt64 : out->bt;
      res->xcd64 = out->xcd64;
      res->ms_schur = res->ms_schur64 = -1.0;
    }
    return A2A_OK;
  }
  const int n = std::min(nrhs, 64);
  const bool il = use_interleave(c, prec) && c->mfma && n >= IL_REM_MIN;
  int tried = 0;
  auto timed = [&](int p, int nn, const TuneCfg& t, double* ms) -> int {
    ++tried;
    return stencil_time(c, clover_h, kappa, A2A_OP_SCHUR, p, nn, 3, t, ms);
  };
  TuneCfg best{};
  double tbest = 1e300;
  // 1. RHS width of the inner stencil
  if (il) {
    for (int w : {48, 32, 16}) {
      if (w > 16 && w - 16 >= ((n + 15) / 16) * 16) continue;  // a group would hold no more sources than w - 16
      TuneCfg t{};
      t.il_width = w;
      double ms = 0;
      A2A_TRY(timed(prec, n, t, &ms));
      if (ms < tbest) {
        tbest = ms;
        best = t;
      }
    }
  } else {
    for (int r : {1, 2, 4}) {
      if (prec == 0 && r > 2) continue;
      TuneCfg t{};
      t.R = r;
      double ms = 0;
      A2A_TRY(timed(prec, n, t, &ms));
      if (ms < tbest) {
        tbest = ms;
        best = t;
      }
    }
  }
  // 2. brick (the default brick in brick order was timed above), and for the matrix-core
  //    stencil the block order: brick order or XCD slabs
  int br[8][3];
  const int nb = brick_choices(g, br, 6);
  best.by = g.by;
  best.bz = g.bz;
  best.bt = g.bt;
  best.slab = il ? c->mfma_slab : -1;
  const TuneCfg first = best;  // timed in step 1
  for (int k = 0; k < nb; ++k)
    for (int sl = 0; sl < (il ? 2 : 1); ++sl) {
      TuneCfg t = first;
      t.by = br[k][0];
      t.bz = br[k][1];
      t.bt = br[k][2];
      if (il) t.slab = sl;
      if (t.by == first.by && t.bz == first.bz && t.bt == first.bt && t.slab == first.slab) continue;
      double ms = 0;
      A2A_TRY(timed(prec, n, t, &ms));
      if (ms < tbest) {
        tbest = ms;
        best = t;
      }
    }
  // 3. FP64 stencils: width, then their own brick and tile order over the XCDs.  Solves with
  //    FP16 / BF16 / FP32 storage spend their FP64 time in the correction-form stencil pair of
  //    reliable updates, whose inputs come from the inner arena, so that pair is what is timed
  //    (the plain FP64 Schur operator ranked bricks differently: two within 0.2% of each other
  //    there differed by 25% in the pair); the FP64-only mode times its Schur operator.
  double t64 = 1e300;
  const int n64 = std::min(nrhs, 48);  // the slot counts of reliable updates: bricks rank differently at 24
  const bool corr = prec != 0 && c->ru_correction && hop_lo_supports(2, 1, prec, 1, false);
  TuneCfg b64 = best;
  b64.il_width = 0;
  b64.slab = -1;
  b64.xcd64 = c->xcd_order ? 1 : 0;
  auto timed64 = [&](const TuneCfg& t, double* ms) -> int {
    if (!corr) return timed(0, n64, t, ms);
    ++tried;
    return ru_time(c, clover_h, kappa, prec, n64, 2, best, t, ms);
  };
  // width x brick x order jointly: which width wins depends on the brick (and on the GPU: the
  // correction-form pair's time varies up to 2x between GPUs, with the ranking of the widths)
  {
    std::vector<TuneCfg> cand;
    for (int r : {1, 2})
      for (int k = -1; k < nb; ++k)
        for (int xo = 0; xo < 2; ++xo) {
          TuneCfg t = b64;
          t.R = r;
          if (k >= 0) {
            t.by = br[k][0];
            t.bz = br[k][1];
            t.bt = br[k][2];
          }
          t.xcd64 = xo;
          bool dup = false;
          for (const TuneCfg& u : cand)
            dup = dup || (u.R == t.R && u.by == t.by && u.bz == t.bz && u.bt == t.bt && u.xcd64 == t.xcd64);
          if (!dup) cand.push_back(t);
        }
    for (const TuneCfg& t : cand) {
      double ms = 0;
      A2A_TRY(timed64(t, &ms));
      if (ms < t64) {
        t64 = ms;
        b64 = t;
      }
    }
  }
  best.R64 = b64.R;
  best.xcd64 = b64.xcd64;
  if (b64.by != best.by || b64.bz != best.bz || b64.bt != best.bt) {
    best.by64 = b64.by;
    best.bz64 = b64.bz;
    best.bt64 = b64.bt;
  }
  c->tuned[key] = best;
  tune_save(c);
  *out = best;
  if (res) {
    std::memset(res, 0, sizeof *res);
    res->il_width = best.il_width;
    res->brick[0] = best.by;
    res->brick[1] = best.bz;
    res->brick[2] = best.bt;
    res->rhs_block = best.R;
    res->rhs_block64 = best.R64;
    res->xcd_slab = best.slab;
    res->brick64[0] = best.by64 ? best.by64 : best.by;
    res->brick64[1] = best.by64 ? best.bz64 : best.bz;
    res->brick64[2] = best.by64 ? best.bt64 : best.bt;
    res->xcd64 = best.xcd64;
    res->ms_schur = tbest;
    res->ms_schur64 = t64;
    res->candidates = tried;
  }
  return A2A_OK;
}

extern "C" int a2a_brick_choices(const a2a_geom* geom, int* out, int maxn) {
  Geo g;
  if (!geom || !out || maxn < 0 || geom_to_geo(geom, &g)) return A2A_EINVAL;
  std::vector<int> tmp(3 * (size_t)std::max(1, maxn));
  const int n = brick_choices(g, (int(*)[3])tmp.data(), maxn);
  std::copy(tmp.begin(), tmp.begin() + 3 * n, out);
  return n;
}

extern "C" int a2a_autotune(a2a_ctx* h, int clover_h, double kappa, int prec, int nrhs, a2a_tune_result* result) {
  if (!h || nrhs <= 0) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  if (check_prec(prec)) return c->fail(A2A_EINVAL, "unknown precision mode");
  TuneCfg t{};
  return autotune_cfg(c, clover_h, kappa, prec, nrhs, &t, result);
}

// =========================================================================================
// solves
// =========================================================================================
extern "C" int a2a_solve_propagators_dev(a2a_ctx* h, int clover_h, const double* src, int nrhs, double kappa,
                                         double csw, double tol, int prec, int max_iter, const double* x0,
                                         double* sol, a2a_solve_info* info) {
  if (!h) return A2A_EINVAL;
  (void)hipSetDevice(h->c.device);
  return solve_core(&h->c, clover_h, src, nrhs, kappa, csw, tol, prec, max_iter, x0, sol, info);
}

extern "C" int a2a_solve_propagators(a2a_ctx* h, int clover_h, const double* src, int nrhs, double kappa,
                                     double csw, double tol, int prec, int max_iter, const double* x0,
                                     double* sol, a2a_solve_info* info) {
  if (!h || !src || !sol) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  CloverField* cf = c->clover(clover_h);
  if (!cf) return c->fail(A2A_EHANDLE, "unknown clover handle");
  if (nrhs <= 0) return c->fail(A2A_EINVAL, "nrhs must be positive");
  const size_t n = (size_t)nrhs * 24 * volume_of(c->gauge(cf->gauge)->g);
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(src[i])) return c->fail(A2A_ENAN, "non-finite source");
  void *ds = nullptr, *dx = nullptr, *d0 = nullptr;
  A2A_TRY(c->dalloc(&ds, n * sizeof(double)));
  int rc = c->dalloc(&dx, n * sizeof(double));
  if (!rc && x0) rc = c->dalloc(&d0, n * sizeof(double));
  if (!rc && hipMemcpyAsync(ds, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    rc = c->fail(A2A_EDEVICE, "host to device copy failed");
  if (!rc && x0 && hipMemcpyAsync(d0, x0, n * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    rc = c->fail(A2A_EDEVICE, "host to device copy failed");
  int solve_rc = A2A_OK;
  if (!rc) {
    solve_rc = solve_core(c, clover_h, (const double*)ds, nrhs, kappa, csw, tol, prec, max_iter, (const double*)d0,
                          (double*)dx, info);
    if (solve_rc == A2A_OK || solve_rc == A2A_ENOTCONV || solve_rc == A2A_EBREAKDOWN)
      rc = copy_to_host(c, sol, dx, n * sizeof(double));
    else
      rc = solve_rc;
  }
  c->sync();
  c->dfree(ds);
  c->dfree(dx);
  c->dfree(d0);
  return rc ? rc : solve_rc;
}

// =========================================================================================
// contractions
// =========================================================================================
static int pion_impl(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol, int n, int mode,
                     double* corr, double* O_host, bool dev) {
  if (!h || !src || !sol || !corr) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (n < 1 || (mode == A2A_PION_UNBIASED && n < 2) || (mode != 0 && mode != 1))
    return c->fail(A2A_EINVAL, "need nrhs >= 2 for the unbiased estimator and mode 0 or 1");
  const size_t nel = (size_t)n * 24 * 2 * g.hv;
  const double *ds = src, *dx = sol;
  void *bs = nullptr, *bx = nullptr;
  if (!dev) {
    A2A_TRY(c->dalloc(&bs, nel * sizeof(double)));
    int rc = c->dalloc(&bx, nel * sizeof(double));
    if (rc) {
      c->dfree(bs);
      return rc;
    }
    (void)hipMemcpyAsync(bs, src, nel * sizeof(double), hipMemcpyHostToDevice, c->stream);
    (void)hipMemcpyAsync(bx, sol, nel * sizeof(double), hipMemcpyHostToDevice, c->stream);
    ds = (const double*)bs;
    dx = (const double*)bx;
  }
  double* O = nullptr;
  int rc = contract_ops(c, g, ds, dx, n, &O);
  void* dc = nullptr;
  if (!rc) rc = c->dalloc(&dc, sizeof(double) * 2 * g.T);
  if (!rc) {
    launch_pion_corr(g.T, n, O, mode, (double*)dc, c->stream);
    rc = copy_to_host(c, corr, dc, sizeof(double) * 2 * g.T);
  }
  if (!rc && O_host) rc = copy_to_host(c, O_host, O, sizeof(double) * 2 * (size_t)g.T * n * n);
  c->sync();
  c->dfree(dc);
  c->dfree(O);
  c->dfree(bs);
  c->dfree(bx);
  return rc;
}

extern "C" int a2a_contract_pion_2pt(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol, int n,
                                     int mode, double* corr, double* O) {
  return pion_impl(h, geom, src, sol, n, mode, corr, O, false);
}

extern "C" int a2a_contract_pion_2pt_dev(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol,
                                         int n, int mode, double* corr, double* O) {
  return pion_impl(h, geom, src, sol, n, mode, corr, O, true);
}

// The pion contraction without any allocation: partial sums (and O when O_dev is null) in the
// device's static scratch array, inputs and outputs in the caller's device memory.
extern "C" int a2a_contract_pion_2pt_noalloc(a2a_ctx* h, const a2a_geom* geom, const double* src,
                                             const double* sol, int n, int mode, double* corr_dev, double* O_dev) {
  if (!h || !src || !sol || !corr_dev) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (n < 1 || (mode == A2A_PION_UNBIASED && n < 2) || (mode != 0 && mode != 1))
    return c->fail(A2A_EINVAL, "need nrhs >= 2 for the unbiased estimator and mode 0 or 1");
  char* base = (char*)scratch_of(c->device);
  if (!base) return c->fail(A2A_EDEVICE, "no scratch address for this device");
  const size_t per = sizeof(double) * 2 * (size_t)g.T * n * n;  // one [T][n][n] complex array
  const size_t o_bytes = O_dev ? 0 : (per + 255) & ~(size_t)255;
  if (o_bytes + per > NOALLOC_SCRATCH_BYTES)
    return c->fail(A2A_EINVAL, "T nrhs^2 too large for the 32 MiB scratch of the allocation-free contraction (" +
                                   std::to_string((o_bytes + per) >> 20) + " MiB needed at the least)");
  // chunks of the K sum as in the allocating call, as many as the scratch holds
  const long K = 12L * g.X * g.Y * g.Z;
  const int ntb = (n + 63) / 64;
  const long want = 4096 / std::max(1, g.T * ntb * ntb);
  const long fit = (long)((NOALLOC_SCRATCH_BYTES - o_bytes) / per);
  const int nchunk = (int)std::max(1L, std::min(std::min(want, (K + 255) / 256), fit));
  double* O = O_dev ? O_dev : (double*)base;
  double* part = (double*)(base + o_bytes);
  launch_stoch_ops(g, n, src, sol, part, nchunk, O, c->stream);
  launch_pion_corr(g.T, n, O, mode, corr_dev, c->stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return c->fail(A2A_EDEVICE, std::string("pion contraction: ") + hipGetErrorString(e));
  return c->sync();
}

static int pipi_impl(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol, int n, double* diag,
                     double* vac, double* pion, bool dev) {
  if (!h || !src || !sol || !diag) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (n < 4 || n % 4 || n / 4 > 32) return c->fail(A2A_EINVAL, "pi-pi needs nrhs = 4m with 1 <= m <= 32");
  const size_t nel = (size_t)n * 24 * 2 * g.hv;
  const double *ds = src, *dx = sol;
  void *bs = nullptr, *bx = nullptr;
  if (!dev) {
    A2A_TRY(c->dalloc(&bs, nel * sizeof(double)));
    int rc = c->dalloc(&bx, nel * sizeof(double));
    if (rc) {
      c->dfree(bs);
      return rc;
    }
    (void)hipMemcpyAsync(bs, src, nel * sizeof(double), hipMemcpyHostToDevice, c->stream);
    (void)hipMemcpyAsync(bx, sol, nel * sizeof(double), hipMemcpyHostToDevice, c->stream);
    ds = (const double*)bs;
    dx = (const double*)bx;
  }
  double* O = nullptr;
  int rc = contract_ops(c, g, ds, dx, n, &O);
  void *dd = nullptr, *dv = nullptr, *dp = nullptr;
  if (!rc) rc = c->dalloc(&dd, sizeof(double) * 2 * 4 * g.T);
  if (!rc) rc = c->dalloc(&dv, sizeof(double) * 2 * g.T);
  if (!rc && pion) rc = c->dalloc(&dp, sizeof(double) * 2 * g.T);
  if (!rc) {
    launch_pipi(g.T, n, O, (double*)dd, (double*)dv, c->stream);
    if (pion) launch_pion_corr(g.T, n, O, A2A_PION_UNBIASED, (double*)dp, c->stream);
    rc = copy_to_host(c, diag, dd, sizeof(double) * 2 * 4 * g.T);
    if (!rc && vac) rc = copy_to_host(c, vac, dv, sizeof(double) * 2 * g.T);
    if (!rc && pion) rc = copy_to_host(c, pion, dp, sizeof(double) * 2 * g.T);
  }
  c->sync();
  c->dfree(dd);
  c->dfree(dv);
  c->dfree(dp);
  c->dfree(O);
  c->dfree(bs);
  c->dfree(bx);
  return rc;
}

extern "C" int a2a_contract_pipi_2pt(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol, int n,
                                     double* diag, double* vac, double* pion) {
  return pipi_impl(h, geom, src, sol, n, diag, vac, pion, false);
}

extern "C" int a2a_contract_pipi_2pt_dev(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol,
                                         int n, double* diag, double* vac, double* pion) {
  return pipi_impl(h, geom, src, sol, n, diag, vac, pion, true);
}

extern "C" int a2a_z2_noise_dev(a2a_ctx* h, const a2a_geom* geom, unsigned long long seed, long long src_offset,
                                int nsrc, double* out) {
  if (!h || !out) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (nsrc <= 0 || src_offset < 0) return c->fail(A2A_EINVAL, "nsrc must be positive, src_offset >= 0");
  launch_z2_noise(2L * g.hv, nsrc, seed, src_offset, out, c->stream);
  A2A_HIP(c, hipGetLastError());
  return c->sync();
}

extern "C" int a2a_kernel_stats(a2a_ctx* h, const char* name, long long* launches, double* total_ms,
                                double* alg_bytes, int reset) {
  if (!h || !name) return A2A_EINVAL;
  Ctx* c = &h->c;
  A2A_TRY(c->timing_collect());
  std::string n(name);
  int k0 = -1, k1 = -1;  // class range [k0, k1]
  if (n == "schur1") k0 = k1 = 0;
  if (n == "schur2") k0 = k1 = 1;
  if (n == "xr") k0 = k1 = 2;
  if (n == "p") k0 = k1 = 3;
  if (n == "s") k0 = k1 = 4;
  if (n == "blas") k0 = 2, k1 = 4;
  if (k0 < 0) return c->fail(A2A_EINVAL, "kernel class must be schur1, schur2, xr, p, s or blas");
  long long nl = 0;
  double ms = 0, by = 0;
  for (int k = k0; k <= k1; ++k) {
    nl += c->t_launches[k];
    ms += c->t_ms[k];
    by += c->t_bytes[k];
  }
  if (launches) *launches = nl;
  if (total_ms) *total_ms = ms;
  if (alg_bytes) *alg_bytes = by;
  if (reset)
    for (int i = 0; i < Ctx::NCLS; ++i) {
      c->t_launches[i] = 0;
      c->t_ms[i] = 0;
      c->t_bytes[i] = 0;
    }
  return A2A_OK;
}

// =========================================================================================
// outer-product fill of the all-to-all propagator (Sec. 7, eq. Sfill) and the two routes to
// sum_{z,x} tr[S1 S2^dag]: through the filled propagators (the paper's method, cost ~ T (12
// L^3)^2 N) and through Gram matrices of sources and solutions (cost ~ T 12 L^3 N^2)
// =========================================================================================
static int fill_geo(Ctx* c, const a2a_geom* geom, int nrhs, int t_src, Geo* g) {
  if (geom_to_geo(geom, g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (nrhs < 1) return c->fail(A2A_EINVAL, "nrhs must be positive");
  if (t_src < 0 || t_src >= g->T) return c->fail(A2A_EINVAL, "source timeslice out of range");
  // M = 12 X Y Z rows and columns of the fill: (M / 64)^2 tiles must fit one launch
  if (12LL * g->X * g->Y * g->Z > (1LL << 21)) return c->fail(A2A_EINVAL, "timeslice too large for the fill");
  return A2A_OK;
}

extern "C" int a2a_fill_propagator_dev(a2a_ctx* h, const a2a_geom* geom, const double* sol, const double* src,
                                       int nrhs, int t_src, int t, int dagger, double* S) {
  if (!h || !sol || !src || !S) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  A2A_TRY(fill_geo(c, geom, nrhs, t_src, &g));
  if (t < 0 || t >= g.T) return c->fail(A2A_EINVAL, "sink timeslice out of range");
  const long long M = 12LL * g.X * g.Y * g.Z, col = M * g.T;  // complex per timeslice, per source
  FillArgs a{};
  a.P[0] = sol + 2 * t * M;
  a.Q[0] = src + 2 * t_src * M;
  a.pm = a.qm = 1;
  a.pk = a.qk = col;
  a.M = a.N = (int)M;
  a.K = nrhs;
  a.scale = 1.0 / nrhs;
  a.out = S;
  a.om = M;
  a.on = 1;
  a.dagger = dagger != 0;
  launch_fill(a, 1, c->stream);
  A2A_HIP(c, hipGetLastError());
  return c->sync();
}

extern "C" int a2a_contract_fill_2pt_dev(a2a_ctx* h, const a2a_geom* geom, const double* sol1, const double* src1,
                                         const double* sol2, const double* src2, int nrhs, int t_src,
                                         double* corr) {
  if (!h || !sol1 || !src1 || !sol2 || !src2 || !corr) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  A2A_TRY(fill_geo(c, geom, nrhs, t_src, &g));
  const long long M = 12LL * g.X * g.Y * g.Z, col = M * g.T;
  FillArgs a{};
  a.P[0] = sol1;
  a.P[1] = sol2;
  a.Q[0] = src1 + 2 * t_src * M;
  a.Q[1] = src2 + 2 * t_src * M;
  a.pm = a.qm = 1;
  a.pk = a.qk = col;
  a.pz = M;  // one sink timeslice per grid row
  a.M = a.N = (int)M;
  a.K = nrhs;
  a.scale = 1.0 / nrhs;
  const long long nb = fill_blocks(a.M, a.N);
  void *part = nullptr, *dc = nullptr;
  A2A_TRY(c->dalloc(&part, sizeof(double) * 2 * (size_t)nb * g.T));
  int rc = c->dalloc(&dc, sizeof(double) * 2 * g.T);
  if (!rc) {
    a.partial = (double*)part;
    launch_fill_contract(a, g.T, (double*)dc, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = c->fail(A2A_EDEVICE, std::string("fill contraction: ") + hipGetErrorString(e));
    if (!rc) rc = copy_to_host(c, corr, dc, sizeof(double) * 2 * g.T);
  }
  c->sync();
  c->dfree(part);
  c->dfree(dc);
  return rc;
}

extern "C" int a2a_contract_gram_2pt_dev(a2a_ctx* h, const a2a_geom* geom, const double* sol1, const double* src1,
                                         const double* sol2, const double* src2, int nrhs, int t_src,
                                         double* corr) {
  if (!h || !sol1 || !src1 || !sol2 || !src2 || !corr) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  A2A_TRY(fill_geo(c, geom, nrhs, t_src, &g));
  const int n = nrhs;
  const long K = 12L * g.X * g.Y * g.Z;
  const int ntb = (n + 63) / 64;
  auto chunks = [&](int nt) {
    long want = 4096 / std::max(1, nt * ntb * ntb);
    return (int)std::max(1L, std::min(want, (K + 255) / 256));
  };
  const int ce = chunks(1), cf = chunks(g.T);
  const size_t nn = (size_t)n * n;
  void *part = nullptr, *E = nullptr, *F = nullptr, *dc = nullptr;
  A2A_TRY(c->dalloc(&part, sizeof(double) * 2 * std::max((size_t)ce, (size_t)g.T * cf) * nn));
  int rc = c->dalloc(&E, sizeof(double) * 2 * nn);
  if (!rc) rc = c->dalloc(&F, sizeof(double) * 2 * nn * g.T);
  if (!rc) rc = c->dalloc(&dc, sizeof(double) * 2 * g.T);
  if (!rc) {
    // E[i][j] = <eta1_i, eta2_j> on t_src; F[t][j][i] = <X2_j, X1_i> on t
    launch_stoch_ops(g, n, src1, src2, (double*)part, ce, (double*)E, c->stream, 0, t_src, 1);
    launch_stoch_ops(g, n, sol2, sol1, (double*)part, cf, (double*)F, c->stream, 0, 0, g.T);
    launch_gram_corr(g.T, n, (const double*)E, (const double*)F, (double*)dc, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = c->fail(A2A_EDEVICE, std::string("Gram contraction: ") + hipGetErrorString(e));
    if (!rc) rc = copy_to_host(c, corr, dc, sizeof(double) * 2 * g.T);
  }
  c->sync();
  c->dfree(part);
  c->dfree(E);
  c->dfree(F);
  c->dfree(dc);
  return rc;
}

// =========================================================================================
// point-source propagators and the pi-pi diagrams that combine them with stochastic
// propagators (Sec. 8)
// =========================================================================================
extern "C" int a2a_point_sources_dev(a2a_ctx* h, const a2a_geom* geom, int t0, const int* x0, double* out) {
  if (!h || !x0 || !out) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (t0 < 0 || t0 >= g.T || x0[0] < 0 || x0[0] >= g.X || x0[1] < 0 || x0[1] >= g.Y || x0[2] < 0 || x0[2] >= g.Z)
    return c->fail(A2A_EINVAL, "point outside the lattice");
  const long site = (((long)t0 * g.Z + x0[2]) * g.Y + x0[1]) * g.X + x0[0];
  launch_point_sources(g, site, out, c->stream);
  A2A_HIP(c, hipGetLastError());
  return c->sync();
}

extern "C" int a2a_contract_pipi_mixed_dev(a2a_ctx* h, const a2a_geom* geom, const double* point_sol, int t0,
                                           const double* src1, const double* sol1, int n1, const double* src2,
                                           const double* sol2, int n2, double* diagrams, double* pieces) {
  if (!h || !point_sol || !src1 || !sol1 || !src2 || !sol2 || !diagrams) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (n1 < 1 || n2 < 1) return c->fail(A2A_EINVAL, "n1 and n2 must be positive");
  if (t0 < 0 || t0 >= g.T) return c->fail(A2A_EINVAL, "source timeslice out of range");
  const int T = g.T;
  const long K = 12L * g.X * g.Y * g.Z;
  // the timeslice Gram matrices <a_r, b_s>_t (no gamma_5): rows from `a`, columns from `b`
  struct Gram {
    const double* a;
    int na;
    const double* b;
    int nb, t_first, nt, nchunk;
    size_t elems;  // complex outputs
  };
  Gram gm[5] = {{point_sol, 12, point_sol, 12, 0, T, 0, 0},  // Pn[t][k][l] = <Sp_k, Sp_l>_t
                {src1, n1, src2, n2, 0, T, 0, 0},             // G[t][i][j] = <eta1_i, eta2_j>_t
                {sol1, n1, sol2, n2, 0, T, 0, 0},             // Fp[t][i][j] = <X1_i, X2_j>_t
                {point_sol, 12, sol1, n1, t0, 1, 0, 0},       // A[k][i] = <Sp_k, X1_i>_t0
                {sol2, n2, point_sol, 12, 0, T, 0, 0}};       // B[t][j][k] = <X2_j, Sp_k>_t
  size_t part_elems = 0;
  for (Gram& q : gm) {
    const long tiles = (long)q.nt * ((q.na + 63) / 64) * ((q.nb + 63) / 64);
    q.nchunk = (int)std::max(1L, std::min(4096 / std::max(1L, tiles), (K + 255) / 256));
    q.elems = (size_t)q.nt * q.na * q.nb;
    part_elems = std::max(part_elems, q.elems * q.nchunk);
  }
  const int nmix = pipi_mixed_chunks(n1);
  void* part = nullptr;
  void* out[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  void *mix = nullptr, *dd = nullptr;
  A2A_TRY(c->dalloc(&part, sizeof(double) * 2 * part_elems));
  int rc = A2A_OK;
  for (int q = 0; q < 5 && !rc; ++q) rc = c->dalloc(&out[q], sizeof(double) * 2 * gm[q].elems);
  if (!rc) rc = c->dalloc(&mix, sizeof(double) * 6 * (size_t)T * nmix);
  if (!rc) rc = c->dalloc(&dd, sizeof(double) * 2 * 7 * (size_t)T);  // diagrams [4][T], pieces [3][T]
  if (!rc) {
    // one partial buffer: every Gram launch pair finishes before the next starts (one stream)
    for (int q = 0; q < 5; ++q)
      launch_stoch_ops(g, gm[q].nb, gm[q].a, gm[q].b, (double*)part, gm[q].nchunk, (double*)out[q], c->stream, 0,
                       gm[q].t_first, gm[q].nt, nullptr, nullptr, gm[q].na);
    double* d = (double*)dd;
    launch_pipi_mixed(T, t0, n1, n2, (const double*)out[0], (const double*)out[1], (const double*)out[2],
                      (const double*)out[3], (const double*)out[4], (double*)mix, d, d + 8 * T, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = c->fail(A2A_EDEVICE, std::string("mixed pi-pi contraction: ") + hipGetErrorString(e));
    if (!rc) rc = copy_to_host(c, diagrams, d, sizeof(double) * 8 * T);
    if (!rc && pieces) rc = copy_to_host(c, pieces, d + 8 * T, sizeof(double) * 6 * T);
  }
  c->sync();
  c->dfree(part);
  for (void* p : out) c->dfree(p);
  c->dfree(mix);
  c->dfree(dd);
  return rc;
}

// =========================================================================================
// dilution and momentum projection (Sec. 7: time-spin-colour dilution; Sec. 5: pions projected
// onto momentum states)
// =========================================================================================
static int dilution_size(int scheme, int T) {
  return scheme == A2A_DILUTE_NONE ? 1 : scheme == A2A_DILUTE_T ? T : scheme == A2A_DILUTE_SC ? 12 : 12 * T;
}

extern "C" int a2a_dilute_dev(a2a_ctx* h, const a2a_geom* geom, const double* noise, int nnoise, int scheme,
                              double* out) {
  if (!h || !noise || !out) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (nnoise < 1) return c->fail(A2A_EINVAL, "nnoise must be positive");
  if (scheme < A2A_DILUTE_NONE || scheme > A2A_DILUTE_TSC) return c->fail(A2A_EINVAL, "unknown dilution scheme");
  launch_dilute(g, nnoise, scheme, dilution_size(scheme, g.T), noise, out, c->stream);
  A2A_HIP(c, hipGetLastError());
  return c->sync();
}

// exp(-i p.y) on the spatial sites of a timeslice (x fastest), the angle reduced exactly
static void momentum_phase(const Geo& g, const int* p, std::vector<double>& ph) {
  const long V3 = (long)g.X * g.Y * g.Z;
  ph.resize(2 * V3);
  const double two_pi = 6.283185307179586476925;
  long s = 0;
  for (int z = 0; z < g.Z; ++z)
    for (int y = 0; y < g.Y; ++y)
      for (int x = 0; x < g.X; ++x, ++s) {
        const long ax = (((long)p[0] * x) % g.X + g.X) % g.X, ay = (((long)p[1] * y) % g.Y + g.Y) % g.Y,
                   az = (((long)p[2] * z) % g.Z + g.Z) % g.Z;
        const double f = (double)ax / g.X + (double)ay / g.Y + (double)az / g.Z;
        ph[2 * s] = std::cos(two_pi * f);
        ph[2 * s + 1] = -std::sin(two_pi * f);
      }
}

extern "C" int a2a_contract_pion_mom_dev(a2a_ctx* h, const a2a_geom* geom, const double* src, const double* sol,
                                         int nrhs, int scheme, int nmom, const int* moms, int mode,
                                         double* corr) {
  if (!h || !src || !sol || !moms || !corr) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  Geo g;
  if (geom_to_geo(geom, &g)) return c->fail(A2A_EINVAL, "bad lattice geometry");
  if (scheme < A2A_DILUTE_NONE || scheme > A2A_DILUTE_TSC) return c->fail(A2A_EINVAL, "unknown dilution scheme");
  const int group = dilution_size(scheme, g.T);
  if (nrhs < 1 || nrhs % group) return c->fail(A2A_EINVAL, "nrhs must be a positive multiple of the dilution size");
  if (mode != 0 && mode != 3) return c->fail(A2A_EINVAL, "mode must be 0 (unbiased) or 3 (raw, all pairs)");
  if (mode == 0 && nrhs / group < 2) return c->fail(A2A_EINVAL, "the unbiased estimator needs two noise vectors");
  if (nmom < 1) return c->fail(A2A_EINVAL, "nmom must be positive");
  const int n = nrhs, nv = nrhs / group;
  // time-diluted pieces live on one timeslice: O(t) keeps only the rows of the pieces on t
  const bool by_time = scheme == A2A_DILUTE_T || scheme == A2A_DILUTE_TSC;
  const int per_t = scheme == A2A_DILUTE_TSC ? 12 : 1;
  const int na = by_time ? nv * per_t : n;
  std::vector<int> rows;
  if (by_time) {
    rows.resize((size_t)g.T * na);
    for (int t = 0; t < g.T; ++t)
      for (int i = 0; i < nv; ++i)
        for (int q = 0; q < per_t; ++q) rows[(size_t)t * na + i * per_t + q] = i * group + per_t * t + q;
  }
  const long K = 12L * g.X * g.Y * g.Z;
  const int ntb = (n + 63) / 64, nta = (na + 63) / 64;
  long want = 4096 / std::max(1, g.T * ntb * nta);
  const int nchunk = (int)std::max(1L, std::min(want, (K + 255) / 256));
  const size_t nn = (size_t)na * n;
  const size_t V3 = (size_t)g.X * g.Y * g.Z;
  void *part = nullptr, *Op = nullptr, *Om = nullptr, *ph = nullptr, *dc = nullptr, *drows = nullptr;
  A2A_TRY(c->dalloc(&part, sizeof(double) * 2 * (size_t)g.T * nchunk * nn));
  int rc = c->dalloc(&Op, sizeof(double) * 2 * (size_t)g.T * nn);
  if (!rc) rc = c->dalloc(&Om, sizeof(double) * 2 * (size_t)g.T * nn);
  if (!rc) rc = c->dalloc(&ph, sizeof(double) * 4 * V3);
  if (!rc) rc = c->dalloc(&dc, sizeof(double) * 2 * g.T);
  if (!rc && by_time) {
    rc = c->dalloc(&drows, sizeof(int) * rows.size());
    if (!rc && hipMemcpyAsync(drows, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, c->stream) !=
                   hipSuccess)
      rc = c->fail(A2A_EDEVICE, "row table upload failed");
  }
  std::vector<double> hp, hm;
  for (int m = 0; m < nmom && !rc; ++m) {
    const int* p = moms + 3 * m;
    const int q[3] = {-p[0], -p[1], -p[2]};
    momentum_phase(g, p, hp);
    momentum_phase(g, q, hm);
    double* php = (double*)ph;
    double* phm = php + 2 * V3;
    if (hipMemcpyAsync(php, hp.data(), sizeof(double) * 2 * V3, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(phm, hm.data(), sizeof(double) * 2 * V3, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      rc = c->fail(A2A_EDEVICE, "phase upload failed");
      break;
    }
    const int* dr = (const int*)drows;
    launch_stoch_ops(g, n, src, sol, (double*)part, nchunk, (double*)Op, c->stream, 1, 0, g.T, php, dr, na);
    launch_stoch_ops(g, n, src, sol, (double*)part, nchunk, (double*)Om, c->stream, 1, 0, g.T, phm, dr, na);
    if (by_time)
      launch_pion_mom_rows(g.T, n, na, dr, group, mode, (const double*)Op, (const double*)Om, (double*)dc,
                           c->stream);
    else
      launch_pion_mom(g.T, n, group, mode, (const double*)Op, (const double*)Om, (double*)dc, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = c->fail(A2A_EDEVICE, std::string("momentum contraction: ") + hipGetErrorString(e));
    if (!rc) rc = copy_to_host(c, corr + 2 * (size_t)m * g.T, dc, sizeof(double) * 2 * g.T);
  }
  c->sync();
  c->dfree(part);
  c->dfree(Op);
  c->dfree(Om);
  c->dfree(ph);
  c->dfree(dc);
  c->dfree(drows);
  return rc;
}

// =========================================================================================
// serving engine: continuous batching
// =========================================================================================
struct Request {
  long long ticket;
  int clover_h;
  double kappa;
  const double* src;
  double* sol;
  int nsrc;
  double tol;
  int prec;
  int max_iter;
  int method = SOLVER_BICGSTAB;
  int state = 0;  // 0 queued, 1 running, 2 done, -1 failed
  int err = A2A_OK;
  double t_submit = 0;
  std::vector<Slot> slots;
};

struct a2a_engine {
  a2a_ctx* h;
  int max_slots = 256;
  int max_queue = 4096;
  std::deque<Request*> queue;
  std::map<long long, std::unique_ptr<Request>> reqs;
  std::unique_ptr<Solver> solvers[8];  // [method * 4 + precision]
  long long next_ticket = 1;
  int active = 0;
};

extern "C" int a2a_engine_create(a2a_ctx* h, const char* policy, a2a_engine** out) {
  if (!h || !out) return A2A_EINVAL;
  auto* e = new a2a_engine();
  e->h = h;
  e->max_slots = (int)json_num(policy, "max_slots", 256);
  e->max_queue = (int)json_num(policy, "max_queue", 4096);
  int ce = (int)json_num(policy, "check_every", h->c.check_every);
  if (e->max_slots < 1 || e->max_queue < 1 || ce < 1) {
    delete e;
    return h->c.fail(A2A_EINVAL, "bad engine policy");
  }
  h->c.check_every = ce;
  *out = e;
  return A2A_OK;
}

extern "C" int a2a_engine_submit(a2a_engine* e, int clover_h, double kappa, const double* src, int nsrc, double tol,
                                 int prec, int max_iter, double* sol, long long* ticket) {
  if (!e || !ticket) return A2A_EINVAL;
  Ctx* c = &e->h->c;
  if (!src || !sol || nsrc <= 0 || !(tol > 0) || check_prec(prec) || max_iter <= 0 || !(kappa > 0))
    return c->fail(A2A_EINVAL, "bad request");
  if (!c->clover(clover_h)) return c->fail(A2A_EHANDLE, "unknown clover handle");
  if (nsrc > e->max_slots) return c->fail(A2A_EINVAL, "request larger than the engine's slot capacity");
  if ((int)e->queue.size() >= e->max_queue) return c->fail(A2A_EAGAIN, "queue full");
  auto r = std::make_unique<Request>();
  r->ticket = e->next_ticket++;
  r->clover_h = clover_h;
  r->kappa = kappa;
  r->src = src;
  r->sol = sol;
  r->nsrc = nsrc;
  r->tol = tol;
  r->prec = prec;
  r->max_iter = max_iter;
  r->method = c->solver;
  r->t_submit = now_seconds();
  e->queue.push_back(r.get());
  *ticket = r->ticket;
  e->reqs[r->ticket] = std::move(r);
  return A2A_OK;
}

static void engine_release(a2a_engine* e, Request* r) {
  Ctx* c = &e->h->c;
  for (auto& s : r->slots) slot_free(c, &s);
  e->active -= r->nsrc;
}

// try to admit one request; returns A2A_OK (admitted), A2A_ENOMEM (no room now), or an error
static int engine_admit(a2a_engine* e, Request* r) {
  Ctx* c = &e->h->c;
  GaugeField* gf;
  CloverField* cf;
  KappaOp* kop;
  int rc = resolve_op(c, r->clover_h, r->kappa, r->prec, &gf, &cf, &kop);
  if (rc) return rc;
  auto& sv = e->solvers[r->method * 4 + r->prec];
  if (!sv) {
    sv = std::make_unique<Solver>(c, r->prec, effective_R(c, r->prec));
    sv->method = r->method;
  }
  const int op = sv->op_index(r->clover_h, r->kappa, kop, gf);
  const long long V = volume_of(gf->g);
  r->slots.assign(r->nsrc, Slot());
  for (int i = 0; i < r->nsrc; ++i) {
    Slot& s = r->slots[i];
    s.op = op;
    s.src = r->src + (size_t)i * 24 * V;
    s.sol = r->sol + (size_t)i * 24 * V;
    s.tol = r->tol;
    s.max_iter = r->max_iter;
    s.t_submit = r->t_submit;
    s.req = r->ticket;
    s.req_idx = i;
  }
  rc = slots_alloc(c, r->slots.data(), r->nsrc, r->prec, gf->g.hv, sv->ops[op].nblk, NVEC_LO, NVEC_HI);
  if (rc) {
    r->slots.clear();
    return rc;
  }
  e->active += r->nsrc;
  std::vector<int> idx;
  for (auto& s : r->slots) {
    idx.push_back((int)sv->live.size());
    sv->add_slot(&s);
  }
  rc = sv->setup(idx);
  std::vector<int> early;
  if (!rc)
    for (int i : idx)
      if (sv->live[i]->state == SS_RUN && sv->live[i]->last_r64 <= sv->live[i]->target) early.push_back(i);
  if (!rc && !early.empty()) {
    rc = sv->finalize(early);
    if (!rc)
      for (int i : early) sv->live[i]->state = sv->live[i]->info.converged ? SS_DONE : SS_RUN;
  }
  if (rc) {
    // undo the admission: the request's slots leave the solver's tables and give back their
    // arenas and ids, so that a retry (ENOMEM) starts from scratch and a failed request holds
    // neither slot capacity nor memory
    (void)c->sync();
    Slot* first = r->slots.data();
    Slot* last = first + r->slots.size();
    auto& lv = sv->live;
    lv.erase(std::remove_if(lv.begin(), lv.end(), [&](Slot* s) { return s >= first && s < last; }), lv.end());
    sv->dirty = true;
    engine_release(e, r);
    r->slots.clear();
    return rc;
  }
  r->state = 1;
  return A2A_OK;
}

extern "C" int a2a_engine_step(a2a_engine* e, int iters, int* active) {
  if (!e || iters < 0) return A2A_EINVAL;
  Ctx* c = &e->h->c;
  (void)hipSetDevice(c->device);
  // admission, first come first served, by slot capacity and the HBM budget
  while (!e->queue.empty()) {
    Request* r = e->queue.front();
    if (r->state == -1) {  // cancelled while queued
      e->queue.pop_front();
      continue;
    }
    if (e->active + r->nsrc > e->max_slots) break;
    int rc = engine_admit(e, r);
    if (rc == A2A_ENOMEM && c->evict_unused_kops() > 0) {  // drop clover fields of finished kappas
      c->err.clear();
      rc = engine_admit(e, r);
    }
    if (rc == A2A_ENOMEM && e->active > 0) {  // wait for memory to free up
      c->err.clear();
      break;
    }
    e->queue.pop_front();
    if (rc) {
      r->state = -1;
      r->err = rc;
      for (auto& s : r->slots) s.state = SS_FAIL;
    }
  }
  // iterate every active slot of every precision and method
  for (auto& sv : e->solvers)
    if (sv) A2A_TRY(sv->run_steps(iters));
  // retire finished requests
  for (auto& kv : e->reqs) {
    Request* r = kv.second.get();
    if (r->state != 1) continue;
    bool all = true, failed = false;
    for (auto& s : r->slots) {
      if (s.state != SS_DONE && s.state != SS_FAIL) all = false;
      if (s.state == SS_FAIL) {
        failed = true;
        if (r->err == A2A_OK) r->err = s.err;
      }
    }
    if (all) {
      r->state = failed ? -1 : 2;
      engine_release(e, r);
    }
  }
  if (active) *active = e->active;
  return A2A_OK;
}

extern "C" int a2a_engine_poll(a2a_engine* e, long long ticket, int* done, a2a_solve_info* info) {
  if (!e || !done) return A2A_EINVAL;
  auto it = e->reqs.find(ticket);
  if (it == e->reqs.end()) return e->h->c.fail(A2A_EHANDLE, "unknown ticket");
  Request* r = it->second.get();
  *done = r->state == 2 ? 1 : (r->state == -1 ? -1 : 0);
  if (info && (r->state == 2 || r->state == -1) && !r->slots.empty())
    for (int i = 0; i < r->nsrc; ++i) info[i] = r->slots[i].info;
  return r->state == -1 ? r->err : A2A_OK;
}

extern "C" int a2a_engine_cancel(a2a_engine* e, long long ticket) {
  if (!e) return A2A_EINVAL;
  auto it = e->reqs.find(ticket);
  if (it == e->reqs.end()) return e->h->c.fail(A2A_EHANDLE, "unknown ticket");
  Request* r = it->second.get();
  if (r->state == 0) {
    r->state = -1;
    r->err = A2A_EINVAL;
  } else if (r->state == 1) {
    for (auto& s : r->slots)
      if (s.state != SS_DONE) {
        s.state = SS_FAIL;
        s.err = A2A_EINVAL;
      }
  }
  return A2A_OK;
}

extern "C" int a2a_engine_destroy(a2a_engine* e) {
  if (!e) return A2A_EINVAL;
  Ctx* c = &e->h->c;
  (void)c->sync();
  for (auto& kv : e->reqs)
    if (kv.second->state == 1) engine_release(e, kv.second.get());
  for (auto& s : e->solvers) s.reset();
  delete e;
  c->release_cache();
  return A2A_OK;
}

extern "C" int a2a_trim(a2a_ctx* h, size_t* released) {
  if (!h) return A2A_EINVAL;
  Ctx* c = &h->c;
  (void)hipSetDevice(c->device);
  const size_t n = c->cached;
  c->release_cache();
  if (released) *released = n;
  return A2A_OK;
}
