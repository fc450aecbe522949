// runtime.cpp -- context, resident fields and the batched mixed-precision BiCGStab solver.
//
// Solve (Sec. 7: X_i = D^{-1} eta_i for every noise source) with even-odd preconditioning:
//   b_o = eta_o + kappa H_oe A_ee^{-1} eta_e,   M = A_oo - kappa^2 H_oe A_ee^{-1} H_eo,
//   M x_o = b_o,   x_e = A_ee^{-1} (eta_e + kappa H_eo x_o).
// The odd system is solved by BiCGStab on all right-hand sides in lock step (one launch
// per step for the whole batch) in the working precision, and corrected by FP64 reliable
// updates: when the iterated residual has dropped by `delta` since the last update, x is
// folded into the FP64 solution and the residual is recomputed from it with FP64 fields.
// A source is done when the FP64 residual of the full system, ||eta - D X|| / ||eta||,
// recomputed after reconstruction, is at most tol.
#include "runtime.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>

namespace a2a {

double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int geom_to_geo(const a2a_geom* geom, Geo* g) {
  if (!geom) return A2A_EINVAL;
  for (int m = 0; m < 4; ++m)
    if (geom->dims[m] < 2 || (geom->dims[m] & 1)) return A2A_EINVAL;
  if (geom->t_bc != 1 && geom->t_bc != -1) return A2A_EINVAL;
  long long V = 1;
  for (int m = 0; m < 4; ++m) V *= geom->dims[m];
  if (V / 2 > (1LL << 30)) return A2A_EINVAL;
  g->X = geom->dims[0];
  g->Y = geom->dims[1];
  g->Z = geom->dims[2];
  g->T = geom->dims[3];
  g->Xh = g->X / 2;
  g->hv = (int)(V / 2);
  g->tbc = geom->t_bc;
  // stencil bricks: the whole x row (xh extent up to 16), then extents in y, z, t that divide
  // the lattice, aiming at BS sites per brick with the extra extent spread over y, z and t
  int bx = g->Xh;
  while (bx > 16 && bx % 2 == 0) bx /= 2;
  g->bxh = (unsigned char)bx;
  int ch[1][3];
  brick_choices(*g, ch, 1);
  g->by = (unsigned char)ch[0][0];
  g->bz = (unsigned char)ch[0][1];
  g->bt = (unsigned char)ch[0][2];
  return A2A_OK;
}

int brick_choices(const Geo& g, int (*out)[3], int maxn) {
  static const int cand[][3] = {{4, 2, 2}, {2, 2, 4}, {2, 4, 2}, {4, 4, 1}, {8, 2, 1}, {8, 1, 2}, {2, 2, 2},
                                {4, 2, 1}, {2, 2, 1}, {4, 1, 1}, {2, 1, 1}, {1, 1, 1}};
  const int target = std::max(1, BS / std::max(1, (int)g.bxh));
  int n = 0;
  for (const auto& c : cand) {
    if (n >= maxn) break;
    if (c[0] * c[1] * c[2] > target) continue;
    if (g.Y % c[0] || g.Z % c[1] || g.T % c[2]) continue;
    out[n][0] = c[0];
    out[n][1] = c[1];
    out[n][2] = c[2];
    ++n;
  }
  return n;
}

// Workgroups are dispatched round-robin over the 8 XCDs (dispatch index i -> XCD i % 8).
// Reorder a tile list so that XCD k receives the k-th contiguous eighth of the logical
// order: neighbouring lattice slabs (and all RHS groups of one slab) share an L2.
void xcd_order(std::vector<int2>& tiles, bool enable) {
  const int n = (int)tiles.size();
  if (!enable || n < 16) return;
  static thread_local std::vector<int2> out;  // reused: the lists are rebuilt at every residual check
  out.resize(n);
  int start[8], cnt[8];
  int acc = 0;
  for (int k = 0; k < 8; ++k) {
    cnt[k] = n / 8 + (k < n % 8 ? 1 : 0);
    start[k] = acc;
    acc += cnt[k];
  }
  for (int i = 0; i < n; ++i) out[i] = tiles[start[i % 8] + i / 8];
  tiles.swap(out);
}

// ------------------------------------------------------------------------------------------
// context memory
// ------------------------------------------------------------------------------------------
int Ctx::dalloc(void** p, size_t n) {
  *p = nullptr;
  if (n == 0) return A2A_OK;
  n = (n + 255) & ~(size_t)255;
  // a cached block of this size, or at most 1/8 larger
  auto it = cache.lower_bound(n);
  if (it != cache.end() && it->first <= n + n / 8) {
    const size_t sz = it->first;
    *p = it->second;
    cache.erase(it);
    cached -= sz;
    used += sz;
    sizes[*p] = sz;
    if (poison) (void)hipMemsetAsync(*p, 0xFF, sz, stream);
    return A2A_OK;
  }
  if (used + n > budget)
    return fail(A2A_ENOMEM, "HBM budget exceeded: need " + std::to_string(n) + " B, " +
                                std::to_string(budget - std::min(budget, used)) + " B left");
  if (used + cached + n > budget) release_cache();
  hipError_t e = hipMalloc(p, n);
  if (e != hipSuccess && cached > 0) {
    (void)hipGetLastError();
    release_cache();
    e = hipMalloc(p, n);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(A2A_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  used += n;
  sizes[*p] = n;
  if (poison) (void)hipMemsetAsync(*p, 0xFF, n, stream);
  return A2A_OK;
}

void Ctx::dfree(void* p) {
  if (!p) return;
  auto it = sizes.find(p);
  if (it == sizes.end()) return;  // not a block of this context
  const size_t sz = it->second;
  used -= sz;
  sizes.erase(it);
  cache.emplace(sz, p);
  cached += sz;
}

void Ctx::release_cache() {
  for (auto& kv : cache) (void)hipFree(kv.second);  // hipFree waits for work still using them
  cache.clear();
  cached = 0;
}

int Ctx::alloc_sid(int nblk, int* sid) {
  int s = -1;
  for (int i = 0; i < (int)sid_used.size(); ++i)
    if (!sid_used[i]) {
      s = i;
      break;
    }
  if (s < 0) {
    if ((int)sid_used.size() >= sid_cap) return fail(A2A_ENOMEM, "too many concurrent right-hand sides");
    s = (int)sid_used.size();
    sid_used.push_back(0);
  }
  sid_used[s] = 1;
  sid_max = std::max(sid_max, s);
  A2A_TRY(ensure_partials(sid_max + 1, nblk));
  *sid = s;
  return A2A_OK;
}

void Ctx::free_sid(int sid) {
  if (sid >= 0 && sid < (int)sid_used.size()) sid_used[sid] = 0;
  while (sid_max >= 0 && !sid_used[sid_max]) --sid_max;
}

int Ctx::ensure_partials(int nslots, int nblk) {
  if (nslots <= partial_slots && nblk <= partial_blk) return A2A_OK;
  int ns = std::max(nslots, partial_slots);
  ns = std::max(ns, 64);
  int nb = std::max(nblk, partial_blk);
  A2A_TRY(sync());
  dfree(partials);
  partials = nullptr;
  void* p;
  A2A_TRY(dalloc(&p, sizeof(double) * 4 * (size_t)ns * nb));
  partials = (double*)p;
  partial_slots = ns;
  partial_blk = nb;
  return A2A_OK;
}

// ------------------------------------------------------------------------------------------
// kernel timing (HIP events on the context stream)
// ------------------------------------------------------------------------------------------
static hipEvent_t take_event(Ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int Ctx::timing_begin(int cls, hipEvent_t* a) {
  (void)cls;
  *a = nullptr;
  if (!timing) return A2A_OK;
  *a = take_event(this);
  if (*a) A2A_HIP(this, hipEventRecord(*a, stream));
  return A2A_OK;
}

int Ctx::timing_end(int cls, hipEvent_t a, double alg_bytes) {
  if (!timing || !a) return A2A_OK;
  hipEvent_t b = take_event(this);
  if (!b) return A2A_OK;
  A2A_HIP(this, hipEventRecord(b, stream));
  pending.push_back({cls, a, b, alg_bytes});
  if (pending.size() > 4096) return timing_collect();
  return A2A_OK;
}

int Ctx::timing_collect() {
  if (pending.empty()) return A2A_OK;
  A2A_TRY(sync());
  for (auto& r : pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      t_launches[r.cls]++;
      t_ms[r.cls] += ms;
      t_bytes[r.cls] += r.bytes;
    }
    ev_pool.push_back(r.a);
    ev_pool.push_back(r.b);
  }
  pending.clear();
  return A2A_OK;
}

// ------------------------------------------------------------------------------------------
// resident fields
// ------------------------------------------------------------------------------------------
static size_t link_bytes(int prec, long hv) {
  switch (prec) {
    case 0: return 4 * LinkF<double>::bytes(hv);
    case 1: return 4 * LinkF<float>::bytes(hv);
    case 2: return 4 * LinkF<_Float16>::bytes(hv);
    default: return 4 * LinkF<bf16_t>::bytes(hv);
  }
}

static size_t clov_bytes(int prec, long hv) {
  switch (prec) {
    case 0: return clover_bytes<double>(hv);
    case 1: return clover_bytes<float>(hv);
    case 2: return clover_bytes<_Float16>(hv);
    default: return clover_bytes<bf16_t>(hv);
  }
}

static size_t spinor_bytes(int prec, long hv) {
  size_t b;
  switch (prec) {
    case 0: b = SpinorF<double>::bytes(hv); break;
    case 1: b = SpinorF<float>::bytes(hv); break;
    case 2: b = SpinorF<_Float16>::bytes(hv); break;
    default: b = SpinorF<bf16_t>::bytes(hv); break;
  }
  return (b + 255) & ~(size_t)255;
}

int Ctx::gauge_links(GaugeField* gf, int prec, void** out0, void** out1) {
  if (!gf->U[prec][0]) {
    void* d[2] = {nullptr, nullptr};
    for (int p = 0; p < 2; ++p) {
      int rc = dalloc(&d[p], link_bytes(prec, gf->g.hv));
      if (rc) {
        dfree(d[0]);
        return rc;
      }
    }
    launch_gauge_to_eo(prec, gf->g, gf->canon, d, stream);
    A2A_HIP(this, hipGetLastError());
    gf->U[prec][0] = d[0];
    gf->U[prec][1] = d[1];
  }
  *out0 = gf->U[prec][0];
  *out1 = gf->U[prec][1];
  return A2A_OK;
}

int Ctx::hop_links(GaugeField* gf, int prec) {
  if (prec != 2 && prec != 3) return A2A_OK;
  if (gf->HL[prec][0]) return A2A_OK;
  void* d[2] = {nullptr, nullptr};
  for (int p = 0; p < 2; ++p) {
    int rc = dalloc(&d[p], (size_t)gf->g.hv * 288);
    if (rc) {
      dfree(d[0]);
      return rc;
    }
  }
  for (int p = 0; p < 2; ++p) launch_hop_links(prec, gf->g, gf->canon, p, d[p], stream);
  A2A_HIP(this, hipGetLastError());
  gf->HL[prec][0] = d[0];
  gf->HL[prec][1] = d[1];
  return A2A_OK;
}

int Ctx::clover_full(KappaOp* k, int prec, long hv) {
  if (prec != 2 && prec != 3) return A2A_OK;
  if (k->AF[prec][0]) return A2A_OK;
  void* d[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < 4; ++i) {
    int rc = dalloc(&d[i], (size_t)hv * 288);
    if (rc) {
      for (int j = 0; j < i; ++j) dfree(d[j]);
      return rc;
    }
  }
  for (int p = 0; p < 2; ++p) {
    launch_clover_full(prec, hv, k->A64[p], d[p], stream);
    launch_clover_full(prec, hv, k->Ai64[p], d[2 + p], stream);
    k->AF[prec][p] = d[p];
    k->AIF[prec][p] = d[2 + p];
  }
  A2A_HIP(this, hipGetLastError());
  return A2A_OK;
}

static void free_kop(Ctx* c, KappaOp* k) {
  for (int p = 0; p < 2; ++p) {
    c->dfree(k->A64[p]);
    c->dfree(k->Ai64[p]);
    for (int q = 1; q < 4; ++q) {
      c->dfree(k->Alo[q][p]);
      c->dfree(k->Ailo[q][p]);
      c->dfree(k->AF[q][p]);
      c->dfree(k->AIF[q][p]);
      k->AF[q][p] = k->AIF[q][p] = nullptr;
    }
    k->A64[p] = k->Ai64[p] = nullptr;
  }
}

// Free the per-kappa clover fields that no solver references (least recently used first is
// not needed: everything unreferenced goes).  Returns the number of bytes released.
size_t Ctx::evict_unused_kops() {
  const size_t before = used;
  for (auto& kv : clovers) {
    auto& v = kv.second->kops;
    for (auto& k : v)
      if (k->refs <= 0) free_kop(this, k.get());
    v.erase(std::remove_if(v.begin(), v.end(), [](const std::unique_ptr<KappaOp>& k) { return k->refs <= 0; }),
            v.end());
  }
  return before - used;
}

// A(kappa), A^{-1}(kappa) for a clover field, FP64 always and `prec` on demand; cached.
int Ctx::kappa_op(CloverField* cf, double kappa, int prec, KappaOp** out) {
  KappaOp* k = nullptr;
  for (auto& kp : cf->kops)
    if (kp->kappa == kappa) k = kp.get();
  GaugeField* gf = gauge(cf->gauge);
  const long hv = gf->g.hv;
  if (!k) {
    auto nk = std::make_unique<KappaOp>();
    nk->kappa = kappa;
    const size_t cb = clov_bytes(0, hv);
    for (int p = 0; p < 2; ++p) {
      void *a = nullptr, *ai = nullptr;
      int rc = dalloc(&a, cb);
      if (!rc) rc = dalloc(&ai, cb);
      if (rc) {
        dfree(a);
        free_kop(this, nk.get());
        return rc;
      }
      nk->A64[p] = (double*)a;
      nk->Ai64[p] = (double*)ai;
      Geo g = gf->g;
      launch_clover_make(g, cf->G[p], kappa * cf->csw, nk->A64[p], nk->Ai64[p], stream);
      A2A_HIP(this, hipGetLastError());
    }
    k = nk.get();
    cf->kops.push_back(std::move(nk));
  }
  if (prec != 0 && !k->Alo[prec][0]) {
    const size_t cb = clov_bytes(prec, hv);
    for (int p = 0; p < 2; ++p) {
      void *a = nullptr, *ai = nullptr;
      int rc = dalloc(&a, cb);
      if (!rc) rc = dalloc(&ai, cb);
      if (rc) {
        dfree(a);
        return rc;
      }
      launch_clover_convert(prec, hv, k->A64[p], a, stream);
      launch_clover_convert(prec, hv, k->Ai64[p], ai, stream);
      A2A_HIP(this, hipGetLastError());
      k->Alo[prec][p] = a;
      k->Ailo[prec][p] = ai;
    }
  }
  k->last_use = ++use_clock;
  *out = k;
  return A2A_OK;
}

// ------------------------------------------------------------------------------------------
// Solver
// ------------------------------------------------------------------------------------------
Solver::Solver(Ctx* c, int p, int r)
    : ctx(c),
      prec(p),
      R(r),
      R64(c->rhs_block64 == 1 ? 1 : 2),
      by(c->brick_by),
      bz(c->brick_bz),
      bt(c->brick_bt),
      mfma_slab(c->mfma_slab) {}

Solver::~Solver() {
  ctx->dfree(d_ops);
  ctx->dfree(d_slots);
  ctx->dfree(d_groups);
  ctx->dfree(d_hop_tiles);
  ctx->dfree(d_vec_tiles);
  ctx->dfree(d_sub_groups);
  ctx->dfree(d_sub_tiles);
  ctx->dfree(d_sub_list);
  ctx->dfree(d_vec_nonil);
  ctx->dfree(d_il_slots);
  ctx->dfree(d_il_tiles);
  ctx->dfree(d_sub_il_slots);
  ctx->dfree(d_ilgroups);
  ctx->dfree(d_il_hop_tiles);
  ctx->dfree(d_groups_nonil);
  ctx->dfree(d_hop_nonil);
  for (auto& o : ops)
    if (o.kop) o.kop->refs--;
}

static int grow(Ctx* c, void** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return A2A_OK;
  size_t n = std::max(need, (size_t)2 * *cap);
  n = std::max(n, (size_t)4096);
  c->dfree(*p);
  *p = nullptr;
  *cap = 0;
  A2A_TRY(c->dalloc(p, n));
  *cap = n;
  return A2A_OK;
}

static void set_mfma_fields(OpDev& d, int prec, const KappaOp* kop, const GaugeField* gf) {
  for (int p = 0; p < 2; ++p) {
    d.HL[p] = (prec == 2 || prec == 3) ? gf->HL[prec][p] : nullptr;
    d.AF[p] = (prec == 2 || prec == 3) ? kop->AF[prec][p] : nullptr;
    d.AIF[p] = (prec == 2 || prec == 3) ? kop->AIF[prec][p] : nullptr;
  }
}

int Solver::op_index(int clover_h, double kappa, KappaOp* kop, const GaugeField* gf) {
  for (int i = 0; i < (int)ops.size(); ++i)
    if (ops[i].clover_h == clover_h && ops[i].kappa == kappa) {
      OpDev d = ops[i].dev;
      set_mfma_fields(d, prec, kop, gf);
      if (std::memcmp(&d, &ops[i].dev, sizeof(OpDev)) != 0) {  // fields built since
        ops[i].dev = d;
        dirty = true;
      }
      return i;
    }
  OpEntry e{};
  e.clover_h = clover_h;
  e.kappa = kappa;
  e.kop = kop;
  kop->refs++;
  e.dev.g = gf->g;
  if (by > 0 && bz > 0 && bt > 0 && gf->g.Y % by == 0 && gf->g.Z % bz == 0 && gf->g.T % bt == 0) {
    e.dev.g.by = (unsigned char)by;  // a tuned brick (any brick tiling the lattice is a valid sweep)
    e.dev.g.bz = (unsigned char)bz;
    e.dev.g.bt = (unsigned char)bt;
  }
  e.dev.kappa = kappa;
  for (int p = 0; p < 2; ++p) {
    e.dev.U[0][p] = gf->U[prec][p];
    e.dev.U[1][p] = gf->U[0][p];
    e.dev.A[1][p] = kop->A64[p];
    e.dev.Ai[1][p] = kop->Ai64[p];
    e.dev.A[0][p] = prec == 0 ? kop->A64[p] : kop->Alo[prec][p];
    e.dev.Ai[0][p] = prec == 0 ? kop->Ai64[p] : kop->Ailo[prec][p];
  }
  set_mfma_fields(e.dev, prec, kop, gf);
  e.nblk = (gf->g.hv + BS - 1) / BS;
  ops.push_back(e);
  dirty = true;
  return (int)ops.size() - 1;
}

int Solver::add_slot(Slot* s) {
  live.push_back(s);
  dirty = true;
  return A2A_OK;
}

// Host table -> device, in stream order.  Small uploads go through the context's pinned staging
// buffer and return at once (the caller's host vector may go away; the device copy happens
// before any later kernel of the stream reads dst); a synchronising copy from the caller's
// memory otherwise.  (Synchronising every upload had left the GPU idle ~14 ms per 32^3x64 step,
// four round trips per subset upload at each residual check.)
static int upload(Ctx* c, void* dst, const void* src, size_t n) {
  if (!n) return A2A_OK;
  const size_t STAGE = c->stage_req ? c->stage_req : (size_t)64 << 20;
  if (!c->stage && !c->stage_failed) {
    if (hipHostMalloc((void**)&c->stage, STAGE, hipHostMallocDefault) == hipSuccess) {
      c->stage_cap = STAGE;
      c->stage_off = 0;
    } else {
      (void)hipGetLastError();
      c->stage = nullptr;
      c->stage_failed = true;
    }
  }
  if (c->stage && n <= c->stage_cap / 4) {
    if (c->stage_off + n > c->stage_cap) A2A_TRY(c->sync());  // frees the whole buffer
    char* p = c->stage + c->stage_off;
    std::memcpy(p, src, n);
    A2A_HIP(c, hipMemcpyAsync(dst, p, n, hipMemcpyHostToDevice, c->stream));
    c->stage_off += (n + 255) & ~(size_t)255;
    return A2A_OK;
  }
  A2A_HIP(c, hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream));
  return c->sync();
}

// Drop operators no live slot uses (their per-kappa clover may then be evicted).
void Solver::gc_ops() {
  std::vector<int> used(ops.size(), 0);
  for (Slot* s : live) used[s->op] = 1;
  bool all = true;
  for (int u : used) all = all && u;
  if (all) return;
  std::vector<int> remap(ops.size(), -1);
  std::vector<OpEntry> keep;
  for (size_t i = 0; i < ops.size(); ++i) {
    if (used[i]) {
      remap[i] = (int)keep.size();
      keep.push_back(ops[i]);
    } else if (ops[i].kop) {
      ops[i].kop->refs--;
    }
  }
  for (Slot* s : live) s->op = remap[s->op];
  ops.swap(keep);
  dirty = true;
}

// Vector-kernel tile lists for the slots idx (indices into live): per-slot tiles of every
// slot, per-slot tiles of the slots outside interleaved groups, and the interleaved lane
// tiles (16 lanes of one group tile) with their site blocks.
static void vec_lists(const std::vector<Slot*>& live, const std::vector<OpEntry>& ops, const std::vector<int>& idx,
                      bool xcd, std::vector<int2>& all, std::vector<int2>& nonil, std::vector<int>& ils,
                      std::vector<int2>& ilt) {
  for (int o = 0; o < (int)ops.size(); ++o) {
    std::vector<int> mine;
    for (int i : idx)
      if (live[i]->op == o) mine.push_back(i);
    if (mine.empty()) continue;
    std::map<std::pair<char*, int>, int> ent;  // (group, tile) -> lane-tile index
    const int e0 = (int)(ils.size() / 16);
    for (int i : mine) {
      const Slot* s = live[i];
      if (!s->il_base) continue;
      auto key = std::make_pair(s->il_base, s->il_lane / 16);
      auto it = ent.find(key);
      int e;
      if (it == ent.end()) {
        e = (int)(ils.size() / 16);
        ent[key] = e;
        ils.insert(ils.end(), 16, -1);
      } else {
        e = it->second;
      }
      ils[(size_t)e * 16 + s->il_lane % 16] = i;
    }
    const int e1 = (int)(ils.size() / 16);
    all.reserve(all.size() + (size_t)ops[o].nblk * mine.size());
    ilt.reserve(ilt.size() + (size_t)ops[o].nblk * (e1 - e0));
    for (int b = 0; b < ops[o].nblk; ++b) {
      for (int i : mine) {
        all.push_back(make_int2(i, b));
        if (!live[i]->il_base) nonil.push_back(make_int2(i, b));
      }
      for (int e = e0; e < e1; ++e) ilt.push_back(make_int2(e, b));
    }
  }
  xcd_order(all, xcd);
  xcd_order(nonil, xcd);
  xcd_order(ilt, xcd);
}

int Solver::rebuild() {
  if (!dirty) return A2A_OK;
  ++gen;  // slot indices and tables change: earlier subset uploads are stale
  gc_ops();
  // ops and slots
  A2A_TRY(grow(ctx, (void**)&d_ops, &cap_ops, sizeof(OpDev) * std::max<size_t>(1, ops.size())));
  std::vector<OpDev> hops(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) hops[i] = ops[i].dev;
  A2A_TRY(upload(ctx, d_ops, hops.data(), sizeof(OpDev) * hops.size()));
  const size_t n = live.size();
  A2A_TRY(grow(ctx, (void**)&d_slots, &cap_slots, sizeof(SlotDev) * std::max<size_t>(1, n)));
  std::vector<SlotDev> hs(n);
  for (size_t i = 0; i < n; ++i) {
    Slot* s = live[i];
    SlotDev& d = hs[i];
    d.op = s->op;
    d.nblk = ops[s->op].nblk;
    d.sid = s->sid;
    d.pad = 0;
    d.arena[0] = s->lo;
    d.arena[1] = s->hi;
    d.vstride[0] = (long long)s->lo_stride;
    d.vstride[1] = (long long)s->hi_stride;
    d.lss = s->lss;
    d.lcs = s->lcs;
    d.lss_x = s->lss_x;
    d.lxoff = s->lxoff;
    d.scal = ctx->scal_pool + (size_t)s->sid * NSCAL;
    d.src = s->src;
    d.sol = s->sol;
    d.x0 = s->x0;
  }
  A2A_TRY(upload(ctx, d_slots, hs.data(), sizeof(SlotDev) * n));
  // groups of R slots sharing an operator, and tile lists
  std::vector<int> groups;
  std::vector<int2> htiles, vtiles, nonil, ilt;
  std::vector<int> ils;
  std::vector<int> every;
  for (size_t i = 0; i < n; ++i) every.push_back((int)i);
  for (int o = 0; o < (int)ops.size(); ++o) {
    std::vector<int> mine;
    for (size_t i = 0; i < n; ++i)
      if (live[i]->op == o) mine.push_back((int)i);
    if (mine.empty()) continue;
    const int g0 = (int)(groups.size() / R);
    const int ng = (int)((mine.size() + R - 1) / R);
    for (int gi = 0; gi < ng; ++gi)
      for (int r = 0; r < R; ++r) {
        size_t k = (size_t)gi * R + r;
        groups.push_back(k < mine.size() ? mine[k] : -1);
      }
    for (int b = 0; b < ops[o].nblk; ++b)
      for (int gi = 0; gi < ng; ++gi) htiles.push_back(make_int2(g0 + gi, b));
  }
  xcd_order(htiles, xcd_hop >= 0 ? xcd_hop != 0 : ctx->xcd_order != 0);
  vec_lists(live, ops, every, ctx->xcd_order, vtiles, nonil, ils, ilt);
  // interleaved groups for the matrix-core stencil, and R-groups of the remaining slots
  std::vector<ILGroupDev> ilg;
  std::vector<int2> ilh, hnon;
  std::vector<int> gnon;
  il_mfma = true;
  il_nt3 = true;
  for (int o = 0; o < (int)ops.size(); ++o) {
    std::map<char*, int> gidx;
    std::vector<int> rest;
    const int e0 = (int)ilg.size();
    for (size_t i = 0; i < n; ++i) {
      const Slot* s = live[i];
      if (s->op != o) continue;
      if (!s->il_base) {
        rest.push_back((int)i);
        continue;
      }
      auto it = gidx.find(s->il_base);
      if (it == gidx.end()) {
        ILGroupDev d{};
        d.op = o;
        d.nt = s->il_nt;
        d.base = s->il_base;
        d.vs = (long long)s->lo_stride;
        for (int l = 0; l < IL_LANES; ++l) d.slot[l] = -1;
        it = gidx.emplace(s->il_base, (int)ilg.size()).first;
        ilg.push_back(d);
      }
      ilg[it->second].slot[s->il_lane] = (int)i;
    }
    const int e1 = (int)ilg.size();
    if (e1 > e0 && !(ops[o].dev.HL[0] && ops[o].dev.AF[0] && ops[o].dev.AIF[0])) il_mfma = false;
    for (int e = e0; e < e1; ++e) il_nt3 = il_nt3 && ilg[e].nt == 3;
    const int g0 = (int)(gnon.size() / R);
    const int ng = (int)((rest.size() + R - 1) / R);
    for (int gi = 0; gi < ng; ++gi)
      for (int r = 0; r < R; ++r) {
        size_t k = (size_t)gi * R + r;
        gnon.push_back(k < rest.size() ? rest[k] : -1);
      }
    // matrix-core stencil: one block per (group, site block), the group's lane tiles inside
    for (int e = e0; e < e1; ++e)
      for (int b = 0; b < ops[o].nblk; ++b) ilh.push_back(make_int2(e, b));
    for (int b = 0; b < ops[o].nblk; ++b)
      for (int gi = 0; gi < ng; ++gi) hnon.push_back(make_int2(g0 + gi, b));
  }
  xcd_order(hnon, ctx->xcd_order);
  // matrix-core blocks: in brick order (XCD k takes every eighth brick), or in XCD slabs (XCD k
  // takes the k-th eighth of the bricks, so that bricks adjacent in every direction run on the
  // same XCD at about the same time and share their faces through its L2); a tuned choice
  xcd_order(ilh, mfma_slab != 0);
  A2A_TRY(grow(ctx, (void**)&d_ilgroups, &cap_ilg, sizeof(ILGroupDev) * std::max<size_t>(1, ilg.size())));
  A2A_TRY(grow(ctx, (void**)&d_il_hop_tiles, &cap_ilh, sizeof(int2) * std::max<size_t>(1, ilh.size())));
  A2A_TRY(grow(ctx, (void**)&d_groups_nonil, &cap_gnonil, sizeof(int) * std::max<size_t>(1, gnon.size())));
  A2A_TRY(grow(ctx, (void**)&d_hop_nonil, &cap_hnonil, sizeof(int2) * std::max<size_t>(1, hnon.size())));
  A2A_TRY(upload(ctx, d_ilgroups, ilg.data(), sizeof(ILGroupDev) * ilg.size()));
  A2A_TRY(upload(ctx, d_il_hop_tiles, ilh.data(), sizeof(int2) * ilh.size()));
  A2A_TRY(upload(ctx, d_groups_nonil, gnon.data(), sizeof(int) * gnon.size()));
  A2A_TRY(upload(ctx, d_hop_nonil, hnon.data(), sizeof(int2) * hnon.size()));
  n_il_hop_tiles = (int)ilh.size();
  n_hop_nonil = (int)hnon.size();
  A2A_TRY(grow(ctx, (void**)&d_vec_nonil, &cap_nonil, sizeof(int2) * std::max<size_t>(1, nonil.size())));
  A2A_TRY(grow(ctx, (void**)&d_il_slots, &cap_ils, sizeof(int) * std::max<size_t>(1, ils.size())));
  A2A_TRY(grow(ctx, (void**)&d_il_tiles, &cap_ilt, sizeof(int2) * std::max<size_t>(1, ilt.size())));
  A2A_TRY(upload(ctx, d_vec_nonil, nonil.data(), sizeof(int2) * nonil.size()));
  A2A_TRY(upload(ctx, d_il_slots, ils.data(), sizeof(int) * ils.size()));
  A2A_TRY(upload(ctx, d_il_tiles, ilt.data(), sizeof(int2) * ilt.size()));
  n_vec_nonil = (int)nonil.size();
  n_il_tiles = (int)ilt.size();
  A2A_TRY(grow(ctx, (void**)&d_groups, &cap_groups, sizeof(int) * std::max<size_t>(1, groups.size())));
  A2A_TRY(grow(ctx, (void**)&d_hop_tiles, &cap_hop, sizeof(int2) * std::max<size_t>(1, htiles.size())));
  A2A_TRY(grow(ctx, (void**)&d_vec_tiles, &cap_vec, sizeof(int2) * std::max<size_t>(1, vtiles.size())));
  A2A_TRY(upload(ctx, d_groups, groups.data(), sizeof(int) * groups.size()));
  A2A_TRY(upload(ctx, d_hop_tiles, htiles.data(), sizeof(int2) * htiles.size()));
  A2A_TRY(upload(ctx, d_vec_tiles, vtiles.data(), sizeof(int2) * vtiles.size()));
  n_hop_tiles = (int)htiles.size();
  n_vec_tiles = (int)vtiles.size();
  dirty = false;
  return A2A_OK;
}

// groups of one slot each (R_sub = 1) or R for a subset of live slots
int Solver::upload_subset(const std::vector<int>& idx, int R_sub) {
  if (!dirty && sub_gen == gen && sub_R == R_sub && sub_idx == idx) return A2A_OK;  // already on the device
  // the lists are rebuilt at every residual check: the solver keeps their buffers
  std::vector<int>& groups = sc_groups;
  std::vector<int2>& htiles = sc_h;
  std::vector<int2>& vtiles = sc_v;
  std::vector<int2>& nonil = sc_n;
  std::vector<int2>& ilt = sc_i;
  std::vector<int>& ils = sc_ils;
  groups.clear();
  htiles.clear();
  vtiles.clear();
  nonil.clear();
  ilt.clear();
  ils.clear();
  for (int o = 0; o < (int)ops.size(); ++o) {
    std::vector<int> mine;
    for (int i : idx)
      if (live[i]->op == o) mine.push_back(i);
    if (mine.empty()) continue;
    const int g0 = (int)(groups.size() / R_sub);
    const int ng = (int)((mine.size() + R_sub - 1) / R_sub);
    for (int gi = 0; gi < ng; ++gi)
      for (int r = 0; r < R_sub; ++r) {
        size_t k = (size_t)gi * R_sub + r;
        groups.push_back(k < mine.size() ? mine[k] : -1);
      }
    htiles.reserve(htiles.size() + (size_t)ops[o].nblk * ng);
    for (int b = 0; b < ops[o].nblk; ++b)
      for (int gi = 0; gi < ng; ++gi) htiles.push_back(make_int2(g0 + gi, b));
  }
  xcd_order(htiles, xcd_sub >= 0 ? xcd_sub != 0 : ctx->xcd_order != 0);
  vec_lists(live, ops, idx, ctx->xcd_order, vtiles, nonil, ils, ilt);
  // one buffer holds [hop tiles | vec tiles | non-interleaved vec tiles | interleaved tiles]
  A2A_TRY(grow(ctx, (void**)&d_sub_groups, &cap_subg, sizeof(int) * std::max<size_t>(1, groups.size())));
  std::vector<int2>& all = sc_all;
  all.clear();
  all.reserve(htiles.size() + vtiles.size() + nonil.size() + ilt.size());
  all.insert(all.end(), htiles.begin(), htiles.end());
  all.insert(all.end(), vtiles.begin(), vtiles.end());
  all.insert(all.end(), nonil.begin(), nonil.end());
  all.insert(all.end(), ilt.begin(), ilt.end());
  A2A_TRY(grow(ctx, (void**)&d_sub_tiles, &cap_subt, sizeof(int2) * std::max<size_t>(1, all.size())));
  A2A_TRY(grow(ctx, (void**)&d_sub_list, &cap_subl, sizeof(int) * std::max<size_t>(1, idx.size())));
  A2A_TRY(grow(ctx, (void**)&d_sub_il_slots, &cap_subils, sizeof(int) * std::max<size_t>(1, ils.size())));
  A2A_TRY(upload(ctx, d_sub_groups, groups.data(), sizeof(int) * groups.size()));
  A2A_TRY(upload(ctx, d_sub_tiles, all.data(), sizeof(int2) * all.size()));
  A2A_TRY(upload(ctx, d_sub_list, idx.data(), sizeof(int) * idx.size()));
  A2A_TRY(upload(ctx, d_sub_il_slots, ils.data(), sizeof(int) * ils.size()));
  sub_nh = (int)htiles.size();
  sub_nv = (int)vtiles.size();
  sub_nn = (int)nonil.size();
  sub_ni = (int)ilt.size();
  sub_n = (int)idx.size();
  sub_idx = idx;
  sub_R = R_sub;
  sub_gen = gen;
  return A2A_OK;
}

int Solver::upload_subset_vec(const std::vector<int>& idx) {
  if (!dirty && sub_gen == gen && sub_R > 0 && sub_idx == idx) return A2A_OK;
  return upload_subset(idx, 1);
}

int Solver::finalize_red(bool sub, int kind) {
  launch_finalize(kind, d_ops, d_slots, sub ? d_sub_list : nullptr, sub ? sub_n : (int)live.size(), ctx->redbuf(),
                  ctx->stream);
  A2A_HIP(ctx, hipGetLastError());
  return A2A_OK;
}

int Solver::hop(bool sub, int n_tiles, int Rk, int psel, int kprec, int out_par, int vin, int vout, int vaux1,
                int vaux2, int vrhat, double ca, double cb, double gsign, int gpow, int inv, int red,
                const char* cls, int fin, int lo_mask) {
  HopArgs a{};
  a.ops = d_ops;
  a.slots = d_slots;
  a.groups = sub ? d_sub_groups : d_groups;
  a.tiles = sub ? d_sub_tiles : d_hop_tiles;
  a.out_par = out_par;
  a.psel = psel;
  a.vin = vin;
  a.vout = vout;
  a.vaux1 = vaux1;
  a.vaux2 = vaux2;
  a.vrhat = vrhat;
  a.ca = ca;
  a.cb = cb;
  a.gsign = gsign;
  a.gpow = gpow;
  a.inv = inv;
  a.red = red;
  long blocks = 0;  // site blocks of all operators: more tiles means several groups per block
  for (const OpEntry& e : ops) blocks += e.nblk;
  a.brick = n_tiles > blocks;
  a.lo_mask = lo_mask;
  a.lo_prec = prec;
  if (psel == 1 && kprec == 0 && by64 > 0) {  // FP64 stencils of setup, reliable updates, reconstruction
    a.by = by64;
    a.bz = bz64;
    a.bt = bt64;
  }
  a.rb = ctx->redbuf();
  const int c = (cls && cls[0] == '1') ? 0 : 1;
  hipEvent_t ev = nullptr;
  if (cls) A2A_TRY(ctx->timing_begin(c, &ev));
  const bool clov = (vaux2 >= 0 && cb != 0.0);
  if (!sub && psel == 0 && kprec == prec && ctx->mfma && il_mfma && n_il_hop_tiles > 0 &&
      hop_mfma_supports(kprec, inv, clov, red, vaux1 >= 0)) {
    // interleaved groups on the matrix cores, the other slots with the per-thread stencil
    HopMArgs m{};
    m.ops = d_ops;
    m.slots = d_slots;
    m.groups = d_ilgroups;
    m.tiles = d_il_hop_tiles;
    m.out_par = out_par;
    m.vin = vin;
    m.vout = vout;
    m.vaux1 = vaux1;
    m.vaux2 = vaux2;
    m.vrhat = vrhat;
    m.ca = ca;
    m.cb = cb;
    m.gsign = gsign;
    m.gpow = gpow;
    m.red = red;
    m.nt3 = il_nt3 ? 1 : 0;
    m.rb = ctx->redbuf();
    launch_hop_mfma(kprec, m, n_il_hop_tiles, inv, clov, ctx->stream);
    a.groups = d_groups_nonil;
    a.tiles = d_hop_nonil;
    a.brick = n_hop_nonil > blocks;
    launch_hop(kprec, Rk, a, n_hop_nonil, ctx->stream);
  } else {
    launch_hop(kprec, Rk, a, n_tiles, ctx->stream);
  }
  A2A_HIP(ctx, hipGetLastError());
  if (cls && ctx->timing) {
    // compulsory bytes: links and clover once per site, every spinor stream once per RHS
    const double sz = kprec == 0 ? 8.0 : kprec == 1 ? 4.0 : 2.0;
    const bool epi = inv || (vaux2 >= 0 && cb != 0.0);
    const int nvec = 2 + (vaux1 >= 0) + (vaux2 >= 0) + (red == RED_ALPHA && vrhat >= 0);
    double bytes = 0;
    for (int o = 0; o < (int)ops.size(); ++o) {
      int n = 0;
      for (Slot* s : live) n += (s->op == o);
      if (!n) continue;
      bytes += (double)ops[o].dev.g.hv * (8 * 18 * sz + (epi ? 72 * sz : 0.0) + (double)n * nvec * 24 * sz);
    }
    A2A_TRY(ctx->timing_end(c, ev, bytes));
  } else if (cls) {
    A2A_TRY(ctx->timing_end(c, ev, 0.0));
  }
  if (red != RED_NONE) A2A_TRY(finalize_red(sub, fin >= 0 ? fin : red));
  return A2A_OK;
}

int Solver::vec(bool sub, int n_tiles, int kind, int par, int use_inv, int vin, int vout) {
  VecArgs a{};
  a.ops = d_ops;
  a.slots = d_slots;
  a.tiles = sub ? d_sub_tiles + sub_nh : d_vec_tiles;
  a.kind = kind;
  a.par = par;
  a.use_inv = use_inv;
  a.vin = vin;
  a.vout = vout;
  a.rb = ctx->redbuf();
  const bool timed = !sub && (kind == VK_BICG_S || kind == VK_BICG_XR || kind == VK_BICG_P || kind == VK_CG_XR ||
                              kind == VK_CG_P);
  hipEvent_t ev = nullptr;
  const int tcls = (kind == VK_BICG_XR || kind == VK_CG_XR) ? 2 : (kind == VK_BICG_P || kind == VK_CG_P) ? 3 : 4;
  if (timed) A2A_TRY(ctx->timing_begin(tcls, &ev));
  const int n_il = sub ? sub_ni : n_il_tiles;
  if (vec_kind_il(kind) && n_il > 0) {  // interleaved slots with the lane mapping, the rest per slot
    VecArgs b = a;
    b.tiles = sub ? d_sub_tiles + sub_nh + sub_nv + sub_nn : d_il_tiles;
    b.ilslots = sub ? d_sub_il_slots : d_il_slots;
    launch_vec_il(prec, b, n_il, ctx->stream);
    a.tiles = sub ? d_sub_tiles + sub_nh + sub_nv : d_vec_nonil;
    launch_vec(prec, a, sub ? sub_nn : n_vec_nonil, ctx->stream);
  } else {
    launch_vec(prec, a, n_tiles, ctx->stream);
  }
  A2A_HIP(ctx, hipGetLastError());
  if (timed) {
    // compulsory bytes per site and RHS: s = r - alpha v reads 2 and writes 1 inner vector;
    // p = r + beta (p - omega v) reads 3, writes 1; the x / r update reads p, s, t, rhat and x
    // and writes r and x; CGNR: x += alpha p, r -= alpha gamma5 q
    // reads p, r, q and x and writes r and x; p = gamma5 u + beta p reads 2 and writes 1
    const double sz = prec == 0 ? 8.0 : prec == 1 ? 4.0 : 2.0;
    const double szx = sz;  // x is stored like the other inner vectors
    const double per = kind == VK_BICG_S   ? 3 * sz
                       : kind == VK_BICG_P ? 4 * sz
                       : kind == VK_CG_P   ? 3 * sz
                       : kind == VK_CG_XR  ? 4 * sz + 2 * szx
                                           : 5 * sz + 2 * szx;
    double bytes = 0;
    for (Slot* s : live) bytes += (double)ops[s->op].dev.g.hv * 24 * per;
    A2A_TRY(ctx->timing_end(tcls, ev, bytes));
  }
  const int red = kind == VK_BICG_XR       ? RED_RHO
                  : kind == VK_RU_RESCALE  ? RED_RU
                  : kind == VK_INIT        ? RED_INIT
                  : kind == VK_CG_XR       ? RED_CG_R
                  : kind == VK_CG_INIT     ? RED_CG_INIT
                  : kind == VK_CG_RESCALE  ? RED_CG_RU
                                           : RED_NONE;
  if (red != RED_NONE) A2A_TRY(finalize_red(sub, red));
  return A2A_OK;
}

int Solver::layout_in(bool sub, int n_tiles, int which_in, int psel, int kprec, int ve, int vo, int g5, int red) {
  LayoutArgs a{};
  a.ops = d_ops;
  a.slots = d_slots;
  a.tiles = sub ? d_sub_tiles + sub_nh : d_vec_tiles;
  a.which_in = which_in;
  a.psel = psel;
  a.v_even = ve;
  a.v_odd = vo;
  a.gamma5 = g5;
  a.red = red;
  a.rb = ctx->redbuf();
  launch_layout_in(kprec, a, n_tiles, ctx->stream);
  A2A_HIP(ctx, hipGetLastError());
  if (red != RED_NONE) A2A_TRY(finalize_red(sub, red));
  return A2A_OK;
}

int Solver::layout_out(bool sub, int n_tiles, int psel, int kprec, int ve, int vo, int g5) {
  LayoutArgs a{};
  a.ops = d_ops;
  a.slots = d_slots;
  a.tiles = sub ? d_sub_tiles + sub_nh : d_vec_tiles;
  a.psel = psel;
  a.v_even = ve;
  a.v_odd = vo;
  a.gamma5 = g5;
  a.red = RED_NONE;
  a.rb = ctx->redbuf();
  launch_layout_out(kprec, a, n_tiles, ctx->stream);
  A2A_HIP(ctx, hipGetLastError());
  return A2A_OK;
}

// One Krylov step for every live slot, up to and including the x / r update.
int Solver::iteration() {
  const int H = n_hop_tiles, Vn = n_vec_tiles;
  if (method == SOLVER_CGNR) {
    // q = M p, alpha = gamma / |q|^2; x += alpha p, r' -= alpha gamma5 q
    A2A_TRY(hop(false, H, R, 0, prec, 0, VL_P, VL_TE, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, "1"));
    A2A_TRY(hop(false, H, R, 0, prec, 1, VL_TE, VL_V, -1, VL_P, -1, 0, 1.0, -1.0, 2, 0, RED_OMEGA, "2",
                RED_CG_ALPHA));
    A2A_TRY(vec(false, Vn, VK_CG_XR));
    for (Slot* s : live) s->iters++;
    return A2A_OK;
  }
  // v = M p (asymmetric: A_oo p - kappa^2 H_oe te; symmetric: p - kappa^2 A_oo^{-1} H_oe te), te =
  // A_ee^{-1} H_eo p
  const int inv2 = sym() ? 2 : 0;
  A2A_TRY(hop(false, H, R, 0, prec, 0, VL_P, VL_TE, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, "1"));
  A2A_TRY(hop(false, H, R, 0, prec, 1, VL_TE, VL_V, -1, VL_P, VL_RHAT, 0, 1.0, -1.0, 2, inv2, RED_ALPHA, "2"));
  A2A_TRY(vec(false, Vn, VK_BICG_S));
  // t = M s
  A2A_TRY(hop(false, H, R, 0, prec, 0, VL_S, VL_TE, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, "1"));
  A2A_TRY(hop(false, H, R, 0, prec, 1, VL_TE, VL_T, -1, VL_S, -1, 0, 1.0, -1.0, 2, inv2, RED_OMEGA, "2"));
  A2A_TRY(vec(false, Vn, VK_BICG_XR));
  for (Slot* s : live) s->iters++;
  return A2A_OK;
}

// CGNR search direction: u = M r' (r' = gamma5 r, so gamma5 u = M^dag r), beta = |u|^2 /
// gamma, p = gamma5 u + beta p.  Runs before every CGNR step, so that a fresh start
// (gamma = 0) and a reliable update (r' replaced, p rescaled) need nothing else.
int Solver::cg_direction() {
  const int H = n_hop_tiles, Vn = n_vec_tiles;
  A2A_TRY(hop(false, H, R, 0, prec, 0, VL_R, VL_TE, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, "1"));
  A2A_TRY(hop(false, H, R, 0, prec, 1, VL_TE, VL_S, -1, VL_R, -1, 0, 1.0, -1.0, 2, 0, RED_OMEGA, "2",
              RED_CG_BETA));
  return vec(false, Vn, VK_CG_P);
}

// FP64: x64 is current; r64 = b - M x64 and |r64|^2 for a subset (uploaded by the caller).
int Solver::true_residual(const std::vector<int>& idx) {
  (void)idx;
  A2A_TRY(hop(true, sub_nh, R64, 1, 0, 0, VH_X, VH_TE, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, nullptr));
  A2A_TRY(hop(true, sub_nh, R64, 1, 0, 1, VH_TE, VH_R, VH_BHAT, VH_X, -1, 1.0, -1.0, 1.0, 2, 0, RED_R64, nullptr));
  return A2A_OK;
}

bool Solver::sym() const { return method == SOLVER_BICGSTAB && ctx->schur_sym; }

// FP64, correction form: r64 -= M (sigma x_lo) for a subset whose inner iterate x_lo holds the
// correction since the last FP64 residual (x64 not yet updated): te = A_ee^{-1} H_eo (sigma
// x_lo), r64 = r64 + kappa^2 H_oe te - A_oo (sigma x_lo), |r64|^2.  The stencils read the
// stored low-precision correction (its values are exact in FP64) and compute in FP64, so r64
// stays the FP64 residual of x64 + sigma x_lo up to FP64 rounding, at a quarter of the bytes of
// the hopping input.  The caller folds x_lo into x64 afterwards.
int Solver::true_residual_corr(const std::vector<int>& idx) {
  (void)idx;
  A2A_TRY(hop(true, sub_nh, R64, 1, 0, 0, VL_X, VH_TE, -1, -1, -1, 0, 0, 1.0, 0, 1, RED_NONE, nullptr, -1, 1));
  A2A_TRY(hop(true, sub_nh, R64, 1, 0, 1, VH_TE, VH_R, VH_R, VL_X, -1, 1.0, -1.0, 1.0, 2, 0, RED_R64, nullptr, -1,
              2));
  return A2A_OK;
}

// Prepare new slots: eta -> even-odd FP64, b = eta_o + kappa H_oe A_ee^{-1} eta_e, x64 = x0 or 0,
// r64 = b - M x64, inner state.  Marks zero / non-finite sources.
int Solver::setup(const std::vector<int>& idx) {
  if (idx.empty()) return A2A_OK;
  if (ctx->fail_setup_enomem > 0) {
    ctx->fail_setup_enomem--;
    return ctx->fail(A2A_ENOMEM, "source preparation: injected out-of-memory (test hook)");
  }
  if (ctx->fail_setup_device > 0) {
    ctx->fail_setup_device--;
    return ctx->fail(A2A_EDEVICE, "source preparation: injected device error (test hook)");
  }
  A2A_TRY(rebuild());
  std::vector<int> with_x0;
  for (int i : idx)
    if (live[i]->x0) with_x0.push_back(i);
  A2A_TRY(upload_subset(idx, R64));
  int nh = sub_nh, nv = sub_nv;
  A2A_TRY(layout_in(true, nv, 0, 1, 0, VH_ETA_E, VH_ETA_O, 0, RED_ETA));
  A2A_TRY(vec(true, nv, VK_CLOVER, 0, 1, VH_ETA_E, VH_TE));
  // without initial guesses r = b - M 0 = b: the b-hat stencil reduces |b|^2 and the inner
  // state starts from b, so no FP64 Schur operator is applied here
  const bool zero_x0 = with_x0.empty();
  A2A_TRY(hop(true, nh, R64, 1, 0, 1, VH_TE, VH_BHAT, VH_ETA_O, -1, -1, 1.0, 0, 1.0, 1, 0,
              zero_x0 ? RED_R64 : RED_NONE, nullptr));
  A2A_TRY(vec(true, nv, VK_ZERO_HI, 0, 0, -1, VH_X));
  if (zero_x0) A2A_TRY(vec(true, nv, VK_COPY_HI, 0, 0, VH_BHAT, VH_R));  // r64 = b - M 0, kept current
  if (!zero_x0) {
    A2A_TRY(upload_subset(with_x0, 1));
    A2A_TRY(layout_in(true, sub_nv, 1, 1, 0, VH_TE, VH_X, 0, RED_NONE));
    A2A_TRY(upload_subset(idx, R64));
    A2A_TRY(true_residual(idx));
  }
  // the symmetric Schur form iterates on A_oo^-1 r64 (applied by the kernel)
  A2A_TRY(vec(true, nv, init_kind(), 0, sym() ? 1 : 0, zero_x0 ? VH_BHAT : VH_R));
  A2A_TRY(ctx->read_scal());
  for (int i : idx) {
    Slot* s = live[i];
    const double* sc = ctx->scal_host + (size_t)s->sid * NSCAL;
    const double e2 = sc[SC_ETAN2], r2 = sc[SC_R64N2];
    if (!std::isfinite(e2) || !std::isfinite(r2)) {
      s->state = SS_FAIL;
      s->err = A2A_ENAN;
      continue;
    }
    s->eta_norm = std::sqrt(e2);
    // the Schur residual b - M x_o equals the full-system residual once x_e is reconstructed
    // (the even part vanishes up to rounding); the fraction leaves room for that rounding and
    // for the drift of the iterated estimate, and the reconstruction's residual decides
    s->target = ctx->target_frac * s->tol * s->eta_norm;
    s->last_r64 = std::sqrt(r2);
    s->state = SS_RUN;
  }
  return A2A_OK;
}

// Reconstruct x_e, compute the FP64 residual of the full system, write the canonical
// solution.  Fills info; returns through slot state.
int Solver::finalize(const std::vector<int>& idx) {
  if (idx.empty()) return A2A_OK;
  A2A_TRY(upload_subset(idx, R64));
  const int nh = sub_nh, nv = sub_nv;
  // x_e = A_ee^{-1} y with y = eta_e + kappa H_eo x_o -> VH_TE, and in the same launch the even
  // residual r_e = eta_e - A_ee x_e + kappa H_eo x_o = y - A_ee x_e (x_e as stored), |r_e|^2
  A2A_TRY(hop(true, nh, R64, 1, 0, 0, VH_X, VH_TE, VH_ETA_E, -1, -1, 1.0, 0, 1.0, 1, 1, RED_RES_E, nullptr));
  // r_o = eta_o - A_oo x_o + kappa H_oe x_e
  A2A_TRY(hop(true, nh, R64, 1, 0, 1, VH_TE, VH_R, VH_ETA_O, VH_X, -1, 1.0, -1.0, 1.0, 1, 0, RED_RES_O, nullptr));
  A2A_TRY(layout_out(true, nv, 1, 0, VH_TE, VH_X, 0));
  A2A_TRY(ctx->read_scal());
  const double t = now_seconds();
  for (int i : idx) {
    Slot* s = live[i];
    const double* sc = ctx->scal_host + (size_t)s->sid * NSCAL;
    const double res = std::sqrt(sc[SC_RES_E] + sc[SC_RES_O]);
    s->info.true_rel_residual = s->eta_norm > 0 ? res / s->eta_norm : 0.0;
    s->info.iters = s->iters;
    s->info.reliable_updates = s->rus;
    s->info.restarts = s->restarts;
    s->info.solver = method;
    s->info.converged = (s->info.true_rel_residual <= s->tol) ? 1 : 0;
    s->info.seconds = t - s->t_submit;
  }
  return A2A_OK;
}

// Slots whose iterated residual estimate is below the target: fold the inner correction into
// x64 and reconstruct, skipping the FP64 Schur residual that a reliable update would compute
// (the reconstruction's residual of the full system decides convergence).  A slot the full
// residual does not accept gets its FP64 Schur residual and continues with a tenfold tighter
// target, like a slot whose reconstruction failed after a reliable update.
int Solver::finish(const std::vector<int>& fin) {
  A2A_TRY(upload_subset_vec(fin));
  A2A_TRY(vec(true, sub_nv, VK_RU_ACCUM));
  A2A_TRY(finalize(fin));
  std::vector<int> again;
  for (int i : fin) {
    Slot* s = live[i];
    s->rus++;
    if (s->info.converged) {
      s->state = SS_DONE;
    } else if (s->iters >= s->max_iter) {
      s->state = SS_FAIL;
      s->err = A2A_ENOTCONV;
    } else {
      again.push_back(i);
    }
  }
  if (again.empty()) return A2A_OK;
  A2A_TRY(upload_subset(again, R64));
  A2A_TRY(true_residual(again));
  A2A_TRY(ctx->read_scal());
  for (int i : again) {
    Slot* s = live[i];
    s->last_r64 = std::sqrt(ctx->scal_host[(size_t)s->sid * NSCAL + SC_R64N2]);
    s->target *= 0.1;
  }
  A2A_TRY(upload_subset_vec(again));
  // the symmetric Schur form iterates on A_oo^-1 r64 (applied by the kernel)
  return vec(true, sub_nv, init_kind(), 0, sym() ? 1 : 0, VH_R);
}

// Residual checks, reliable updates, restarts, convergence and retirement.
int Solver::check() {
  A2A_TRY(ctx->read_scal());
  std::vector<int> ru, restart, fin;
  // CGNR with FP16 storage: its iterate accumulates about three times as many FP16-rounded
  // updates between reliable updates as BiCGStab's, so it is flushed at 0.1
  const double delta = prec == 0                                 ? ctx->delta_64
                       : prec == 3                                 ? ctx->delta_bf16
                       : (prec == 2 && method == SOLVER_CGNR)      ? ctx->delta_cgnr
                                                                   : ctx->delta_lo;
  for (int i = 0; i < (int)live.size(); ++i) {
    Slot* s = live[i];
    if (s->state != SS_RUN) continue;
    const double* sc = ctx->scal_host + (size_t)s->sid * NSCAL;
    const double est = std::sqrt(sc[SC_RNORM2]) * sc[SC_SIGMA];
    if (sc[SC_FLAGS] != 0.0 || !std::isfinite(est)) {
      restart.push_back(i);
    } else if (est <= s->target && s->rus > 0 && !ctx->force_breakdown) {
      fin.push_back(i);  // converged by the estimate: the reconstruction checks the full residual
    } else if (est <= s->target || est <= delta * s->last_r64 || s->iters >= s->max_iter) {
      ru.push_back(i);
    }
  }
  if (!fin.empty()) A2A_TRY(finish(fin));
  if (ru.empty() && restart.empty()) return A2A_OK;
  std::vector<int> all(ru);
  all.insert(all.end(), restart.begin(), restart.end());
  if (!restart.empty()) {  // a broken-down inner iterate may hold inf/NaN: drop it, keep x64
    A2A_TRY(upload_subset_vec(restart));
    A2A_TRY(vec(true, sub_nv, VK_ZERO_X));
  }
  // reliable updates in correction form (mixed precision): r64 -= M (sigma x_lo), then x64 +=
  // sigma x_lo; restarts (and the FP64-only mode) recompute r64 = b - M x64 from x64
  const bool corr = prec != 0 && ctx->ru_correction && hop_lo_supports(R64, 1, prec, 1, false) &&
                    hop_lo_supports(R64, 2, prec, 0, true);
  if (corr) {
    if (!restart.empty()) {
      A2A_TRY(upload_subset(restart, R64));
      A2A_TRY(true_residual(restart));
    }
    if (!ru.empty()) {
      A2A_TRY(upload_subset(ru, R64));
      A2A_TRY(true_residual_corr(ru));
      A2A_TRY(upload_subset_vec(ru));
      A2A_TRY(vec(true, sub_nv, VK_RU_ACCUM));
    }
  } else {
    if (!ru.empty()) {
      A2A_TRY(upload_subset_vec(ru));
      A2A_TRY(vec(true, sub_nv, VK_RU_ACCUM));
    }
    A2A_TRY(upload_subset(all, R64));
    A2A_TRY(true_residual(all));
  }
  A2A_TRY(ctx->read_scal());
  std::vector<int> done, rescale, reinit;
  for (int i : all) {
    Slot* s = live[i];
    s->rus++;
    const double* sc = ctx->scal_host + (size_t)s->sid * NSCAL;
    const double r = std::sqrt(sc[SC_R64N2]);
    const bool was_restart = std::find(restart.begin(), restart.end(), i) != restart.end();
    if (ctx->debug)
      std::fprintf(stderr, "[a2a] slot %d iter %d: est %.3e true %.3e last %.3e target %.3e flags %g%s\n", s->sid,
                   s->iters, std::sqrt(sc[SC_RNORM2]) * sc[SC_SIGMA], r, s->last_r64, s->target, sc[SC_FLAGS],
                   was_restart ? " (breakdown)" : "");
    if (!std::isfinite(r)) {
      s->state = SS_FAIL;
      s->err = A2A_EBREAKDOWN;
      done.push_back(i);
      continue;
    }
    if (r <= s->target || s->iters >= s->max_iter) {
      done.push_back(i);
      s->last_r64 = r;
      continue;
    }
    if (ctx->force_breakdown && method == SOLVER_BICGSTAB) {  // test hook: a breakdown at the first update
      s->state = SS_FAIL;
      s->err = A2A_EBREAKDOWN;
      s->last_r64 = r;
      done.push_back(i);
      continue;
    }
    if (was_restart || r > 0.9 * s->last_r64) {
      s->stagn++;
      s->restarts++;
      if (s->restarts > 50) {
        s->state = SS_FAIL;
        s->err = A2A_EBREAKDOWN;
        done.push_back(i);
        continue;
      }
      reinit.push_back(i);
    } else {
      rescale.push_back(i);
    }
    s->last_r64 = r;
  }
  if (!rescale.empty()) {
    A2A_TRY(upload_subset_vec(rescale));
    // the symmetric Schur form iterates on A_oo^-1 r64 (applied by the kernel)
    A2A_TRY(vec(true, sub_nv, method == SOLVER_CGNR ? VK_CG_RESCALE : VK_RU_RESCALE, 0, sym() ? 1 : 0, VH_R));
  }
  if (!reinit.empty()) {
    A2A_TRY(upload_subset_vec(reinit));
    // the symmetric Schur form iterates on A_oo^-1 r64 (applied by the kernel)
    A2A_TRY(vec(true, sub_nv, init_kind(), 0, sym() ? 1 : 0, VH_R));
  }
  if (!done.empty()) {
    A2A_TRY(finalize(done));
    std::vector<int> again;
    for (int i : done) {
      Slot* s = live[i];
      if (s->state == SS_FAIL) continue;
      if (s->info.converged) {
        s->state = SS_DONE;
      } else if (s->iters >= s->max_iter) {
        s->state = SS_FAIL;
        s->err = A2A_ENOTCONV;
      } else {  // reconstruction rounding: tighten and continue from the current x
        s->target *= 0.1;
        again.push_back(i);
      }
    }
    if (!again.empty()) {
      A2A_TRY(upload_subset_vec(again));
      // the symmetric Schur form iterates on A_oo^-1 r64 (applied by the kernel)
      A2A_TRY(vec(true, sub_nv, init_kind(), 0, sym() ? 1 : 0, VH_R));
    }
  }
  return A2A_OK;
}

// Drop finished slots from the device tables.
int Solver::retire() {
  size_t before = live.size();
  live.erase(std::remove_if(live.begin(), live.end(),
                            [](Slot* s) { return s->state == SS_DONE || s->state == SS_FAIL; }),
             live.end());
  if (live.size() != before) dirty = true;
  return A2A_OK;
}

// Up to `iters` steps of every live slot, with residual checks every check_every steps and
// after the last; stops early when no slot is left.
// Residual checks every check_every iterations; in the tail of a batch (at most a quarter of
// the most slots this solver has run at once still live) after every iteration, so that the
// last sources, which keep their whole lane groups busy, stop as soon as they converge.
int Solver::run_steps(int iters) {
  A2A_TRY(retire());
  for (int k = 1; k <= iters && !live.empty(); ++k) {
    A2A_TRY(rebuild());
    peak_live = std::max(peak_live, live.size());
    if (method == SOLVER_CGNR) A2A_TRY(cg_direction());
    A2A_TRY(iteration());
    const bool tail = ctx->tail_checks && 4 * live.size() <= peak_live;
    if (k % ctx->check_every == 0 || k == iters || tail) {
      A2A_TRY(check());
      A2A_TRY(retire());
      A2A_TRY(rebuild());
      if (live.empty()) break;
    }
    if (method == SOLVER_BICGSTAB) A2A_TRY(vec(false, n_vec_tiles, VK_BICG_P));
  }
  return A2A_OK;
}

// Iterate every live slot until all are done (or fail).
int Solver::run_until_done(int max_outer_iters) { return run_steps(max_outer_iters); }

}  // namespace a2a
